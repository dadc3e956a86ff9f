/*
 * ldo_ff.c -- CPU FP64 oracle for the learned far field (test infrastructure
 * only; see ldo.h for the rules it follows).
 *
 * The pair sum is split at a near cutoff r_c: pairs with r < r_c are summed
 * exactly (LJ + Coulomb); the Coulomb sum over r >= r_c is the "far field".
 * The far field is modelled as
 *     E_far(i) ~ E_coarse(cell of i) + E_mlp(features of i)
 * where E_coarse is the field at the centre of i's grid cell from the
 * monopole and dipole moments of every grid cell outside the B x B x B block
 * around that cell, and the MLP sees the normalised moments of the B^3 block
 * plus i's offset inside its cell.  Fields are in units of sqrt(kT l_B) per
 * unit length squared, so the force is q_hat_i E with q_hat = q sqrt(kT l_B).
 *
 * Everything here is FP64.  The MLP forward can emulate the GPU's BF16
 * operands: inputs, weights and hidden activations are rounded to BF16
 * (round to nearest even) before each matrix product; products and sums stay
 * FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ldo.h"

/* BF16 round-to-nearest-even of an FP64 value (via its FP32 rounding, as a
 * device converting an FP32 register would see it). */
double ldo_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (double)f;   /* inf / nan */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static void cell_of(const double x[3], int G, double L, int c[3]) {
    const double h = 2.0 * L / G;
    for (int k = 0; k < 3; ++k) {
        int v = (int)floor((x[k] + L) / h);
        if (v < 0) v = 0;
        if (v > G - 1) v = G - 1;
        c[k] = v;
    }
}

static double centre(int ci, int G, double L) { return -L + (ci + 0.5) * (2.0 * L / G); }

/* Moments of the G^3 grid over [-L, L]^3: per cell Q = sum q_hat, P = sum
 * q_hat (x - centre).  out is [G^3 * 4], cell index (iz * G + iy) * G + ix. */
void ldo_ff_moments(int64_t n, const double* x, const double* qhat, int G, double L,
                    double* out) {
    memset(out, 0, sizeof(double) * 4 * (size_t)G * G * G);
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        cell_of(&x[3 * i], G, L, c);
        const size_t k = ((size_t)c[2] * G + c[1]) * G + c[0];
        out[4 * k] += qhat[i];
        out[4 * k + 1] += qhat[i] * (x[3 * i] - centre(c[0], G, L));
        out[4 * k + 2] += qhat[i] * (x[3 * i + 1] - centre(c[1], G, L));
        out[4 * k + 3] += qhat[i] * (x[3 * i + 2] - centre(c[2], G, L));
    }
}

/* Field at every cell centre from the monopole + dipole of every cell
 * outside the B^3 block (Chebyshev cell distance > B/2) around it:
 *   E = Q r / r^3 + (3 (P.r) r / r^2 - P) / r^3,  r = target - source. */
void ldo_ff_coarse(int G, double L, int B, const double* mom, double* E) {
    const int half = B / 2;
    const size_t M = (size_t)G * G * G;
#pragma omp parallel for schedule(dynamic, 16)
    for (size_t t = 0; t < M; ++t) {
        const int tx = (int)(t % G), ty = (int)((t / G) % G), tz = (int)(t / ((size_t)G * G));
        double ex = 0.0, ey = 0.0, ez = 0.0;
        for (size_t s = 0; s < M; ++s) {
            const int sx = (int)(s % G), sy = (int)((s / G) % G), sz = (int)(s / ((size_t)G * G));
            if (abs(sx - tx) <= half && abs(sy - ty) <= half && abs(sz - tz) <= half) continue;
            const double Q = mom[4 * s], Px = mom[4 * s + 1], Py = mom[4 * s + 2],
                         Pz = mom[4 * s + 3];
            if (Q == 0.0 && Px == 0.0 && Py == 0.0 && Pz == 0.0) continue;
            const double rx = centre(tx, G, L) - centre(sx, G, L);
            const double ry = centre(ty, G, L) - centre(sy, G, L);
            const double rz = centre(tz, G, L) - centre(sz, G, L);
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double r = sqrt(r2);
            const double r3 = r2 * r;
            const double pr = Px * rx + Py * ry + Pz * rz;
            ex += Q * rx / r3 + (3.0 * pr * rx / r2 - Px) / r3;
            ey += Q * ry / r3 + (3.0 * pr * ry / r2 - Py) / r3;
            ez += Q * rz / r3 + (3.0 * pr * rz / r2 - Pz) / r3;
        }
        E[3 * t] = ex;
        E[3 * t + 1] = ey;
        E[3 * t + 2] = ez;
    }
}

/* Pair forces (LJ + Coulomb, as ldo_pair_forces) restricted to pairs with
 * r < r_c, and the far Coulomb field sum_{j: r >= r_c} q_hat_j r_ij / r^3
 * (without the q_hat_i factor), for the listed rows (NULL: all). */
void ldo_ff_split(int64_t n, const double* x, const int32_t* type, const double* q,
                  const ldo_params* p, double rc, const int64_t* rows, int64_t n_rows,
                  double* F_near, double* E_far) {
    if (rows == NULL) n_rows = n;
    const double s = sqrt(p->kT * p->bjerrum);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        double fx = 0, fy = 0, fz = 0, ex = 0, ey = 0, ez = 0;
        double cfx = 0, cfy = 0, cfz = 0, cex = 0, cey = 0, cez = 0;  /* Kahan terms */
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                         dz = x[3 * i + 2] - x[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rr = sqrt(r2);
            double gx = 0, gy = 0, gz = 0;
            if (rr < rc) {
                const int ti = type[i], tj = type[j];
                const double sg = 0.5 * (p->sigma[ti] + p->sigma[tj]);
                const double e = p->use_eps_matrix ? p->eps_matrix[ti * LDO_MAX_TYPES + tj]
                                                   : sqrt(p->eps[ti] * p->eps[tj]);
                if (r2 < (p->lj_cut * sg) * (p->lj_cut * sg)) {
                    const double sr2 = sg * sg / r2, sr6 = sr2 * sr2 * sr2;
                    const double g = 24.0 * e * (2.0 * sr6 * sr6 - sr6) / r2;
                    gx += g * dx; gy += g * dy; gz += g * dz;
                }
                const double k = p->kT * p->bjerrum * q[i] * q[j] / (r2 * rr);
                gx += k * dx; gy += k * dy; gz += k * dz;
                double y, t;
                y = gx - cfx; t = fx + y; cfx = (t - fx) - y; fx = t;
                y = gy - cfy; t = fy + y; cfy = (t - fy) - y; fy = t;
                y = gz - cfz; t = fz + y; cfz = (t - fz) - y; fz = t;
            } else {
                const double k = s * q[j] / (r2 * rr);
                double y, t;
                y = k * dx - cex; t = ex + y; cex = (t - ex) - y; ex = t;
                y = k * dy - cey; t = ey + y; cey = (t - ey) - y; ey = t;
                y = k * dz - cez; t = ez + y; cez = (t - ez) - y; ez = t;
            }
        }
        if (F_near) { F_near[3 * r] = fx; F_near[3 * r + 1] = fy; F_near[3 * r + 2] = fz; }
        if (E_far) { E_far[3 * r] = ex; E_far[3 * r + 1] = ey; E_far[3 * r + 2] = ez; }
    }
}

/* The split with the near region = the B^3 block of grid cells around i's
 * cell (the cell of a particle as in ldo_ff_moments).  Coulomb of pairs in
 * the block and LJ of every pair within its LJ range go to F_near; the
 * Coulomb field of the particles outside the block goes to E_far. */
void ldo_ff_split_block(int64_t n, const double* x, const int32_t* type, const double* q,
                        const ldo_params* p, int G, double L, int B, const int64_t* rows,
                        int64_t n_rows, double* F_near, double* E_far) {
    if (rows == NULL) n_rows = n;
    const double s = sqrt(p->kT * p->bjerrum);
    const int half = B / 2;
    int* cell = (int*)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) cell_of(&x[3 * j], G, L, &cell[3 * j]);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        double fx = 0, fy = 0, fz = 0, ex = 0, ey = 0, ez = 0;
        double cfx = 0, cfy = 0, cfz = 0, cex = 0, cey = 0, cez = 0;  /* Kahan terms */
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                         dz = x[3 * i + 2] - x[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rr = sqrt(r2);
            const int inblock = abs(cell[3 * j] - cell[3 * i]) <= half &&
                                abs(cell[3 * j + 1] - cell[3 * i + 1]) <= half &&
                                abs(cell[3 * j + 2] - cell[3 * i + 2]) <= half;
            const int ti = type[i], tj = type[j];
            const double sg = 0.5 * (p->sigma[ti] + p->sigma[tj]);
            double gx = 0, gy = 0, gz = 0;
            int near = 0;
            if (r2 < (p->lj_cut * sg) * (p->lj_cut * sg)) {
                const double e = p->use_eps_matrix ? p->eps_matrix[ti * LDO_MAX_TYPES + tj]
                                                   : sqrt(p->eps[ti] * p->eps[tj]);
                const double sr2 = sg * sg / r2, sr6 = sr2 * sr2 * sr2;
                const double g = 24.0 * e * (2.0 * sr6 * sr6 - sr6) / r2;
                gx += g * dx; gy += g * dy; gz += g * dz;
                near = 1;
            }
            if (inblock) {
                const double k = p->kT * p->bjerrum * q[i] * q[j] / (r2 * rr);
                gx += k * dx; gy += k * dy; gz += k * dz;
                near = 1;
            } else {
                const double k = s * q[j] / (r2 * rr);
                double y, t;
                y = k * dx - cex; t = ex + y; cex = (t - ex) - y; ex = t;
                y = k * dy - cey; t = ey + y; cey = (t - ey) - y; ey = t;
                y = k * dz - cez; t = ez + y; cez = (t - ez) - y; ez = t;
            }
            if (near) {
                double y, t;
                y = gx - cfx; t = fx + y; cfx = (t - fx) - y; fx = t;
                y = gy - cfy; t = fy + y; cfy = (t - fy) - y; fy = t;
                y = gz - cfz; t = fz + y; cfz = (t - fz) - y; fz = t;
            }
        }
        if (F_near) { F_near[3 * r] = fx; F_near[3 * r + 1] = fy; F_near[3 * r + 2] = fz; }
        if (E_far) { E_far[3 * r] = ex; E_far[3 * r + 1] = ey; E_far[3 * r + 2] = ez; }
    }
    free(cell);
}

/* Derivative tensors of g(R) = 1/|R| up to fourth order at R (full,
 * symmetric; T1[a], T2[a][b], T3[a][b][c], T4[a][b][c][d]):
 *   d_a g       = -R_a / R^3
 *   d_ab g      = (3 R_a R_b - R^2 delta_ab) / R^5
 *   d_abc g     = -15 R_a R_b R_c / R^7 + 3 (delta_ab R_c + delta_ac R_b + delta_bc R_a) / R^5
 *   d_abcd g    = 105 R_a R_b R_c R_d / R^9
 *                 - 15 (delta_ab R_c R_d + delta_ac R_b R_d + delta_ad R_b R_c
 *                       + delta_bc R_a R_d + delta_bd R_a R_c + delta_cd R_a R_b) / R^7
 *                 + 3 (delta_ab delta_cd + delta_ac delta_bd + delta_ad delta_bc) / R^5 */
static void inv_r_derivs(const double R[3], double T1[3], double T2[3][3], double T3[3][3][3],
                         double T4[3][3][3][3]) {
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double r = sqrt(r2);
    const double i3 = 1.0 / (r2 * r), i5 = i3 / r2, i7 = i5 / r2, i9 = i7 / r2;
#define D(a, b) ((a) == (b) ? 1.0 : 0.0)
    for (int a = 0; a < 3; ++a) {
        T1[a] = -R[a] * i3;
        for (int b = 0; b < 3; ++b) {
            T2[a][b] = 3.0 * R[a] * R[b] * i5 - r2 * D(a, b) * i5;
            for (int c = 0; c < 3; ++c) {
                T3[a][b][c] = -15.0 * R[a] * R[b] * R[c] * i7 +
                              3.0 * (D(a, b) * R[c] + D(a, c) * R[b] + D(b, c) * R[a]) * i5;
                for (int d = 0; d < 3; ++d)
                    T4[a][b][c][d] =
                        105.0 * R[a] * R[b] * R[c] * R[d] * i9 -
                        15.0 * (D(a, b) * R[c] * R[d] + D(a, c) * R[b] * R[d] +
                                D(a, d) * R[b] * R[c] + D(b, c) * R[a] * R[d] +
                                D(b, d) * R[a] * R[c] + D(c, d) * R[a] * R[b]) * i7 +
                        3.0 * (D(a, b) * D(c, d) + D(a, c) * D(b, d) + D(a, d) * D(b, c)) * i5;
            }
        }
    }
#undef D
}

/* Adds one source's field, gradient and Hessian at R = target - source
 * centre (see ldo_ff_local). */
static void add_source(const double R[3], double Q, const double P[3], double E[3],
                       double J[3][3], double H[3][3][3]) {
    double T1[3], T2[3][3], T3[3][3][3], T4[3][3][3][3];
    inv_r_derivs(R, T1, T2, T3, T4);
    for (int c = 0; c < 3; ++c) {
        E[c] += -Q * T1[c];
        for (int a = 0; a < 3; ++a) E[c] += P[a] * T2[a][c];
        for (int d = 0; d < 3; ++d) {
            J[c][d] += -Q * T2[c][d];
            for (int a = 0; a < 3; ++a) J[c][d] += P[a] * T3[a][c][d];
            for (int e = 0; e < 3; ++e) {
                H[c][d][e] += -Q * T3[c][d][e];
                for (int a = 0; a < 3; ++a) H[c][d][e] += P[a] * T4[a][c][d][e];
            }
        }
    }
}

static const int J_IDX[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
static const int H_IDX[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                 {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};

static void pack_local(const double E[3], double J[3][3], double H[3][3][3], double* o) {
    for (int k = 0; k < 3; ++k) o[k] = E[k];
    for (int k = 0; k < 6; ++k) o[3 + k] = J[J_IDX[k][0]][J_IDX[k][1]];
    for (int k = 0; k < 10; ++k) o[9 + k] = H[H_IDX[k][0]][H_IDX[k][1]][H_IDX[k][2]];
}

/* Local expansion at each cell centre.  A source cell with moments (Q, P)
 * about its centre c_s has the potential phi(x) = Q g(R) - P_a d_a g(R),
 * R = x - c_s (the expansion of sum q_hat / |x - x_j| to dipole order), so
 *   E_c  = -d_c phi    = -Q d_c g   + P_a d_ac g
 *   J_cd = d_d E_c     = -Q d_cd g  + P_a d_acd g
 *   H_cde = d_de E_c   = -Q d_cde g + P_a d_acde g
 * evaluated at R = c_t - c_s and summed over the cells outside the block. */
void ldo_ff_local(int G, double L, int B, const double* mom, double* out) {
    const int half = B / 2;
    const size_t M = (size_t)G * G * G;
#pragma omp parallel for schedule(dynamic, 16)
    for (size_t t = 0; t < M; ++t) {
        const int tc[3] = {(int)(t % G), (int)((t / G) % G), (int)(t / ((size_t)G * G))};
        double E[3] = {0, 0, 0}, J[3][3] = {{0}}, H[3][3][3] = {{{0}}};
        for (size_t s = 0; s < M; ++s) {
            const int sc[3] = {(int)(s % G), (int)((s / G) % G), (int)(s / ((size_t)G * G))};
            if (abs(sc[0] - tc[0]) <= half && abs(sc[1] - tc[1]) <= half &&
                abs(sc[2] - tc[2]) <= half)
                continue;
            const double Q = mom[4 * s], P[3] = {mom[4 * s + 1], mom[4 * s + 2], mom[4 * s + 3]};
            if (Q == 0.0 && P[0] == 0.0 && P[1] == 0.0 && P[2] == 0.0) continue;
            double R[3];
            for (int k = 0; k < 3; ++k) R[k] = centre(tc[k], G, L) - centre(sc[k], G, L);
            add_source(R, Q, P, E, J, H);
        }
        pack_local(E, J, H, out + 19 * t);
    }
}

/* Two-level version (G even).  Parent cells are the 2x2x2 blocks of cells
 * (a (G/2)^3 grid of side 2h); a parent's moments are its children's moments
 * moved to the parent centre, Q_p = sum Q_c, P_p = sum (P_c + Q_c (c_c - c_p))
 * -- exactly the monopole and dipole of its particles about c_p.  For target
 * cell t with parent T, a parent within Chebyshev distance D of T contributes
 * its children one by one (those outside t's B^3 block, as in
 * ldo_ff_local); every other parent contributes through its own moments.
 * Each cell outside the block is counted once (a parent farther than D >= 1
 * holds no cell of the block); D >= G/2 gives ldo_ff_local. */
void ldo_ff_local2(int G, double L, int B, int D, const double* mom, double* out) {
    const int half = B / 2;
    const int Gp = G / 2;
    const size_t M = (size_t)G * G * G, Mp = (size_t)Gp * Gp * Gp;
    double* pm = (double*)calloc(4 * Mp, sizeof(double));
    for (size_t c = 0; c < M; ++c) {
        const int cc[3] = {(int)(c % G), (int)((c / G) % G), (int)(c / ((size_t)G * G))};
        const size_t p = ((size_t)(cc[2] / 2) * Gp + cc[1] / 2) * Gp + cc[0] / 2;
        pm[4 * p] += mom[4 * c];
        for (int k = 0; k < 3; ++k)
            pm[4 * p + 1 + k] += mom[4 * c + 1 + k] +
                                 mom[4 * c] * (centre(cc[k], G, L) - centre(cc[k] / 2, Gp, L));
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (size_t t = 0; t < M; ++t) {
        const int tc[3] = {(int)(t % G), (int)((t / G) % G), (int)(t / ((size_t)G * G))};
        const int T[3] = {tc[0] / 2, tc[1] / 2, tc[2] / 2};
        double E[3] = {0, 0, 0}, J[3][3] = {{0}}, H[3][3][3] = {{{0}}};
        for (size_t p = 0; p < Mp; ++p) {
            const int pc[3] = {(int)(p % Gp), (int)((p / Gp) % Gp), (int)(p / ((size_t)Gp * Gp))};
            const int near = abs(pc[0] - T[0]) <= D && abs(pc[1] - T[1]) <= D &&
                             abs(pc[2] - T[2]) <= D;
            if (!near) {
                const double Q = pm[4 * p], P[3] = {pm[4 * p + 1], pm[4 * p + 2], pm[4 * p + 3]};
                if (Q == 0.0 && P[0] == 0.0 && P[1] == 0.0 && P[2] == 0.0) continue;
                double R[3];
                for (int k = 0; k < 3; ++k) R[k] = centre(tc[k], G, L) - centre(pc[k], Gp, L);
                add_source(R, Q, P, E, J, H);
                continue;
            }
            for (int ch = 0; ch < 8; ++ch) {
                const int sc[3] = {2 * pc[0] + (ch & 1), 2 * pc[1] + ((ch >> 1) & 1),
                                   2 * pc[2] + (ch >> 2)};
                if (abs(sc[0] - tc[0]) <= half && abs(sc[1] - tc[1]) <= half &&
                    abs(sc[2] - tc[2]) <= half)
                    continue;
                const size_t s = ((size_t)sc[2] * G + sc[1]) * G + sc[0];
                const double Q = mom[4 * s], P[3] = {mom[4 * s + 1], mom[4 * s + 2], mom[4 * s + 3]};
                if (Q == 0.0 && P[0] == 0.0 && P[1] == 0.0 && P[2] == 0.0) continue;
                double R[3];
                for (int k = 0; k < 3; ++k) R[k] = centre(tc[k], G, L) - centre(sc[k], G, L);
                add_source(R, Q, P, E, J, H);
            }
        }
        pack_local(E, J, H, out + 19 * t);
    }
    free(pm);
}

void ldo_ff_local_eval(int64_t n, const double* x, int G, double L, const double* loc,
                       double* E) {
    static const int J_OF[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        cell_of(&x[3 * i], G, L, c);
        const double* o = loc + 19 * (((size_t)c[2] * G + c[1]) * G + c[0]);
        const double d[3] = {x[3 * i] - centre(c[0], G, L), x[3 * i + 1] - centre(c[1], G, L),
                             x[3 * i + 2] - centre(c[2], G, L)};
        for (int a = 0; a < 3; ++a) {
            double v = o[a];
            for (int b = 0; b < 3; ++b) {
                /* J[a][b] is dE_a/dx_b; the packed J is symmetric */
                v += o[3 + J_OF[a][b]] * d[b];
                for (int e = 0; e < 3; ++e) {
                    /* H[a][b][e]: sort the three indices to find the packed slot */
                    int k[3] = {a, b, e}, tmp;
                    if (k[0] > k[1]) { tmp = k[0]; k[0] = k[1]; k[1] = tmp; }
                    if (k[1] > k[2]) { tmp = k[1]; k[1] = k[2]; k[2] = tmp; }
                    if (k[0] > k[1]) { tmp = k[0]; k[0] = k[1]; k[1] = tmp; }
                    int slot = 0;
                    for (int u = 0; u <= 2; ++u)
                        for (int w = u; w <= 2; ++w)
                            for (int z = w; z <= 2; ++z) {
                                if (u == k[0] && w == k[1] && z == k[2]) goto found;
                                ++slot;
                            }
                found:
                    v += 0.5 * o[9 + slot] * d[b] * d[e];
                }
            }
            E[3 * i + a] = v;
        }
    }
}

/* MLP features of each particle: the B^3 block of cell moments around its
 * cell (cells outside the grid read as zero), ordered dz-major then dy then
 * dx, each cell as (Q / sq, Px / (sq h), Py / (sq h), Pz / (sq h)), then the
 * offset (x - centre) / h.  X is [n * (4 B^3 + 3)]. */
void ldo_ff_features(int64_t n, const double* x, int G, double L, int B, const double* mom,
                     double sq, double* X) {
    const double h = 2.0 * L / G;
    const int half = B / 2;
    const int K = 4 * B * B * B + 3;
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        cell_of(&x[3 * i], G, L, c);
        double* row = X + (size_t)i * K;
        int f = 0;
        for (int dz = -half; dz <= half; ++dz)
            for (int dy = -half; dy <= half; ++dy)
                for (int dx = -half; dx <= half; ++dx) {
                    const int cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= G || cy >= G || cz >= G) {
                        row[f] = row[f + 1] = row[f + 2] = row[f + 3] = 0.0;
                    } else {
                        const size_t k = ((size_t)cz * G + cy) * G + cx;
                        row[f] = mom[4 * k] / sq;
                        row[f + 1] = mom[4 * k + 1] / (sq * h);
                        row[f + 2] = mom[4 * k + 2] / (sq * h);
                        row[f + 3] = mom[4 * k + 3] / (sq * h);
                    }
                    f += 4;
                }
        for (int k = 0; k < 3; ++k) row[f + k] = (x[3 * i + k] - centre(c[k], G, L)) / h;
    }
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z) {
    const double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* y = W3 silu(W2 silu(W1 x + b1) + b2) + b3 for m rows of X [m*K].  Weights
 * are row-major [in][out]: W1 [K*H], W2 [H*H], W3 [H*O].  bf16 != 0 rounds x,
 * the weights and both hidden activations to BF16 before each product.
 * Optional saves: Z1, A1, Z2, A2 [m*H] (pre-activations and activations as
 * fed to the next product). */
void ldo_mlp_forward(int64_t m, int K, int H, int O, const double* X, const double* W1,
                     const double* b1, const double* W2, const double* b2, const double* W3,
                     const double* b3, int bf16, double* Y, double* Z1, double* A1, double* Z2,
                     double* A2) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        double* z1 = (double*)malloc(sizeof(double) * H);
        double* a1 = (double*)malloc(sizeof(double) * H);
        double* z2 = (double*)malloc(sizeof(double) * H);
        double* a2 = (double*)malloc(sizeof(double) * H);
        const double* xr = X + (size_t)r * K;
        for (int j = 0; j < H; ++j) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) {
                const double a = bf16 ? ldo_bf16(xr[k]) : xr[k];
                const double w = bf16 ? ldo_bf16(W1[(size_t)k * H + j]) : W1[(size_t)k * H + j];
                acc += a * w;
            }
            z1[j] = acc + b1[j];
            a1[j] = silu(z1[j]);
            if (bf16) a1[j] = ldo_bf16(a1[j]);
        }
        for (int j = 0; j < H; ++j) {
            double acc = 0.0;
            for (int k = 0; k < H; ++k) {
                const double w = bf16 ? ldo_bf16(W2[(size_t)k * H + j]) : W2[(size_t)k * H + j];
                acc += a1[k] * w;
            }
            z2[j] = acc + b2[j];
            a2[j] = silu(z2[j]);
            if (bf16) a2[j] = ldo_bf16(a2[j]);
        }
        for (int j = 0; j < O; ++j) {
            double acc = 0.0;
            for (int k = 0; k < H; ++k) {
                const double w = bf16 ? ldo_bf16(W3[(size_t)k * O + j]) : W3[(size_t)k * O + j];
                acc += a2[k] * w;
            }
            Y[(size_t)r * O + j] = acc + b3[j];
        }
        if (Z1) memcpy(Z1 + (size_t)r * H, z1, sizeof(double) * H);
        if (A1) memcpy(A1 + (size_t)r * H, a1, sizeof(double) * H);
        if (Z2) memcpy(Z2 + (size_t)r * H, z2, sizeof(double) * H);
        if (A2) memcpy(A2 + (size_t)r * H, a2, sizeof(double) * H);
        free(z1); free(a1); free(z2); free(a2);
    }
}

/* Loss L = mean over the m x O outputs of (y - t)^2 and its gradients with
 * respect to every weight and bias (manual backpropagation through the
 * forward above, same bf16 mode; derivatives are FP64).  Returns L. */
double ldo_mlp_backward(int64_t m, int K, int H, int O, const double* X, const double* T,
                        const double* W1, const double* b1, const double* W2, const double* b2,
                        const double* W3, const double* b3, int bf16, double* dW1, double* db1,
                        double* dW2, double* db2, double* dW3, double* db3) {
    double* Y = (double*)malloc(sizeof(double) * (size_t)m * O);
    double* Z1 = (double*)malloc(sizeof(double) * (size_t)m * H);
    double* A1 = (double*)malloc(sizeof(double) * (size_t)m * H);
    double* Z2 = (double*)malloc(sizeof(double) * (size_t)m * H);
    double* A2 = (double*)malloc(sizeof(double) * (size_t)m * H);
    ldo_mlp_forward(m, K, H, O, X, W1, b1, W2, b2, W3, b3, bf16, Y, Z1, A1, Z2, A2);
    memset(dW1, 0, sizeof(double) * (size_t)K * H);
    memset(db1, 0, sizeof(double) * H);
    memset(dW2, 0, sizeof(double) * (size_t)H * H);
    memset(db2, 0, sizeof(double) * H);
    memset(dW3, 0, sizeof(double) * (size_t)H * O);
    memset(db3, 0, sizeof(double) * O);
    double loss = 0.0;
    double* dy = (double*)malloc(sizeof(double) * O);
    double* d2 = (double*)malloc(sizeof(double) * H);
    double* d1 = (double*)malloc(sizeof(double) * H);
    const double norm = 1.0 / ((double)m * O);
    for (int64_t r = 0; r < m; ++r) {
        const double* xr = X + (size_t)r * K;
        for (int j = 0; j < O; ++j) {
            const double e = Y[(size_t)r * O + j] - T[(size_t)r * O + j];
            loss += e * e * norm;
            dy[j] = 2.0 * e * norm;
            db3[j] += dy[j];
        }
        for (int k = 0; k < H; ++k) {
            double acc = 0.0;
            for (int j = 0; j < O; ++j) {
                dW3[(size_t)k * O + j] += A2[(size_t)r * H + k] * dy[j];
                const double w = bf16 ? ldo_bf16(W3[(size_t)k * O + j]) : W3[(size_t)k * O + j];
                acc += w * dy[j];
            }
            d2[k] = acc * dsilu(Z2[(size_t)r * H + k]);
            db2[k] += d2[k];
        }
        for (int k = 0; k < H; ++k) {
            double acc = 0.0;
            for (int j = 0; j < H; ++j) {
                dW2[(size_t)k * H + j] += A1[(size_t)r * H + k] * d2[j];
                const double w = bf16 ? ldo_bf16(W2[(size_t)k * H + j]) : W2[(size_t)k * H + j];
                acc += w * d2[j];
            }
            d1[k] = acc * dsilu(Z1[(size_t)r * H + k]);
            db1[k] += d1[k];
        }
        for (int k = 0; k < K; ++k) {
            const double a = bf16 ? ldo_bf16(xr[k]) : xr[k];
            for (int j = 0; j < H; ++j) dW1[(size_t)k * H + j] += a * d1[j];
        }
    }
    free(dy); free(d2); free(d1);
    free(Y); free(Z1); free(A1); free(Z2); free(A2);
    return loss;
}
