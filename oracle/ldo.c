/*
 * ldo.c -- CPU FP64 oracle (test infrastructure only; see ldo.h).
 *
 * Written for reading, not for speed: one scalar loop per formula, FP64
 * throughout, ascending-index Neumaier sums.  Build with -ffp-contract=off and
 * without -ffast-math so that each line rounds as written.
 */
#include "ldo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Neumaier (improved Kahan) summation.                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64-bit     */
/* multiplications with the Weyl key schedule.                              */
/* ------------------------------------------------------------------------ */
void ldo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 23-bit uniform ((u >> 9) + 1/2) 2^-23 in (0,1); every value is exact in
 * FP32 as well as FP64, so a single-precision consumer sees the same U. */
static double u23(uint32_t u) { return ((double)(u >> 9) + 0.5) * (1.0 / 8388608.0); }

void ldo_gauss3(int64_t id, int64_t step, uint64_t seed, uint32_t tag, double xi[3]) {
    uint32_t ctr[4], key[2], r[4];
    ctr[0] = (uint32_t)(uint64_t)id;
    ctr[1] = (uint32_t)(uint64_t)step;
    ctr[2] = (uint32_t)((uint64_t)step >> 32);
    ctr[3] = tag;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    ldo_philox4x32_10(ctr, key, r);
    double U0 = u23(r[0]), U1 = u23(r[1]), U2 = u23(r[2]), U3 = u23(r[3]);
    double a = sqrt(-2.0 * log(U0));
    double b = sqrt(-2.0 * log(U2));
    xi[0] = a * cos(2.0 * M_PI * U1);
    xi[1] = a * sin(2.0 * M_PI * U1);
    xi[2] = b * cos(2.0 * M_PI * U3);
}

/* ------------------------------------------------------------------------ */
/* Initial placement: uniform in the ball, no overlaps (section 2.1).       */
/* ------------------------------------------------------------------------ */
int64_t ldo_sample_ball(int64_t n, const int32_t* type, const double* sigma, double R0,
                        uint64_t seed, int64_t max_tries, double* x) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        int placed = 0;
        for (int64_t k = 0; k < max_tries && !placed; ++k) {
            uint32_t ctr[4] = {(uint32_t)i, (uint32_t)k, 0u, 1u}, r[4];
            ldo_philox4x32_10(ctr, key, r);
            double v[3];
            for (int c = 0; c < 3; ++c) v[c] = 2.0 * u23(r[c]) - 1.0;
            if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > 1.0) continue;
            double c3[3];
            for (int c = 0; c < 3; ++c) c3[c] = (double)(float)(R0 * v[c]);
            int clash = 0;
            for (int64_t j = 0; j < i && !clash; ++j) {
                const double s = 0.5 * (sigma[type[i]] + sigma[type[j]]);
                const double dx = c3[0] - x[3 * j];
                const double dy = c3[1] - x[3 * j + 1];
                const double dz = c3[2] - x[3 * j + 2];
                if (dx * dx + dy * dy + dz * dz < s * s) clash = 1;
            }
            if (clash) continue;
            for (int c = 0; c < 3; ++c) x[3 * i + c] = c3[c];
            placed = 1;
        }
        if (!placed) return i;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Droplet radius R(t) (section 2.1, section 2.2 step (iii)).               */
/* ------------------------------------------------------------------------ */
double ldo_radius_at(const ldo_radius* R, double t) {
    if (R->kind == LDO_R_LINEAR) {
        double f = (R->T > 0.0) ? t / R->T : 1.0;
        if (f > 1.0) f = 1.0;
        if (f < 0.0) f = 0.0;
        return R->R0 + (R->R1 - R->R0) * f;
    }
    if (R->kind == LDO_R_SQUARE_LAW) {
        double r2 = R->R0 * R->R0 - 2.0 * R->a * t;
        double m2 = R->R_min * R->R_min;
        if (r2 < m2) r2 = m2;
        return sqrt(r2);
    }
    if (R->kind == LDO_R_TABLE) {
        /* the knot interval holding t, by a plain scan from the end */
        const int m = R->n_knots < LDO_R_TABLE_MAX ? R->n_knots : LDO_R_TABLE_MAX;
        if (m < 1) return R->R0;      /* no table: the library refuses such a schedule */
        if (t >= R->tab_t[m - 1]) return R->tab_R[m - 1];
        if (t <= R->tab_t[0]) return R->tab_R[0];
        int k = m - 1;
        while (R->tab_t[k - 1] > t) --k;
        const double w = (t - R->tab_t[k - 1]) / (R->tab_t[k] - R->tab_t[k - 1]);
        return (1.0 - w) * R->tab_R[k - 1] + w * R->tab_R[k];
    }
    return R->R0;
}

/* ------------------------------------------------------------------------ */
/* Pair parameters.                                                          */
/* ------------------------------------------------------------------------ */
static double sigma_ij(const ldo_params* p, int ti, int tj) {
    return 0.5 * (p->sigma[ti] + p->sigma[tj]);
}
static double eps_ij(const ldo_params* p, int ti, int tj) {
    if (p->use_eps_matrix) return p->eps_matrix[ti * LDO_MAX_TYPES + tj];
    return sqrt(p->eps[ti] * p->eps[tj]);
}

/* One row of the pair sum: force on particle i from every j != i, in
 * ascending j.  LJ: 4 eps [(s/r)^12 - (s/r)^6], truncated at lj_cut * s_ij
 * without shift.  Coulomb: kT l_B q_i q_j / r, over all pairs (or truncated
 * without shift at coul_cut). */
static void pair_row(int64_t i, int64_t n, const double* pos, const int32_t* type,
                     const double* q, const ldo_params* p,
                     double F[3], double* S, double* Ulj, double* Uc) {
    nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, sS = {0, 0}, slj = {0, 0}, sc = {0, 0};
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const int ti = type[i];
    const double cq = p->kT * p->bjerrum;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const int tj = type[j];
        double dx = xi - pos[3 * j];
        double dy = yi - pos[3 * j + 1];
        double dz = zi - pos[3 * j + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        double r = sqrt(r2);
        /* Lennard-Jones */
        double s = sigma_ij(p, ti, tj);
        double rc = p->lj_cut * s;
        if (r2 < rc * rc) {
            double e = eps_ij(p, ti, tj);
            double sr2 = (s * s) / r2;
            double sr6 = sr2 * sr2 * sr2;
            double sr12 = sr6 * sr6;
            /* -dU/dr / r, so that f = (-dU/dr) * (r_vec / r) */
            double g = 24.0 * e * (2.0 * sr12 - sr6) / r2;
            nsum_add(&fx, g * dx);
            nsum_add(&fy, g * dy);
            nsum_add(&fz, g * dz);
            nsum_add(&sS, fabs(g) * r);
            nsum_add(&slj, 0.5 * 4.0 * e * (sr12 - sr6));
        }
        /* Coulomb */
        if (p->coul_cut <= 0.0 || r < p->coul_cut) {
            double k = cq * q[i] * q[j];
            double g = k / (r2 * r);
            nsum_add(&fx, g * dx);
            nsum_add(&fy, g * dy);
            nsum_add(&fz, g * dz);
            nsum_add(&sS, fabs(k) / r2);
            nsum_add(&sc, 0.5 * k / r);
        }
    }
    F[0] = nsum_get(&fx);
    F[1] = nsum_get(&fy);
    F[2] = nsum_get(&fz);
    *S = nsum_get(&sS);
    *Ulj = nsum_get(&slj);
    *Uc = nsum_get(&sc);
}

void ldo_pair_forces(int64_t n, const double* pos, const int32_t* type, const double* q,
                     const ldo_params* p, const int64_t* rows, int64_t n_rows,
                     double* F, double* S, double* U) {
    if (rows == NULL) n_rows = n;
    double* ulj = (double*)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(double));
    double* uc = (double*)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = rows ? rows[r] : r;
        double f[3], s, a, b;
        pair_row(i, n, pos, type, q, p, f, &s, &a, &b);
        if (F) { F[3 * r] = f[0]; F[3 * r + 1] = f[1]; F[3 * r + 2] = f[2]; }
        if (S) S[r] = s;
        ulj[r] = a;
        uc[r] = b;
    }
    if (U) {
        nsum a = {0, 0}, b = {0, 0};
        for (int64_t r = 0; r < n_rows; ++r) { nsum_add(&a, ulj[r]); nsum_add(&b, uc[r]); }
        U[0] = nsum_get(&a);
        U[1] = nsum_get(&b);
    }
    free(ulj);
    free(uc);
}

/* ------------------------------------------------------------------------ */
/* External forces (section 2.2 steps (iv)-(v)).                            */
/* ------------------------------------------------------------------------ */
void ldo_external_force(const double x[3], int32_t t, const ldo_params* p, double R,
                        double F[3]) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    F[0] = F[1] = F[2] = 0.0;
    /* Surface spring: equilibrium wall_offset inside the surface, pushing
     * inward only (a one-sided harmonic wall).  Band mode: the spring acts
     * only within one NP radius of the surface on either side. */
    double Rw = R - p->wall_offset[t];
    int active = (r > Rw);
    if (p->wall_band) {
        double h = 0.5 * p->sigma[t];
        active = active && (r > R - h) && (r < R + h);
    }
    if (active && r > 0.0) {
        double m = -p->k_wall[t] * (r - Rw) / r;
        F[0] += m * x[0];
        F[1] += m * x[1];
        F[2] += m * x[2];
    }
    /* Gravity with buoyancy folded into the mass. */
    F[0] += p->mass[t] * p->gravity[0];
    F[1] += p->mass[t] * p->gravity[1];
    F[2] += p->mass[t] * p->gravity[2];
    /* Centrifugal force from the droplet's rotation. */
    double c = p->mass[t] * p->omega * p->omega;
    F[0] += c * x[0];
    F[1] += c * x[1];
    if (p->rotation == 0) F[2] += c * x[2];
}

/* ------------------------------------------------------------------------ */
/* Overdamped Euler-Maruyama (section 2.2 step (vi)).                       */
/* ------------------------------------------------------------------------ */
int64_t ldo_run(int64_t n, double* x, const int32_t* type, const double* q,
                const int64_t* ids, const ldo_params* p, const ldo_radius* R,
                double dt, int64_t n_steps, uint64_t seed, int64_t* step, double* t) {
    double* Fp = (double*)malloc((size_t)n * 3 * sizeof(double));
    int64_t bad = -1;
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t n_now = *step;
        const double t_new = *t + dt;
        /* The new radius comes before the surface forces (steps (iii)-(iv)). */
        const double Rn = ldo_radius_at(R, t_new);
        ldo_pair_forces(n, x, type, q, p, NULL, n, Fp, NULL, NULL);
        int flag = 0;
#pragma omp parallel for schedule(static) reduction(| : flag)
        for (int64_t i = 0; i < n; ++i) {
            const int ti = type[i];
            double Fe[3];
            ldo_external_force(&x[3 * i], ti, p, Rn, Fe);
            const double mu = 1.0 / p->gamma[ti];
            double xi[3] = {0.0, 0.0, 0.0};
            double amp = 0.0;
            if (p->noise != 0 && p->kT > 0.0) {
                ldo_gauss3(ids ? ids[i] : i, n_now, seed, 0u, xi);
                amp = sqrt(2.0 * p->kT * mu * dt);
                if (p->noise == 2) {
                    /* fixed magnitude sqrt(3) (same mean square), random direction */
                    double m = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
                    double f = sqrt(3.0) / m;
                    xi[0] *= f; xi[1] *= f; xi[2] *= f;
                }
            }
            for (int c = 0; c < 3; ++c) {
                double d = mu * dt * (Fp[3 * i + c] + Fe[c]) + amp * xi[c];
                if (!isfinite(d) || (p->jump_max > 0.0 && fabs(d) > p->jump_max)) flag = 1;
                x[3 * i + c] += d;
            }
        }
        if (flag && bad < 0) bad = n_now;
        *t = t_new;
        *step = n_now + 1;
    }
    free(Fp);
    return bad;
}

/* One Euler-Maruyama step for the listed rows only: the pair forces on each
 * listed particle come from all n particles at their current positions, so
 * the new positions of a sample can be checked without running the whole
 * system.  x_rows_out is [n_rows*3]; step / t are not advanced. */
int64_t ldo_step_rows(int64_t n, const double* x, const int32_t* type, const double* q,
                      const int64_t* ids, const ldo_params* p, const ldo_radius* R,
                      double dt, uint64_t seed, int64_t step, double t,
                      const int64_t* rows, int64_t n_rows, double* x_rows_out) {
    double* Fp = (double*)malloc((size_t)(n_rows > 0 ? n_rows : 1) * 3 * sizeof(double));
    const double Rn = ldo_radius_at(R, t + dt);
    ldo_pair_forces(n, x, type, q, p, rows, n_rows, Fp, NULL, NULL);
    int flag = 0;
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = rows[r];
        const int ti = type[i];
        double Fe[3];
        ldo_external_force(&x[3 * i], ti, p, Rn, Fe);
        const double mu = 1.0 / p->gamma[ti];
        double xi[3] = {0.0, 0.0, 0.0};
        double amp = 0.0;
        if (p->noise != 0 && p->kT > 0.0) {
            ldo_gauss3(ids ? ids[i] : i, step, seed, 0u, xi);
            amp = sqrt(2.0 * p->kT * mu * dt);
            if (p->noise == 2) {
                double m = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
                double f = sqrt(3.0) / m;
                xi[0] *= f; xi[1] *= f; xi[2] *= f;
            }
        }
        for (int c = 0; c < 3; ++c) {
            double d = mu * dt * (Fp[3 * r + c] + Fe[c]) + amp * xi[c];
            if (!isfinite(d) || (p->jump_max > 0.0 && fabs(d) > p->jump_max)) flag = 1;
            x_rows_out[3 * r + c] = x[3 * i + c] + d;
        }
    }
    free(Fp);
    return flag ? step : -1;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                              */
/* ------------------------------------------------------------------------ */
void ldo_diagnostics(int64_t n, const double* x, const int32_t* type, const double* q,
                     const ldo_params* p, double R, double out[10]) {
    double* F = (double*)malloc((size_t)n * 3 * sizeof(double));
    double U[2];
    ldo_pair_forces(n, x, type, q, p, NULL, n, F, NULL, U);
    nsum uw = {0, 0}, ug = {0, 0}, uc = {0, 0}, fx = {0, 0}, fy = {0, 0}, fz = {0, 0};
    double fmax = 0.0, xmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int t = type[i];
        const double* xi = &x[3 * i];
        double r = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        double Rw = R - p->wall_offset[t];
        int active = (r > Rw);
        if (p->wall_band) {
            double h = 0.5 * p->sigma[t];
            active = active && (r > R - h) && (r < R + h);
        }
        if (active) nsum_add(&uw, 0.5 * p->k_wall[t] * (r - Rw) * (r - Rw));
        nsum_add(&ug, -p->mass[t] * (p->gravity[0] * xi[0] + p->gravity[1] * xi[1] +
                                     p->gravity[2] * xi[2]));
        double rho2 = xi[0] * xi[0] + xi[1] * xi[1] + (p->rotation == 0 ? xi[2] * xi[2] : 0.0);
        nsum_add(&uc, -0.5 * p->mass[t] * p->omega * p->omega * rho2);
        nsum_add(&fx, F[3 * i]);
        nsum_add(&fy, F[3 * i + 1]);
        nsum_add(&fz, F[3 * i + 2]);
        double fm = sqrt(F[3 * i] * F[3 * i] + F[3 * i + 1] * F[3 * i + 1] +
                         F[3 * i + 2] * F[3 * i + 2]);
        if (fm > fmax) fmax = fm;
        if (r > xmax) xmax = r;
    }
    out[0] = U[0];
    out[1] = U[1];
    out[2] = nsum_get(&uw);
    out[3] = nsum_get(&ug);
    out[4] = nsum_get(&uc);
    out[5] = nsum_get(&fx);
    out[6] = nsum_get(&fy);
    out[7] = nsum_get(&fz);
    out[8] = fmax;
    out[9] = xmax;
    free(F);
}

double ldo_msd(int64_t n, const double* x, const double* x0) {
    nsum s = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[3 * i] - x0[3 * i];
        double dy = x[3 * i + 1] - x0[3 * i + 1];
        double dz = x[3 * i + 2] - x0[3 * i + 2];
        nsum_add(&s, dx * dx + dy * dy + dz * dz);
    }
    return n > 0 ? nsum_get(&s) / (double)n : 0.0;
}

/* ------------------------------------------------------------------------ */
/* RDF, Eq. (6), and radial concentration, Eq. (8) (section 3.2).           */
/* ------------------------------------------------------------------------ */
void ldo_rdf(int64_t n, const double* x, double r_max, int32_t n_bins, double V,
             const double centre[3], uint64_t* counts, uint64_t* ccounts,
             double* g, double* cbar) {
    const double dr = r_max / n_bins;
    for (int b = 0; b < n_bins; ++b) { counts[b] = 0; ccounts[b] = 0; }
#pragma omp parallel
    {
        uint64_t* loc = (uint64_t*)calloc((size_t)n_bins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t j = i + 1; j < n; ++j) {
                double dx = x[3 * i] - x[3 * j];
                double dy = x[3 * i + 1] - x[3 * j + 1];
                double dz = x[3 * i + 2] - x[3 * j + 2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r < r_max) {
                    int b = (int)floor(r / dr);
                    if (b >= 0 && b < n_bins) loc[b] += 1;
                }
            }
        }
#pragma omp critical
        for (int b = 0; b < n_bins; ++b) counts[b] += loc[b];
        free(loc);
    }
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[3 * i] - centre[0];
        double dy = x[3 * i + 1] - centre[1];
        double dz = x[3 * i + 2] - centre[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r < r_max) {
            int b = (int)floor(r / dr);
            if (b >= 0 && b < n_bins) ccounts[b] += 1;
        }
    }
    for (int b = 0; b < n_bins; ++b) {
        double r0 = b * dr, r1 = (b + 1) * dr;
        double dV = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        /* sum_i psi_i / N over (N-1) dV / V, with sum_i psi_i = 2 * pair count */
        if (g) g[b] = (2.0 * (double)counts[b] / (double)n) / ((double)(n - 1) * dV / V);
        if (cbar) cbar[b] = ((double)ccounts[b] / (double)n) / (dV / V);
    }
}

/* ------------------------------------------------------------------------ */
/* Fractal dimension (section 3.1).                                          */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

void ldo_fractal(int64_t n, const double* x, double k_f, double d, double eps0,
                 int32_t max_scales, double out[4], int64_t* box_counts) {
    /* Eq. (4): centre of mass; Eq. (3): radius of gyration. */
    nsum cx = {0, 0}, cy = {0, 0}, cz = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        nsum_add(&cx, x[3 * i]);
        nsum_add(&cy, x[3 * i + 1]);
        nsum_add(&cz, x[3 * i + 2]);
    }
    double r0[3] = {nsum_get(&cx) / n, nsum_get(&cy) / n, nsum_get(&cz) / n};
    nsum s2 = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double dx = r0[0] - x[3 * i], dy = r0[1] - x[3 * i + 1], dz = r0[2] - x[3 * i + 2];
        nsum_add(&s2, dx * dx + dy * dy + dz * dz);
    }
    double Rg = sqrt(nsum_get(&s2) / n);
    out[0] = Rg;
    /* Eq. (2) solved for D_f. */
    out[1] = log((double)n / k_f) / log(2.0 * Rg / d);

    /* Box counting: boxes of side eps0 * 2^k anchored at the bounding-box
     * minimum, for every k with eps_k <= R_g; slope of ln N(eps) against
     * ln eps over k >= 1. */
    double lo[3] = {x[0], x[1], x[2]};
    for (int64_t i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
    uint64_t* keys = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(max_scales > 0 ? max_scales : 1));
    double* ly = (double*)malloc(sizeof(double) * (size_t)(max_scales > 0 ? max_scales : 1));
    int K = 0;
    for (int k = 0; k < max_scales; ++k) {
        double e = eps0 * ldexp(1.0, k);
        if (e > Rg) break;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t ix = (uint64_t)floor((x[3 * i] - lo[0]) / e);
            uint64_t iy = (uint64_t)floor((x[3 * i + 1] - lo[1]) / e);
            uint64_t iz = (uint64_t)floor((x[3 * i + 2] - lo[2]) / e);
            keys[i] = (ix << 42) | (iy << 21) | iz;
        }
        qsort(keys, (size_t)n, sizeof(uint64_t), cmp_u64);
        int64_t cnt = n > 0 ? 1 : 0;
        for (int64_t i = 1; i < n; ++i) cnt += (keys[i] != keys[i - 1]);
        if (box_counts) box_counts[k] = cnt;
        lx[k] = log(e);
        ly[k] = log((double)cnt);
        K = k + 1;
    }
    out[3] = (double)K;
    if (K >= 3) {
        /* ordinary least squares over k = 1 .. K-1 */
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        const int m = K - 1;
        for (int k = 1; k < K; ++k) { sx += lx[k]; sy += ly[k]; }
        const double mx = sx / m, my = sy / m;
        for (int k = 1; k < K; ++k) {
            sxx += (lx[k] - mx) * (lx[k] - mx);
            sxy += (lx[k] - mx) * (ly[k] - my);
        }
        out[2] = -sxy / sxx;
    } else {
        out[2] = NAN;
    }
    free(lx);
    free(ly);
    free(keys);
}
