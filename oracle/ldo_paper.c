/*
 * ldo_paper.c -- CPU FP64 oracle of the paper's own time-stepping scheme,
 * section 2.2 steps (i)-(vi) read literally with the forces of section 2.1.
 *
 * TEST INFRASTRUCTURE ONLY (see ldo.h): loaded by the tests, the smoke check
 * and the benchmark's CPU-baseline leg; it shares nothing with the GPU
 * library.
 *
 * Step (i)-(ii): a pair interacts when closer than range_factor (r_i + r_j)
 * with r = sigma / 2 (the paper uses 4); both the LJ and the Coulomb force
 * are truncated there without shifting.  The all-pairs loop below is the
 * definition; the cell list of step (i) only decides which pairs can be in
 * range, so it does not appear here.
 *
 * Steps (iii)-(vi): Newton's equation with the Stokes drag of the liquid,
 *   v <- v + dt (F_pair + F_ext(R(t + dt)) - gamma v) / m,
 *   v <- v + kick u          (u a uniformly random unit vector),
 *   x <- x + dt v,
 * m the inertial mass per type, gamma the drag coefficient, F_ext the surface
 * spring, gravity and centrifugal force of ldo_external_force.  The random
 * direction is the normalised triple of ldo_gauss3 (isotropic, so uniform on
 * the sphere).
 */
#include <math.h>
#include <stdlib.h>

#include "ldo.h"

typedef struct {
    double s, c;
} psum;
static void psum_add(psum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double psum_get(const psum* a) { return a->s + a->c; }

static double p_sigma(const ldo_params* p, int a, int b) { return 0.5 * (p->sigma[a] + p->sigma[b]); }
static double p_eps(const ldo_params* p, int a, int b) {
    if (p->use_eps_matrix) return p->eps_matrix[a * LDO_MAX_TYPES + b];
    return sqrt(p->eps[a] * p->eps[b]);
}

void ldo_paper_forces(int64_t n, const double* pos, const int32_t* type, const double* q,
                      const ldo_params* p, const ldo_paper* m, const int64_t* rows,
                      int64_t n_rows, double* F, double* S) {
    const double cq = p->kT * p->bjerrum;
    const int64_t nr = rows ? n_rows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nr; ++k) {
        const int64_t i = rows ? rows[k] : k;
        psum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, ss = {0, 0};
        const int ti = type[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const int tj = type[j];
            const double dx = pos[3 * i] - pos[3 * j];
            const double dy = pos[3 * i + 1] - pos[3 * j + 1];
            const double dz = pos[3 * i + 2] - pos[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            /* range_factor (r_i + r_j) = range_factor sigma_ij */
            const double s = p_sigma(p, ti, tj);
            const double rint = m->range_factor * s;
            if (!(r2 < rint * rint)) continue;
            const double r = sqrt(r2);
            const double e = p_eps(p, ti, tj);
            const double sr2 = s * s / r2, sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
            const double glj = 24.0 * e * (2.0 * sr12 - sr6) / r2;   /* -dU/dr / r */
            const double k = cq * q[i] * q[j];
            const double gc = k / (r2 * r);
            const double g = glj + gc;
            psum_add(&fx, g * dx);
            psum_add(&fy, g * dy);
            psum_add(&fz, g * dz);
            psum_add(&ss, fabs(glj) * r + fabs(k) / r2);
        }
        if (F) {
            F[3 * k] = psum_get(&fx);
            F[3 * k + 1] = psum_get(&fy);
            F[3 * k + 2] = psum_get(&fz);
        }
        if (S) S[k] = psum_get(&ss);
    }
}

int64_t ldo_paper_run(int64_t n, double* x, double* v, const int32_t* type, const double* q,
                      const int64_t* ids, const ldo_params* p, const ldo_paper* m,
                      const ldo_radius* R, double dt, int64_t n_steps, uint64_t seed,
                      int64_t* step, double* t) {
    double* Fp = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    int64_t bad = -1;
    for (int64_t k = 0; k < n_steps; ++k) {
        const int64_t n_now = *step;
        const double t_new = *t + dt;
        const double Rn = ldo_radius_at(R, t_new);   /* step (iii) before step (iv) */
        ldo_paper_forces(n, x, type, q, p, m, NULL, 0, Fp, NULL);
        int flag = 0;
#pragma omp parallel for schedule(static) reduction(| : flag)
        for (int64_t i = 0; i < n; ++i) {
            const int ti = type[i];
            double Fe[3];
            ldo_external_force(&x[3 * i], ti, p, Rn, Fe);
            const double g = p->gamma[ti], mi = m->inertial_mass[ti];
            double u[3] = {0.0, 0.0, 0.0};
            if (m->kick > 0.0) {
                double xi[3];
                ldo_gauss3(ids ? ids[i] : i, n_now, seed, 0u, xi);
                const double len = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
                for (int c = 0; c < 3; ++c) u[c] = xi[c] / len;
            }
            for (int c = 0; c < 3; ++c) {
                double vc = v[3 * i + c] + dt * (Fp[3 * i + c] + Fe[c] - g * v[3 * i + c]) / mi;
                vc += m->kick * u[c];
                const double d = dt * vc;
                if (!isfinite(d) || (p->jump_max > 0.0 && fabs(d) > p->jump_max)) flag = 1;
                v[3 * i + c] = vc;
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
