/*
 * ldo_agg.c -- CPU oracle of the aggregate statistics the paper extracts in
 * post-processing (section 2.1: the number of sub-aggregates and aggregate
 * statistics; section 1: the number of NPs at the droplet surface, N_surf).
 *
 * TEST INFRASTRUCTURE ONLY (see ldo.h).
 *
 * Sub-aggregates: connected components of the contact graph, two NPs in
 * contact when r < contact_factor sigma_ij (sigma_ij the LB contact
 * diameter).  Union-find over all pairs in index order; every union hangs
 * the larger root under the smaller, so each component's root is its
 * smallest index, which is the label.
 *
 * N_surf: NPs whose distance from the droplet surface is below one NP
 * radius, | |x| - R | < sigma_t / 2, counted per type.
 *
 * Surface fractal dimension (section 3.1: the fractal equation, Eqs. (2)-(4),
 * taken at dimension two on the sphere): the surface NPs above, their
 * contact-graph components, and for the largest component (ties: the
 * smallest label) the radius of gyration from geodesic distances on the
 * sphere of radius R about the component's mean direction, then D_f from
 * N = k_f (2 R_g / d)^D_f.
 */
#include <math.h>
#include <stdlib.h>

#include "ldo.h"

static int64_t uf_find(int64_t* parent, int64_t a) {
    while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
    }
    return a;
}

int64_t ldo_components(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                       double contact_factor, int64_t* labels) {
    int64_t* parent = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            const double dx = x[3 * i] - x[3 * j];
            const double dy = x[3 * i + 1] - x[3 * j + 1];
            const double dz = x[3 * i + 2] - x[3 * j + 2];
            const double s = contact_factor * 0.5 * (p->sigma[type[i]] + p->sigma[type[j]]);
            if (!(dx * dx + dy * dy + dz * dz < s * s)) continue;
            int64_t a = uf_find(parent, i), b = uf_find(parent, j);
            if (a == b) continue;
            if (a < b) parent[b] = a;
            else parent[a] = b;
        }
    }
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = uf_find(parent, i);
        if (labels) labels[i] = r;
        if (r == i) ++count;
    }
    free(parent);
    return count;
}

void ldo_surface_count(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                       double R, int64_t* counts) {
    for (int t = 0; t < p->n_types; ++t) counts[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double r = sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] +
                              x[3 * i + 2] * x[3 * i + 2]);
        if (fabs(r - R) < 0.5 * p->sigma[type[i]]) ++counts[type[i]];
    }
}

/* Angle between the unit vectors a and b, from the sine (cross product) and
 * the cosine (dot product): accurate also for small angles, where acos of
 * the dot product loses half the digits. */
static double angle_between(const double a[3], const double b[3]) {
    const double cx = a[1] * b[2] - a[2] * b[1];
    const double cy = a[2] * b[0] - a[0] * b[2];
    const double cz = a[0] * b[1] - a[1] * b[0];
    return atan2(sqrt(cx * cx + cy * cy + cz * cz), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

void ldo_surface_fractal(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                         double R, double contact_factor, double k_f, double d, int64_t stats[3],
                         double out[3], int64_t* labels) {
    /* 1. the surface NPs, in index order */
    int64_t* idx = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t ns = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double r = sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] +
                              x[3 * i + 2] * x[3 * i + 2]);
        if (labels) labels[i] = -1;
        if (fabs(r - R) < 0.5 * p->sigma[type[i]]) idx[ns++] = i;
    }
    /* 2. components of the contact graph among them; the root of each is its
     *    smallest original index */
    int64_t* parent = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* size = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
    for (int64_t a = 0; a < ns; ++a) {
        const int64_t i = idx[a];
        for (int64_t b = a + 1; b < ns; ++b) {
            const int64_t j = idx[b];
            const double dx = x[3 * i] - x[3 * j];
            const double dy = x[3 * i + 1] - x[3 * j + 1];
            const double dz = x[3 * i + 2] - x[3 * j + 2];
            const double s = contact_factor * 0.5 * (p->sigma[type[i]] + p->sigma[type[j]]);
            if (!(dx * dx + dy * dy + dz * dz < s * s)) continue;
            const int64_t ri = uf_find(parent, i), rj = uf_find(parent, j);
            if (ri == rj) continue;
            if (ri < rj) parent[rj] = ri;
            else parent[ri] = rj;
        }
    }
    int64_t comps = 0, best = -1;
    for (int64_t a = 0; a < ns; ++a) {
        const int64_t r = uf_find(parent, idx[a]);
        if (labels) labels[idx[a]] = r;
        ++size[r];
    }
    for (int64_t a = 0; a < ns; ++a) {
        const int64_t i = idx[a];
        if (uf_find(parent, i) != i) continue;
        ++comps;
        if (best < 0 || size[i] > size[best]) best = i;   /* index order: ties keep the smaller */
    }
    stats[0] = comps;
    stats[1] = best < 0 ? 0 : size[best];
    stats[2] = best;
    out[0] = out[1] = out[2] = NAN;
    if (best >= 0) {
        /* 3. the largest component's mean direction and mean diameter */
        double su[3] = {0.0, 0.0, 0.0}, ssig = 0.0;
        int64_t m = 0;
        for (int64_t a = 0; a < ns; ++a) {
            const int64_t i = idx[a];
            if (uf_find(parent, i) != best) continue;
            const double r = sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] +
                                  x[3 * i + 2] * x[3 * i + 2]);
            for (int k = 0; k < 3; ++k) su[k] += x[3 * i + k] / r;
            ssig += p->sigma[type[i]];
            ++m;
        }
        const double nu = sqrt(su[0] * su[0] + su[1] * su[1] + su[2] * su[2]);
        const double dm = d > 0.0 ? d : ssig / (double)m;
        if (nu > 0.0) {
            const double u0[3] = {su[0] / nu, su[1] / nu, su[2] / nu};
            /* 4. radius of gyration from the geodesic distances R theta_i */
            double s2 = 0.0;
            for (int64_t a = 0; a < ns; ++a) {
                const int64_t i = idx[a];
                if (uf_find(parent, i) != best) continue;
                const double r = sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] +
                                      x[3 * i + 2] * x[3 * i + 2]);
                const double u[3] = {x[3 * i] / r, x[3 * i + 1] / r, x[3 * i + 2] / r};
                const double g = R * angle_between(u, u0);
                s2 += g * g;
            }
            const double Rg = sqrt(s2 / (double)m);
            out[0] = Rg;
            out[1] = dm;
            /* 5. the fractal equation at dimension two */
            if (m >= 2) out[2] = log((double)m / k_f) / log(2.0 * Rg / dm);
        }
    }
    free(size);
    free(parent);
    free(idx);
}
