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
