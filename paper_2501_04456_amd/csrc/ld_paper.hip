// The paper's own scheme, section 2.2 steps (i)-(vi) read literally with the
// forces of section 2.1:
//
//   (i)   slots sorted by cells of side >= the largest pair range;
//   (ii)  pair forces of the pairs closer than range_factor (r_i + r_j),
//         r = sigma / 2, LJ and Coulomb both truncated there without shift,
//         summed over the 27 cells around each particle;
//   (iii) R(t + dt);
//   (iv)-(v) surface spring (band-limited with ld_params.wall_band), gravity,
//         centrifugal force;
//   (vi)  Newton's equation with Stokes drag and the random velocity vector:
//         v <- v + dt (F_pair + F_ext - gamma v) / m,  v <- v + kick u,
//         x <- x + dt v,
//         u the normalised Box-Muller triple of the context's noise stream
//         (uniform on the unit sphere).
//
// Pairs in range are few per particle (tens while dispersed, hundreds once
// aggregated), so the pair math is FP64 throughout: the range test agrees
// with FP64 positions and the forces need no compensation.  Velocities are
// FP64, positions stay (hi, lo) FP32 pairs.
#include <algorithm>
#include <cmath>
#include <new>

#include "ld_host.h"
#include "ld_update_core.h"

namespace ld {

using host::fail;

constexpr int kPmMaxCells = 64;         // cells per axis at most

struct PmGrid {
    double L;                           // half width of the cube holding every particle
    double hc;                          // cell side (>= the largest pair range)
    int Gc;                             // cells per axis
    int pad;
};

// Pair constants: range^2, sigma^2 and 24 eps per type pair (FP64).
struct PmTable {
    int T;
    double rint2[kMaxTypes * kMaxTypes];
    double sig2[kMaxTypes * kMaxTypes];
    double e24[kMaxTypes * kMaxTypes];
    double inv_m[kMaxTypes];            // 1 / inertial mass
    double gamma[kMaxTypes];
    double rmax;                        // largest pair range
    double kick;
};

struct PaperMode {
    ld_paper_config cfg{};
    PmTable tab{};
    double* v = nullptr;                // [3][n] velocities, slot order
    double* v2 = nullptr;               // [3][n] second buffer (re-sort)
    double* F = nullptr;                // [3][n] pair forces, slot order
    PmGrid* grid = nullptr;             // device
    int* cfirst = nullptr;              // [64^3 + 1] first slot of every cell
};

namespace {

constexpr int kB = 256;
constexpr int kNC = kPmMaxCells * kPmMaxCells * kPmMaxCells;
constexpr int kPmWin = 4;               // candidates loaded together (2 and 8 are slower)

__global__ __launch_bounds__(kB) void k_pm_absmax(const float4* __restrict__ pos, int n,
                                                  float* part) {
    __shared__ float red[kB];
    float m = 0.f;
    for (int s = blockIdx.x * kB + threadIdx.x; s < n; s += gridDim.x * kB) {
        const float4 h = pos[s];
        m = fmaxf(m, fmaxf(fabsf(h.x), fmaxf(fabsf(h.y), fabsf(h.z))));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ __forceinline__ int pm_cell1(double x, double L, double h, int G) {
    int c = (int)floor((x + L) / h);
    return c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
}

// Grid from the 64 partial maxima (block 0 stores it), cell keys
// (cell << 32 | slot) from the FP64 positions, and the first radix pass's
// digit counts of each radix tile.
__global__ __launch_bounds__(kB) void k_pm_keys(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo, int n,
                                                const float* __restrict__ part, double rmax,
                                                PmGrid* g, unsigned long long* keys,
                                                unsigned* hist, int nwg) {
    __shared__ PmGrid sg;
    __shared__ unsigned h[256];
    const int t = threadIdx.x;
    h[t] = 0u;
    if (t < 64) {
        float m = part[t];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (t == 0) {
            m = fmaxf(m, 1e-3f);
            const double L = (double)(m * 1.0009765625f);
            int G = (int)floor(2.0 * L / rmax);
            G = G < 1 ? 1 : (G > kPmMaxCells ? kPmMaxCells : G);
            sg.L = L;
            sg.Gc = G;
            sg.hc = 2.0 * L / G;
            sg.pad = 0;
            if (blockIdx.x == 0) *g = sg;
        }
    }
    __syncthreads();
    const int G = sg.Gc;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int s = blockIdx.x * kRadixTile + r * kB + t;
        if (s < n) {
            const float4 hp = pos[s], l = lo[s];
            const int cx = pm_cell1((double)hp.x + (double)l.x, sg.L, sg.hc, G),
                      cy = pm_cell1((double)hp.y + (double)l.y, sg.L, sg.hc, G),
                      cz = pm_cell1((double)hp.z + (double)l.z, sg.L, sg.hc, G);
            const unsigned c = (unsigned)((cz * G + cy) * G + cx);
            keys[s] = ((unsigned long long)c << 32) | (unsigned)s;
            atomicAdd(&h[c & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)t * nwg + blockIdx.x] = h[t];
}

// First slot of every cell of the grid (G^3 cells, G from the device grid).
__global__ __launch_bounds__(kB) void k_pm_first(const unsigned long long* __restrict__ keys,
                                                 int n, const PmGrid* __restrict__ g,
                                                 int* cfirst) {
    const int G = g->Gc;
    fill_cell_first(keys, n, G * G * G, blockIdx.x * kB + threadIdx.x, cfirst);
}

// Velocities follow the slots: v2[.][s] = v[.][src(s)].
__global__ __launch_bounds__(kB) void k_pm_permute_v(const unsigned long long* __restrict__ keys,
                                                     int n, const double* __restrict__ v,
                                                     double* __restrict__ v2) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const int src = (int)(unsigned)keys[s];
    v2[s] = v[src];
    v2[(size_t)n + s] = v[(size_t)n + src];
    v2[2 * (size_t)n + s] = v[2 * (size_t)n + src];
}

// Step (ii): the truncated pair forces on slot i from the 27 cells around
// its cell, in cell order and slot order within a cell (FP64).  The three
// cells of an x-row are consecutive in key order, so their slots form one
// range [cfirst[a], cfirst[b + 1]) and nine ranges cover the 27 cells.  Each
// candidate is first screened in FP32 from its hi word against the largest
// range widened by the screen's worst rounding (coordinates within L: hi
// rounding and the FP32 difference move each component by <= L 2^-22, the
// squared sum by a few ulp), so every pair the FP64 test keeps passes the
// screen; only the survivors load lo and the type.
__global__ __launch_bounds__(kB) void k_pm_forces(const float4* __restrict__ pos,
                                                  const float4* __restrict__ lo,
                                                  const int* __restrict__ typ,
                                                  const unsigned long long* __restrict__ keys,
                                                  const PmGrid* __restrict__ g,
                                                  const int* __restrict__ cfirst, int n,
                                                  PmTable tb, double* F) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const PmGrid gr = *g;
    const double wide = tb.rmax + gr.L * 0x1p-20;
    const float screen2 = (float)(wide * wide * (1.0 + 0x1p-18));
    const float4 hi = pos[i], li = lo[i];
    const double xi = (double)hi.x + (double)li.x, yi = (double)hi.y + (double)li.y,
                 zi = (double)hi.z + (double)li.z;
    const int ti = typ[i];
    const double qi = (double)hi.w;                 // q_hat = q sqrt(kT l_B)
    const int G = gr.Gc;
    const int c = (int)(keys[i] >> 32);
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < G - 1 ? cx + 1 : G - 1;
    // the nine row ranges first (independent loads), empty where the row
    // falls outside the grid
    int r0[9], r1[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int z = cz + k / 3 - 1, y = cy + k % 3 - 1;
        const bool in = z >= 0 && z < G && y >= 0 && y < G;
        const int row = (z * G + y) * G;
        r0[k] = in ? cfirst[row + x0] : 0;
        r1[k] = in ? cfirst[row + x1 + 1] : 0;
    }
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int j1 = r1[k];
        for (int jb = r0[k]; jb < j1; jb += kPmWin) {
            // kPmWin candidates' hi words in flight, then screened in order
            float4 hq[kPmWin];
#pragma unroll
            for (int u = 0; u < kPmWin; ++u) hq[u] = pos[min(jb + u, j1 - 1)];
#pragma unroll
            for (int u = 0; u < kPmWin; ++u) {
                const int j = jb + u;
                const float4 hj = hq[u];
                const float sx = hj.x - hi.x, sy = hj.y - hi.y, sz = hj.z - hi.z;
                if (j >= j1 || !(fmaf(sz, sz, fmaf(sy, sy, sx * sx)) < screen2) || j == i)
                    continue;
                const float4 lj = lo[j];
                const double ddx = xi - ((double)hj.x + (double)lj.x);
                const double ddy = yi - ((double)hj.y + (double)lj.y);
                const double ddz = zi - ((double)hj.z + (double)lj.z);
                const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                const int p = ti * tb.T + typ[j];
                if (!(r2 < tb.rint2[p])) continue;
                const double ir2 = 1.0 / r2;
                const double s2 = tb.sig2[p] * ir2, s6 = s2 * s2 * s2;
                const double glj = tb.e24[p] * (2.0 * s6 * s6 - s6) * ir2;
                const double gc = qi * (double)hj.w * ir2 * sqrt(ir2);
                const double gg = glj + gc;
                fx += gg * ddx;
                fy += gg * ddy;
                fz += gg * ddz;
            }
        }
    }
    F[i] = fx;
    F[(size_t)n + i] = fy;
    F[2 * (size_t)n + i] = fz;
}

// Steps (iii)-(vi) for one slot.
__global__ __launch_bounds__(kB) void k_pm_update(float4* pos, float4* lo,
                                                  const int* __restrict__ typ,
                                                  const int* __restrict__ oid,
                                                  const double* __restrict__ F, double* v, int n,
                                                  double dt, unsigned long long seed, PmTable tb,
                                                  ExtParams P, DevState* st) {
    const long long step = st->step;
    const double R = radius_at(P.R, st->t + dt);   // the new radius precedes the surface force
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    float4 h = pos[s], l = lo[s];
    const int ty = typ[s];
    const double x[3] = {(double)h.x + (double)l.x, (double)h.y + (double)l.y,
                         (double)h.z + (double)l.z};
    double Fe[3];
    upd::ext_force(x, ty, R, P, Fe);
    double u[3] = {0.0, 0.0, 0.0};
    if (tb.kick > 0.0) {
        double xi[3];
        upd::gauss3((uint32_t)oid[s], (unsigned long long)step, seed, xi);
        const double len = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        u[0] = xi[0] / len;
        u[1] = xi[1] / len;
        u[2] = xi[2] / len;
    }
    const double g = tb.gamma[ty], im = tb.inv_m[ty];
    bool ok = true;
    double xn[3];
    for (int c = 0; c < 3; ++c) {
        double vc = v[(size_t)c * n + s];
        vc = vc + dt * (F[(size_t)c * n + s] + Fe[c] - g * vc) * im;
        vc += tb.kick * u[c];
        const double d = dt * vc;
        if (!isfinite(d) || (P.jump_max > 0.0 && fabs(d) > P.jump_max)) ok = false;
        v[(size_t)c * n + s] = vc;
        xn[c] = x[c] + d;
    }
    if (!ok) atomicMin(&st->bad_step, (unsigned long long)step);
    h.x = (float)xn[0];
    h.y = (float)xn[1];
    h.z = (float)xn[2];
    l = make_float4((float)(xn[0] - (double)h.x), (float)(xn[1] - (double)h.y),
                    (float)(xn[2] - (double)h.z), 0.f);
    pos[s] = h;
    lo[s] = l;
}

// Slot-order [3][n] -> original order [n][3].
__global__ __launch_bounds__(kB) void k_pm_to_orig(const double* __restrict__ src,
                                                   const int* __restrict__ oid, int n,
                                                   double* __restrict__ dst) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const size_t o = 3 * (size_t)oid[s];
    dst[o] = src[s];
    dst[o + 1] = src[(size_t)n + s];
    dst[o + 2] = src[2 * (size_t)n + s];
}

// Original order [n][3] -> slot order [3][n].
__global__ __launch_bounds__(kB) void k_pm_from_orig(const double* __restrict__ src,
                                                     const int* __restrict__ oid, int n,
                                                     double* __restrict__ dst) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const size_t o = 3 * (size_t)oid[s];
    dst[s] = src[o];
    dst[(size_t)n + s] = src[o + 1];
    dst[2 * (size_t)n + s] = src[o + 2];
}

#define PM_LAUNCH(kernel, grid, block, ...)                                               \
    do {                                                                                  \
        hipLaunchKernelGGL(kernel, grid, block, 0, __VA_ARGS__);                          \
        HIP_TRY(hipGetLastError());                                                       \
    } while (0)

template <class T>
bool pm_alloc(T** p, size_t count) {
    return hipMalloc(p, sizeof(T) * (count > 0 ? count : 1)) == hipSuccess;
}

// Steps (i)-(ii) at the current positions: re-sort by cell (slot arrays and
// velocities swapped with their second buffers) and the pair forces into F.
ld_status pm_forces(ld_ctx* c, hipStream_t s) {
    PaperMode* m = c->pm;
    const int n = (int)c->n;
    PM_LAUNCH(k_pm_absmax, dim3(64), dim3(kB), s, c->pos, n, c->sb.bounds_part);
    const int nwg = radix_tiles(n);
    PM_LAUNCH(k_pm_keys, dim3(nwg), dim3(kB), s, c->pos, c->lo, n, c->sb.bounds_part,
              m->tab.rmax, m->grid, c->sb.keys, c->sb.hist, nwg);
    int bits = 1;
    while ((1 << bits) < kNC) ++bits;
    unsigned long long* keys = nullptr;    // the buffer the sorted keys end in
    HIP_TRY(launch_radix_by_high(c->sb.keys, reinterpret_cast<unsigned long long*>(c->sb.tmp4),
                                 n, bits, c->sb.hist, s, true, &keys));
    if (!c->pos2) {
        if (!(pm_alloc(&c->pos2, (size_t)n) && pm_alloc(&c->lo2, (size_t)n) &&
              pm_alloc(&c->typ2, (size_t)n) && pm_alloc(&c->oid2, (size_t)n)))
            return fail(LD_ENOMEM, "cannot allocate the second slot arrays");
    }
    HIP_TRY(permute_slots_into(keys, n, c->pos, c->lo, c->typ, c->oid, c->pos2, c->lo2,
                               c->typ2, c->oid2, s));
    PM_LAUNCH(k_pm_permute_v, dim3((n + kB - 1) / kB), dim3(kB), s, keys, n, m->v, m->v2);
    std::swap(c->pos, c->pos2);
    std::swap(c->lo, c->lo2);
    std::swap(c->typ, c->typ2);
    std::swap(c->oid, c->oid2);
    std::swap(m->v, m->v2);
    c->graph_len = -1;                 // a captured graph holds the old addresses
    PM_LAUNCH(k_pm_first, dim3((n + kB - 1) / kB), dim3(kB), s, keys, n, m->grid, m->cfirst);
    PM_LAUNCH(k_pm_forces, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, c->typ, keys,
              m->grid, m->cfirst, n, m->tab, m->F);
    c->steps_since_sort = 0;
    return LD_OK;
}

}  // namespace

void pm_free(ld_ctx* c) {
    if (!c->pm) return;
    PaperMode* m = c->pm;
    void* b[] = {m->v, m->v2, m->F, m->grid, m->cfirst};
    for (void* p : b)
        if (p) (void)hipFree(p);
    delete m;
    c->pm = nullptr;
}

ld_status pm_step(ld_ctx* c, double dt, hipStream_t s) {
    PaperMode* m = c->pm;
    const int n = (int)c->n;
    ld_status st = pm_forces(c, s);
    if (st != LD_OK) return st;
    PM_LAUNCH(k_pm_update, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, c->typ, c->oid,
              m->F, m->v, n, dt, (unsigned long long)c->seed, m->tab, c->ext, c->st);
    HIP_TRY(launch_advance(c->st, dt, s));
    return LD_OK;
}

}  // namespace ld

using namespace ld;
using namespace ld::host;

extern "C" {

ld_status ld_paper_enable(ld_ctx* c, const ld_paper_config* cfg) {
    g_err.clear();
    if (!c || !cfg) return fail(LD_EINVAL, "ctx and cfg are required");
    if (ff_active(c)) return fail(LD_ESTATE, "the learned far field is on (ld_ff_mode 0 first)");
    if (!(cfg->range_factor > 0.0) || !std::isfinite(cfg->range_factor))
        return fail(LD_EINVAL, "range_factor must be positive");
    if (!(cfg->kick >= 0.0) || !std::isfinite(cfg->kick))
        return fail(LD_EINVAL, "kick must be >= 0");
    const int T = c->p.n_types;
    for (int t = 0; t < T; ++t)
        if (!(cfg->inertial_mass[t] > 0.0) || !std::isfinite(cfg->inertial_mass[t]))
            return fail(LD_EINVAL, "inertial_mass[%d] must be positive", t);
    HIP_TRY(hipStreamSynchronize(c->stream));
    pm_free(c);
    PaperMode* m = new (std::nothrow) PaperMode();
    if (!m) return fail(LD_ENOMEM, "host allocation failed");
    m->cfg = *cfg;
    PmTable& tb = m->tab;
    tb.T = T;
    tb.rmax = 0.0;
    for (int a = 0; a < T; ++a)
        for (int b = 0; b < T; ++b) {
            const double sg = 0.5 * (c->p.sigma[a] + c->p.sigma[b]);
            const double e = c->p.use_eps_matrix ? c->p.eps_matrix[a * LD_MAX_TYPES + b]
                                                 : std::sqrt(c->p.eps[a] * c->p.eps[b]);
            const double rint = cfg->range_factor * sg;   // range_factor (r_a + r_b)
            tb.rint2[a * T + b] = rint * rint;
            tb.sig2[a * T + b] = sg * sg;
            tb.e24[a * T + b] = 24.0 * e;
            tb.rmax = std::max(tb.rmax, rint);
        }
    for (int t = 0; t < T; ++t) {
        tb.inv_m[t] = 1.0 / cfg->inertial_mass[t];
        tb.gamma[t] = c->p.gamma[t];
    }
    tb.kick = cfg->kick;
    const size_t N = (size_t)c->n;
    bool ok = pm_alloc(&m->v, 3 * N) && pm_alloc(&m->v2, 3 * N) && pm_alloc(&m->F, 3 * N) &&
              pm_alloc(&m->grid, 1) && pm_alloc(&m->cfirst, (size_t)kNC + 1);
    if (ok) {
        std::vector<double> zero(3 * N, 0.0);
        ok = hipMemcpy(m->v, zero.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice) ==
             hipSuccess;
    }
    c->pm = m;
    if (!ok) {
        pm_free(c);
        return fail(LD_ENOMEM, "cannot allocate the paper scheme's buffers");
    }
    return LD_OK;
}

ld_status ld_paper_disable(ld_ctx* c) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (c->pm) HIP_TRY(launch_boxes(c->pos, (int)c->n, c->box, c->stream));   // cell order
    HIP_TRY(hipStreamSynchronize(c->stream));
    pm_free(c);
    return LD_OK;
}

ld_status ld_paper_forces(ld_ctx* c, double* F) {
    g_err.clear();
    if (!c || !F) return fail(LD_EINVAL, "ctx and F are required");
    if (!c->pm) return fail(LD_ESTATE, "ld_paper_enable first");
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    ld_status st = pm_forces(c, s);
    if (st != LD_OK) return st;
    HIP_TRY(launch_boxes(c->pos, n, c->box, s));   // the slot order changed
    double* dF = c->work;
    PM_LAUNCH(k_pm_to_orig, dim3((n + kB - 1) / kB), dim3(kB), s, c->pm->F, c->oid, n, dF);
    HIP_TRY(copy_out(F, dF, sizeof(double) * 3 * (size_t)n, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LD_OK;
}

ld_status ld_paper_get_velocities(ld_ctx* c, double* v) {
    g_err.clear();
    if (!c || !v) return fail(LD_EINVAL, "ctx and v are required");
    if (!c->pm) return fail(LD_ESTATE, "ld_paper_enable first");
    const int n = (int)c->n;
    double* d = c->work;
    PM_LAUNCH(k_pm_to_orig, dim3((n + kB - 1) / kB), dim3(kB), c->stream, c->pm->v, c->oid, n, d);
    HIP_TRY(copy_out(v, d, sizeof(double) * 3 * (size_t)n, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LD_OK;
}

ld_status ld_paper_set_velocities(ld_ctx* c, const double* v) {
    g_err.clear();
    if (!c || !v) return fail(LD_EINVAL, "ctx and v are required");
    if (!c->pm) return fail(LD_ESTATE, "ld_paper_enable first");
    const size_t N = (size_t)c->n;
    std::vector<double> h;
    ld_status st = read_host(h, v, 3 * N, c->stream);
    if (st != LD_OK) return st;
    for (double x : h)
        if (!std::isfinite(x)) return fail(LD_EINVAL, "velocities must be finite");
    double* d = c->work;
    HIP_TRY(hipMemcpyAsync(d, h.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->stream));
    PM_LAUNCH(k_pm_from_orig, dim3(((int)N + kB - 1) / kB), dim3(kB), c->stream, d, c->oid, (int)N,
              c->pm->v);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LD_OK;
}

}  // extern "C"
