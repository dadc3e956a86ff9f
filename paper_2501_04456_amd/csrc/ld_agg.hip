// Aggregate statistics the paper extracts in post-processing (section 2.1:
// the number of sub-aggregates and aggregate statistics; section 1: N_surf,
// the number of NPs at the droplet surface; section 3.1: the surface
// fractal dimension, the fractal equation taken at dimension two on the
// sphere).
//
// Sub-aggregates are the connected components of the contact graph, a pair
// in contact when r < contact_factor sigma_ij.  Candidates come from a cell
// list (cells of side >= the largest contact distance, radix-sorted keys;
// the context's slot order is left alone) and are united lock-free: a union
// hangs the larger root under the smaller with a compare-and-swap, so parent
// indices only decrease, no cycle can form and every component ends with
// its smallest (cell-sorted) index as root.  The label reported is the
// smallest original index of the component.  Every wait-free retry loop is
// bounded; exceeding the bound raises an error flag instead of spinning.
#include <algorithm>
#include <climits>
#include <cmath>
#include <limits>
#include <vector>

#include "ld_host.h"

namespace ld {

using host::fail;

namespace {

constexpr int kB = 256;
constexpr int kAMaxCells = 64;
constexpr int kANC = kAMaxCells * kAMaxCells * kAMaxCells;
constexpr int kAMaxIter = 1 << 16;      // bound of every retry loop

struct AgGrid {
    double L, hc;
    int Gc, pad;
};

struct AgTable {
    int T;
    double rc2[kMaxTypes * kMaxTypes];  // (contact_factor sigma_ij)^2
    double half_sigma[kMaxTypes];
};

__global__ __launch_bounds__(kB) void k_ag_absmax(const float4* __restrict__ pos, int n,
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

__device__ __forceinline__ int ag_cell1(double x, double L, double h, int G) {
    int c = (int)floor((x + L) / h);
    return c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
}

// Grid (block 0 stores it), cell keys (cell << 32 | slot) from the FP64
// positions and the first radix pass's digit counts per radix tile.
__global__ __launch_bounds__(kB) void k_ag_keys(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo, int n,
                                                const float* __restrict__ part, double rc,
                                                AgGrid* g, unsigned long long* keys,
                                                unsigned* hist, int nwg) {
    __shared__ AgGrid sg;
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
            int G = (int)floor(2.0 * L / rc);
            G = G < 1 ? 1 : (G > kAMaxCells ? kAMaxCells : G);
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
            const int cx = ag_cell1((double)hp.x + (double)l.x, sg.L, sg.hc, G),
                      cy = ag_cell1((double)hp.y + (double)l.y, sg.L, sg.hc, G),
                      cz = ag_cell1((double)hp.z + (double)l.z, sg.L, sg.hc, G);
            const unsigned c = (unsigned)((cz * G + cy) * G + cx);
            keys[s] = ((unsigned long long)c << 32) | (unsigned)s;
            atomicAdd(&h[c & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)t * nwg + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(kB) void k_ag_fill(int* a, int m, int v) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < m) a[k] = v;
}

__global__ __launch_bounds__(kB) void k_ag_iota(int* a, int m) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < m) a[k] = k;
}

// First slot of every cell of the grid (G^3 cells, G from the device grid):
// the slots of cells a..b of the sorted keys are [cfirst[a], cfirst[b + 1]).
__global__ __launch_bounds__(kB) void k_ag_first(const unsigned long long* __restrict__ keys,
                                                 int n, const AgGrid* __restrict__ g,
                                                 int* cfirst) {
    const int G = g->Gc;
    fill_cell_first(keys, n, G * G * G, blockIdx.x * kB + threadIdx.x, cfirst);
}

// Squared FP32 screen for candidate pairs: the range widened by the worst
// rounding of an FP32 difference of hi words (coordinates within the cube
// half width L: hi rounding and the difference move each component by at
// most L 2^-22, the squared sum by a few ulp), so every pair the FP64 test
// keeps passes it.
__device__ __forceinline__ float ag_screen2(double range, double L) {
    const double w = range + L * 0x1p-20;
    return (float)(w * w * (1.0 + 0x1p-18));
}

// Root of a: a bounded walk up the parent links with path halving (a
// non-root's link is moved to its grandparent, still an ancestor with a
// smaller index, so no cycle can form and roots are never written here).
__device__ __forceinline__ int ag_find(int* parent, int a, int* err) {
    for (int it = 0; it < kAMaxIter; ++it) {
        const int p = __hip_atomic_load(&parent[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == a) return a;
        const int gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp != p)
            __hip_atomic_store(&parent[a], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a = gp;
    }
    atomicOr(err, 1);
    return a;
}

__device__ __forceinline__ void ag_unite(int* parent, int a, int b, int* err) {
    for (int it = 0; it < kAMaxIter; ++it) {
        a = ag_find(parent, a, err);
        b = ag_find(parent, b, err);
        if (a == b) return;
        if (a > b) {
            const int x = a;
            a = b;
            b = x;
        }
        if (atomicCAS(&parent[b], b, a) == b) return;   // b was still a root: hung under a
    }
    atomicOr(err, 1);
}

// Every contact pair (k, m), m > k in cell-sorted order, from the 27 cells
// around k's cell; with SURF only pairs of two surface NPs (surf[slot] != 0).
template <bool SURF>
__global__ __launch_bounds__(kB) void k_ag_hook(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo,
                                                const int* __restrict__ typ,
                                                const unsigned long long* __restrict__ keys,
                                                const AgGrid* __restrict__ g,
                                                const int* __restrict__ cfirst, int n,
                                                AgTable tb, const int* __restrict__ surf,
                                                int* parent, int* err) {
    // the oracle's operand order, no fused multiply-add: a pair within an ulp
    // of the contact distance lands on the same side in both
#pragma clang fp contract(off)
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= n) return;
    const unsigned long long key = keys[k];
    const int i = (int)(unsigned)key;
    if (SURF && !surf[i]) return;
    const float4 hi = pos[i], li = lo[i];
    const double xi = (double)hi.x + (double)li.x, yi = (double)hi.y + (double)li.y,
                 zi = (double)hi.z + (double)li.z;
    const int ti = typ[i];
    const int G = g->Gc;
    const int c = (int)(key >> 32);
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    for (int dz = -1; dz <= 1; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= G) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = cy + dy;
            if (y < 0 || y >= G) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = cx + dx;
                if (x < 0 || x >= G) continue;
                const int cc = (z * G + y) * G + x;
                const int m1 = cfirst[cc + 1];
                for (int m = max(cfirst[cc], k + 1); m < m1; ++m) {
                    const int j = (int)(unsigned)keys[m];
                    if (SURF && !surf[j]) continue;
                    const float4 hj = pos[j], lj = lo[j];
                    const double ddx = xi - ((double)hj.x + (double)lj.x);
                    const double ddy = yi - ((double)hj.y + (double)lj.y);
                    const double ddz = zi - ((double)hj.z + (double)lj.z);
                    if (ddx * ddx + ddy * ddy + ddz * ddz < tb.rc2[ti * tb.T + typ[j]])
                        ag_unite(parent, k, m, err);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kB) void k_ag_flatten(int* parent, int n, int* root, int* err) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < n) root[k] = ag_find(parent, k, err);
}

// Per root: the smallest original index (label) and the size.  Lanes of a
// wavefront with the same root combine first (one atomic per root per
// wavefront, so a giant component costs one atomic per wavefront).
// With a surface mask only surface NPs count.
__global__ __launch_bounds__(kB) void k_ag_roots(const int* __restrict__ root,
                                                 const unsigned long long* __restrict__ keys,
                                                 const int* __restrict__ oid,
                                                 const int* __restrict__ surf, int n, int* minoid,
                                                 int* size) {
    const int k = blockIdx.x * kB + threadIdx.x;
    const int slot = k < n ? (int)(unsigned)keys[k] : 0;
    const bool live = k < n && (!surf || surf[slot]);
    const int r = live ? root[k] : -1;
    const int o = live ? oid[slot] : INT_MAX;
    unsigned long long todo = __ballot(live);
    const int lane = threadIdx.x % 64;
    for (int it = 0; it < 64 && todo; ++it) {
        const int leader = __ffsll((long long)todo) - 1;
        const int rl = __shfl(r, leader);
        const unsigned long long same = __ballot(live && r == rl);
        int mo = (same >> lane) & 1ull ? o : INT_MAX;
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) mo = min(mo, __shfl_xor(mo, w));
        if (lane == leader) {
            atomicMin(&minoid[rl], mo);
            atomicAdd(&size[rl], __popcll(same));
        }
        todo &= ~same;
    }
}

// labels (original order) and per-workgroup partial statistics:
// [components, aggregates (size >= 2), largest size].
__global__ __launch_bounds__(kB) void k_ag_label(const int* __restrict__ root,
                                                 const unsigned long long* __restrict__ keys,
                                                 const int* __restrict__ oid,
                                                 const int* __restrict__ minoid,
                                                 const int* __restrict__ size, int n,
                                                 int* labels, long long* part) {
    __shared__ long long red[3][kB];
    const int k = blockIdx.x * kB + threadIdx.x;
    long long comp = 0, agg = 0, big = 0;
    if (k < n) {
        const int r = root[k];
        if (labels) labels[oid[(int)(unsigned)keys[k]]] = minoid[r];
        if (r == k) {
            comp = 1;
            agg = size[k] >= 2 ? 1 : 0;
            big = size[k];
        }
    }
    red[0][threadIdx.x] = comp;
    red[1][threadIdx.x] = agg;
    red[2][threadIdx.x] = big;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
            red[2][threadIdx.x] = max(red[2][threadIdx.x], red[2][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// N_surf partials per workgroup and type: | |x| - R | < sigma_t / 2.
__global__ __launch_bounds__(kB) void k_ag_surface(const float4* __restrict__ pos,
                                                   const float4* __restrict__ lo,
                                                   const int* __restrict__ typ, int n, double R,
                                                   AgTable tb, long long* part) {
#pragma clang fp contract(off)
    __shared__ int cnt[kMaxTypes];
    if (threadIdx.x < kMaxTypes) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s < n) {
        const float4 h = pos[s], l = lo[s];
        const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y,
                     z = (double)h.z + (double)l.z;
        const int t = typ[s];
        if (fabs(sqrt(x * x + y * y + z * z) - R) < tb.half_sigma[t]) atomicAdd(&cnt[t], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxTypes) part[(size_t)blockIdx.x * kMaxTypes + threadIdx.x] = cnt[threadIdx.x];
}

// Surface flag per slot: | |x| - R | < sigma_t / 2 (as k_ag_surface).
__global__ __launch_bounds__(kB) void k_sf_flag(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo,
                                                const int* __restrict__ typ, int n, double R,
                                                AgTable tb, int* surf) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y,
                 z = (double)h.z + (double)l.z;
    surf[s] = fabs(sqrt(x * x + y * y + z * z) - R) < tb.half_sigma[typ[s]] ? 1 : 0;
}

// Labels of surface NPs (-1 elsewhere) and per-workgroup partials:
// [surface components, the largest packed as size << 32 | (INT_MAX - label)],
// so the maximum is the largest size and, among equal sizes, the smallest
// label.
__global__ __launch_bounds__(kB) void k_sf_label(const int* __restrict__ root,
                                                 const unsigned long long* __restrict__ keys,
                                                 const int* __restrict__ oid,
                                                 const int* __restrict__ surf,
                                                 const int* __restrict__ minoid,
                                                 const int* __restrict__ size, int n,
                                                 int* labels, long long* part) {
    __shared__ long long red[2][kB];
    const int k = blockIdx.x * kB + threadIdx.x;
    long long comp = 0, best = -1;
    if (k < n) {
        const int slot = (int)(unsigned)keys[k];
        const int r = root[k];
        const bool on = surf[slot] != 0;
        if (labels) labels[oid[slot]] = on ? minoid[r] : -1;
        if (on && r == k) {
            comp = 1;
            best = ((long long)size[k] << 32) | (long long)(unsigned)(INT_MAX - minoid[k]);
        }
    }
    red[0][threadIdx.x] = comp;
    red[1][threadIdx.x] = best;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) part[2 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Direction of a surface NP (FP64 hi + lo) and whether it belongs to the
// component labelled `label`.
__device__ __forceinline__ bool sf_member(const float4* __restrict__ pos,
                                          const float4* __restrict__ lo,
                                          const unsigned long long* __restrict__ keys,
                                          const int* __restrict__ root,
                                          const int* __restrict__ surf,
                                          const int* __restrict__ minoid, int k, int label,
                                          double u[3], int* slot) {
    const int sl = (int)(unsigned)keys[k];
    *slot = sl;
    if (!surf[sl] || minoid[root[k]] != label) return false;
    const float4 h = pos[sl], l = lo[sl];
    const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y,
                 z = (double)h.z + (double)l.z;
    const double r = sqrt(x * x + y * y + z * z);
    u[0] = x / r;
    u[1] = y / r;
    u[2] = z / r;
    return true;
}

// Per-workgroup sums over the component's NPs of the unit direction and of
// sigma: dpart[4 * block + {0, 1, 2, 3}].
__global__ __launch_bounds__(kB) void k_sf_sums(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo,
                                                const int* __restrict__ typ,
                                                const unsigned long long* __restrict__ keys,
                                                const int* __restrict__ root,
                                                const int* __restrict__ surf,
                                                const int* __restrict__ minoid, int n, int label,
                                                AgTable tb, double* dpart) {
    __shared__ double red[4][kB];
    const int k = blockIdx.x * kB + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < n) {
        double u[3];
        int sl;
        if (sf_member(pos, lo, keys, root, surf, minoid, k, label, u, &sl)) {
            v[0] = u[0];
            v[1] = u[1];
            v[2] = u[2];
            v[3] = 2.0 * tb.half_sigma[typ[sl]];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) dpart[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Per-workgroup sums of the squared angle between each member's direction
// and u0 (from the sine and cosine, accurate for small angles).
__global__ __launch_bounds__(kB) void k_sf_theta(const float4* __restrict__ pos,
                                                 const float4* __restrict__ lo,
                                                 const unsigned long long* __restrict__ keys,
                                                 const int* __restrict__ root,
                                                 const int* __restrict__ surf,
                                                 const int* __restrict__ minoid, int n, int label,
                                                 double u0x, double u0y, double u0z,
                                                 double* dpart) {
    __shared__ double red[kB];
    const int k = blockIdx.x * kB + threadIdx.x;
    double v = 0.0;
    if (k < n) {
        double u[3];
        int sl;
        if (sf_member(pos, lo, keys, root, surf, minoid, k, label, u, &sl)) {
            const double cx = u[1] * u0z - u[2] * u0y, cy = u[2] * u0x - u[0] * u0z,
                         cz = u[0] * u0y - u[1] * u0x;
            const double th = atan2(sqrt(cx * cx + cy * cy + cz * cz),
                                    u[0] * u0x + u[1] * u0y + u[2] * u0z);
            v = th * th;
        }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dpart[blockIdx.x] = red[0];
}

constexpr int kRdfMaxBins = 4096;

__global__ __launch_bounds__(kB) void k_ag_zero64(unsigned long long* a, int m) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < m) a[k] = 0ull;
}

// Pair-distance histogram of Eq. (6) from the cell-sorted slots (cells of
// side >= r_max): every pair (k, m), m > k in sorted order, over the 27
// cells around k's.  The distance is formed exactly as in the all-pairs
// histogram (FP64 hi + lo, the same operand order, no contraction; the
// squares make it independent of the pair's orientation), so every pair
// falls in the same bin.
__global__ __launch_bounds__(kB) void k_ag_rdf(const float4* __restrict__ pos,
                                               const float4* __restrict__ lo,
                                               const unsigned long long* __restrict__ keys,
                                               const AgGrid* __restrict__ g,
                                               const int* __restrict__ cfirst, int n,
                                               double r_max, int n_bins, double dr,
                                               unsigned long long* counts) {
#pragma clang fp contract(off)
    __shared__ unsigned int hist[kRdfMaxBins];
    for (int b = threadIdx.x; b < n_bins; b += kB) hist[b] = 0u;
    __syncthreads();
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < n) {
        const unsigned long long key = keys[k];
        const int i = (int)(unsigned)key;
        const float4 hi = pos[i], li = lo[i];
        const double xi = (double)hi.x + (double)li.x, yi = (double)hi.y + (double)li.y,
                     zi = (double)hi.z + (double)li.z;
        const int G = g->Gc;
        const float screen2 = ag_screen2(r_max, g->L);
        const int c = (int)(key >> 32);
        const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < G - 1 ? cx + 1 : G - 1;
        for (int dz = -1; dz <= 1; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= G) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= G) continue;
                const int row = (z * G + y) * G;
                const int m1 = cfirst[row + x1 + 1];
                for (int m = max(cfirst[row + x0], k + 1); m < m1; ++m) {
                    const int j = (int)(unsigned)keys[m];
                    const float4 hj = pos[j], lj = lo[j];
                    const float sx = hj.x - hi.x, sy = hj.y - hi.y, sz = hj.z - hi.z;
                    if (!(fmaf(sz, sz, fmaf(sy, sy, sx * sx)) < screen2)) continue;
                    const double ex = xi - ((double)hj.x + (double)lj.x);
                    const double ey = yi - ((double)hj.y + (double)lj.y);
                    const double ez = zi - ((double)hj.z + (double)lj.z);
                    const double r = sqrt(ex * ex + ey * ey + ez * ez);
                    if (r < r_max) {
                        const int b = (int)floor(r / dr);
                        if (b >= 0 && b < n_bins) atomicAdd(&hist[b], 1u);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += kB)
        if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

#define AG_LAUNCH(kernel, grid, block, ...)                                               \
    do {                                                                                  \
        hipLaunchKernelGGL(kernel, grid, block, 0, __VA_ARGS__);                          \
        HIP_TRY(hipGetLastError());                                                       \
    } while (0)

// Scratch of the aggregate calls (allocated on first use, kept by the context).
struct AgBufs {
    int* cfirst;     // [kANC + 1] first slot of every cell
    int* parent;     // [n]
    int* root;       // [n]
    int* minoid;     // [n]
    int* size;       // [n]
    int* labels;     // [n]
    int* err;        // [1]
    long long* part; // [blocks * kMaxTypes]
    double* dpart;   // [blocks * 4]
    int* surf;       // [n] surface flag per slot
    AgGrid* grid;    // [1]
};

// Carve the scratch out of one allocation, every piece 256-byte aligned;
// with base == nullptr only the total size is computed.
size_t ag_layout(char* base, size_t n, AgBufs* b) {
    const size_t blocks = (n + kB - 1) / kB;
    size_t off = 0;
    auto take = [&](size_t nbytes) {
        char* q = base ? base + off : nullptr;
        off += (nbytes + 255) / 256 * 256;
        return q;
    };
    b->grid = reinterpret_cast<AgGrid*>(take(sizeof(AgGrid)));
    b->part = reinterpret_cast<long long*>(take(blocks * kMaxTypes * sizeof(long long)));
    b->dpart = reinterpret_cast<double*>(take(blocks * 4 * sizeof(double)));
    b->surf = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->cfirst = reinterpret_cast<int*>(take((kANC + 1) * sizeof(int)));
    b->parent = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->root = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->minoid = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->size = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->labels = reinterpret_cast<int*>(take(n * sizeof(int)));
    b->err = reinterpret_cast<int*>(take(sizeof(int)));
    return off;
}

ld_status ag_buffers(ld_ctx* c, AgBufs* b) {
    const size_t n = (size_t)c->n;
    if (!c->agg) {
        const size_t bytes = ag_layout(nullptr, n, b);
        if (hipMalloc(&c->agg, bytes) != hipSuccess) {
            c->agg = nullptr;
            return fail(LD_ENOMEM, "cannot allocate the aggregate scratch");
        }
    }
    ag_layout(reinterpret_cast<char*>(c->agg), n, b);
    return LD_OK;
}

// Contact distances (contact_factor sigma_ij)^2 and half diameters; returns
// the largest contact distance.
double ag_table(const ld_ctx* c, double contact_factor, AgTable* tb) {
    tb->T = c->p.n_types;
    double rc = 0.0;
    for (int a = 0; a < tb->T; ++a) {
        for (int q = 0; q < tb->T; ++q) {
            const double d = contact_factor * 0.5 * (c->p.sigma[a] + c->p.sigma[q]);
            tb->rc2[a * tb->T + q] = d * d;
            rc = std::max(rc, d);
        }
        tb->half_sigma[a] = 0.5 * c->p.sigma[a];
    }
    return rc;
}

#define AG_RUN(kernel, grid, ...)                                                         \
    do {                                                                                  \
        hipLaunchKernelGGL(kernel, grid, dim3(kB), 0, s, __VA_ARGS__);                    \
        const hipError_t e_ = hipGetLastError();                                          \
        if (e_ != hipSuccess) return e_;                                                  \
    } while (0)

// Cell sort for cells of side >= rc: grid, keys (cell << 32 | slot) sorted by
// cell, and every cell's first slot.  *keys_out: the sorted keys.
hipError_t ag_cells(ld_ctx* c, const AgBufs& b, double rc, unsigned long long** keys_out) {
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    const int blocks = (n + kB - 1) / kB;
    AG_RUN(k_ag_absmax, dim3(64), c->pos, n, c->sb.bounds_part);
    const int nwg = radix_tiles(n);
    AG_RUN(k_ag_keys, dim3(nwg), c->pos, c->lo, n, c->sb.bounds_part, rc, b.grid, c->sb.keys,
           c->sb.hist, nwg);
    int bits = 1;
    while ((1 << bits) < kANC) ++bits;
    unsigned long long* keys = nullptr;
    const hipError_t e = launch_radix_by_high(
        c->sb.keys, reinterpret_cast<unsigned long long*>(c->sb.tmp4), n, bits, c->sb.hist, s,
        true, &keys);
    if (e != hipSuccess) return e;
    AG_RUN(k_ag_first, dim3(blocks), keys, n, b.grid, b.cfirst);
    *keys_out = keys;
    return hipSuccess;
}

// Cell sort, lock-free union of the contact pairs (with surf: only pairs of
// two surface NPs), roots, and per root the size and smallest original index
// (counting only surface NPs with surf).  *keys_out: the cell-sorted keys.
hipError_t ag_union(ld_ctx* c, const AgBufs& b, const AgTable& tb, double rc, const int* surf,
                    unsigned long long** keys_out) {
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    const int blocks = (n + kB - 1) / kB;
    const dim3 gn(blocks);
    unsigned long long* keys = nullptr;
    const hipError_t ec = ag_cells(c, b, rc, &keys);
    if (ec != hipSuccess) return ec;
    AG_RUN(k_ag_iota, gn, b.parent, n);
    AG_RUN(k_ag_fill, dim3(1), b.err, 1, 0);
    if (surf)
        AG_RUN(k_ag_hook<true>, gn, c->pos, c->lo, c->typ, keys, b.grid, b.cfirst, n, tb, surf,
               b.parent, b.err);
    else
        AG_RUN(k_ag_hook<false>, gn, c->pos, c->lo, c->typ, keys, b.grid, b.cfirst, n, tb,
               nullptr, b.parent, b.err);
    AG_RUN(k_ag_flatten, gn, b.parent, n, b.root, b.err);
    AG_RUN(k_ag_fill, gn, b.minoid, n, INT_MAX);
    AG_RUN(k_ag_fill, gn, b.size, n, 0);
    AG_RUN(k_ag_roots, gn, b.root, keys, c->oid, surf, n, b.minoid, b.size);
#undef AG_RUN
    *keys_out = keys;
    return hipSuccess;
}

}  // namespace

void ag_free(ld_ctx* c) {
    if (c->agg) (void)hipFree(c->agg);
    c->agg = nullptr;
}

// Eq. (6) pair counts into counts[n_bins] (device) through the cell sort,
// when the grid of cells of side >= r_max has at least 3 cells per axis;
// *used = false leaves the counts to the all-pairs histogram.  The slot
// order is not changed.
ld_status ag_rdf_pairs(ld_ctx* c, double r_max, int n_bins, unsigned long long* counts,
                       bool* used) {
    *used = false;
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    // the grid the key kernel will derive (same partial maxima, same rule)
    AG_LAUNCH(k_ag_absmax, dim3(64), dim3(kB), s, c->pos, n, c->sb.bounds_part);
    float part[64];
    HIP_TRY(hipMemcpyAsync(part, c->sb.bounds_part, sizeof part, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float m = 0.f;
    for (float v : part) m = std::max(m, v);
    m = std::max(m, 1e-3f);
    const double L = (double)(m * 1.0009765625f);
    if ((int)std::floor(2.0 * L / r_max) < 3) return LD_OK;
    AgBufs b{};
    ld_status st = ag_buffers(c, &b);
    if (st != LD_OK) return st;
    unsigned long long* keys = nullptr;
    HIP_TRY(ag_cells(c, b, r_max, &keys));
    const int blocks = (n + kB - 1) / kB;
    AG_LAUNCH(k_ag_zero64, dim3((n_bins + kB - 1) / kB), dim3(kB), s, counts, n_bins);
    AG_LAUNCH(k_ag_rdf, dim3(blocks), dim3(kB), s, c->pos, c->lo, keys, b.grid, b.cfirst, n,
              r_max, n_bins, r_max / n_bins, counts);
    *used = true;
    return LD_OK;
}

}  // namespace ld

using namespace ld;
using namespace ld::host;

extern "C" {

ld_status ld_aggregates(ld_ctx* c, double contact_factor, int64_t stats[3], int32_t* labels) {
    g_err.clear();
    if (!c || !stats) return fail(LD_EINVAL, "ctx and stats are required");
    if (!(contact_factor > 0.0) || !std::isfinite(contact_factor))
        return fail(LD_EINVAL, "contact_factor must be positive");
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    AgBufs b{};
    ld_status st = ag_buffers(c, &b);
    if (st != LD_OK) return st;
    AgTable tb{};
    const double rc = ag_table(c, contact_factor, &tb);
    unsigned long long* keys = nullptr;
    HIP_TRY(ag_union(c, b, tb, rc, nullptr, &keys));
    const int blocks = (n + kB - 1) / kB;
    AG_LAUNCH(k_ag_label, dim3(blocks), dim3(kB), s, b.root, keys, c->oid, b.minoid, b.size, n,
              labels ? b.labels : nullptr, b.part);
    std::vector<long long> part(3 * (size_t)blocks);
    int err = 0;
    HIP_TRY(hipMemcpyAsync(part.data(), b.part, sizeof(long long) * part.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, b.err, sizeof(int), hipMemcpyDeviceToHost, s));
    if (labels) HIP_TRY(copy_out(labels, b.labels, sizeof(int32_t) * (size_t)n, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) return fail(LD_EHIP, "contact-graph union did not settle within its bound");
    long long comp = 0, agg = 0, big = 0;
    for (int k = 0; k < blocks; ++k) {
        comp += part[3 * (size_t)k];
        agg += part[3 * (size_t)k + 1];
        big = std::max(big, part[3 * (size_t)k + 2]);
    }
    stats[0] = comp;
    stats[1] = agg;
    stats[2] = big;
    return LD_OK;
}

ld_status ld_surface_fractal(ld_ctx* c, double R, double contact_factor, double k_f, double d,
                             int64_t stats[3], double out[3], int32_t* labels) {
    g_err.clear();
    if (!c || !stats || !out) return fail(LD_EINVAL, "ctx, stats and out are required");
    if (!(contact_factor > 0.0) || !std::isfinite(contact_factor))
        return fail(LD_EINVAL, "contact_factor must be positive");
    if (!(k_f > 0.0) || !std::isfinite(k_f)) return fail(LD_EINVAL, "k_f must be positive");
    if (std::isnan(d)) return fail(LD_EINVAL, "d is NaN");
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    if (!(R >= 0.0)) {      // negative: the droplet's radius at the current time
        DevState ds;
        HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        R = radius_at(c->R, ds.t);
    }
    AgBufs b{};
    ld_status st = ag_buffers(c, &b);
    if (st != LD_OK) return st;
    AgTable tb{};
    const double rc = ag_table(c, contact_factor, &tb);
    const int blocks = (n + kB - 1) / kB;
    AG_LAUNCH(k_sf_flag, dim3(blocks), dim3(kB), s, c->pos, c->lo, c->typ, n, R, tb, b.surf);
    unsigned long long* keys = nullptr;
    HIP_TRY(ag_union(c, b, tb, rc, b.surf, &keys));
    AG_LAUNCH(k_sf_label, dim3(blocks), dim3(kB), s, b.root, keys, c->oid, b.surf, b.minoid,
              b.size, n, labels ? b.labels : nullptr, b.part);
    std::vector<long long> part(2 * (size_t)blocks);
    int err = 0;
    HIP_TRY(hipMemcpyAsync(part.data(), b.part, sizeof(long long) * part.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, b.err, sizeof(int), hipMemcpyDeviceToHost, s));
    if (labels) HIP_TRY(copy_out(labels, b.labels, sizeof(int32_t) * (size_t)n, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) return fail(LD_EHIP, "contact-graph union did not settle within its bound");
    long long comp = 0, best = -1;
    for (int k = 0; k < blocks; ++k) {
        comp += part[2 * (size_t)k];
        best = std::max(best, part[2 * (size_t)k + 1]);
    }
    const double nan = std::numeric_limits<double>::quiet_NaN();
    out[0] = out[1] = out[2] = nan;
    stats[0] = comp;
    if (comp == 0) {
        stats[1] = 0;
        stats[2] = -1;
        return LD_OK;
    }
    const long long m = best >> 32;
    const int label = INT_MAX - (int)(unsigned)(best & 0xffffffffLL);
    stats[1] = m;
    stats[2] = label;
    // the component's mean direction and mean diameter (partials summed in
    // workgroup order, so the result does not depend on timing)
    std::vector<double> dp(4 * (size_t)blocks);
    AG_LAUNCH(k_sf_sums, dim3(blocks), dim3(kB), s, c->pos, c->lo, c->typ, keys, b.root, b.surf,
              b.minoid, n, label, tb, b.dpart);
    HIP_TRY(hipMemcpyAsync(dp.data(), b.dpart, sizeof(double) * dp.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double su[3] = {0.0, 0.0, 0.0}, ssig = 0.0;
    for (int k = 0; k < blocks; ++k) {
        su[0] += dp[4 * (size_t)k];
        su[1] += dp[4 * (size_t)k + 1];
        su[2] += dp[4 * (size_t)k + 2];
        ssig += dp[4 * (size_t)k + 3];
    }
    const double nu = std::sqrt(su[0] * su[0] + su[1] * su[1] + su[2] * su[2]);
    if (!(nu > 0.0)) return LD_OK;
    const double dm = d > 0.0 ? d : ssig / (double)m;
    AG_LAUNCH(k_sf_theta, dim3(blocks), dim3(kB), s, c->pos, c->lo, keys, b.root, b.surf,
              b.minoid, n, label, su[0] / nu, su[1] / nu, su[2] / nu, b.dpart);
    HIP_TRY(hipMemcpyAsync(dp.data(), b.dpart, sizeof(double) * blocks, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double s2 = 0.0;
    for (int k = 0; k < blocks; ++k) s2 += dp[(size_t)k];
    const double Rg = R * std::sqrt(s2 / (double)m);
    out[0] = Rg;
    out[1] = dm;
    if (m >= 2) out[2] = std::log((double)m / k_f) / std::log(2.0 * Rg / dm);
    return LD_OK;
}

ld_status ld_surface_count(ld_ctx* c, double R, int64_t* counts) {
    g_err.clear();
    if (!c || !counts) return fail(LD_EINVAL, "ctx and counts are required");
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    if (!(R >= 0.0)) {      // negative: the droplet's radius at the current time
        DevState ds;
        HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        R = radius_at(c->R, ds.t);
    }
    AgBufs b{};
    ld_status st = ag_buffers(c, &b);
    if (st != LD_OK) return st;
    AgTable tb{};
    tb.T = c->p.n_types;
    for (int a = 0; a < tb.T; ++a) tb.half_sigma[a] = 0.5 * c->p.sigma[a];
    const int blocks = (n + kB - 1) / kB;
    AG_LAUNCH(k_ag_surface, dim3(blocks), dim3(kB), s, c->pos, c->lo, c->typ, n, R, tb, b.part);
    std::vector<long long> part((size_t)blocks * kMaxTypes);
    HIP_TRY(hipMemcpyAsync(part.data(), b.part, sizeof(long long) * part.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t < tb.T; ++t) {
        long long v = 0;
        for (int k = 0; k < blocks; ++k) v += part[(size_t)k * kMaxTypes + t];
        counts[t] = v;
    }
    return LD_OK;
}

}  // extern "C"
