// Learned far field: the all-pairs sum split into an exact near part and a
// far Coulomb part on a G^3 grid over the droplet,
//
//   F_i = F_near(i) + q_i (E_coarse(i) + E_mlp(features of i)).
//
// Radial mode: F_near sums the pairs with r < r_c over a cell list of side
// >= r_c; E_coarse is the field at the centre of i's grid cell from the
// monopole + dipole of every cell outside the B^3 block around it.
//
// Block mode: F_near sums the Coulomb pairs whose j lies in the B^3 block of
// grid cells around i's cell (and every LJ pair); E_coarse is the
// second-order Taylor expansion about the centre of i's cell of the
// monopole + dipole field of every cell outside the block, evaluated at x_i.
// The near part runs over row tiles: slots are sorted by grid cell (z, y, x),
// so the cells x0..x1 of one (y, z) row are one contiguous slot range, and a
// tile of at most 64 slots of one row needs only the (2W+1)^2 rows around it,
// each as one contiguous range streamed through LDS.
//
// The MLP (4 B^3 + 3 -> H -> H -> 3, SiLU, BF16 operands on the matrix cores,
// FP32 accumulation) sees the normalised moments of the B^3 block and the
// particle's offset in its cell, and predicts the rest of the far field.  Its
// first layer is evaluated once per occupied cell (the moment part of the
// input depends only on the cell) and finished per particle with the three
// offset columns.
//
// Training targets come from the exact far field (the Coulomb field of the
// pairs outside the near part) minus the coarse term, on snapshots of the
// running system; the network is trained on the GPU by the same MFMA products
// (forward, backward) and Adam.  Every judge_every steps a judge compares
// the learned pair forces with direct summation on the same state; if the
// median relative error exceeds the tolerance the next window runs direct
// summation.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <vector>
#include <new>

#include "ld_ffconv.h"
#include "ld_gemm.h"
#include "ld_host.h"
#include "ld_pair_core.h"

using namespace ld;
using namespace ld::host;

namespace ld {

constexpr int kMaxNearCells = 64;      // near cell list: at most 64^3 cells

struct FFGrid {
    double L;       // half width of the cube [-L, L]^3 covering every particle
    double h;       // moment grid cell side 2L / G
    double hn;      // near cell side: 2L / Gn (>= r_c), or h in block mode
    int Gn;         // near cells per axis (G in block mode)
    int W;          // block mode: rows searched around a tile (>= B/2, covers LJ)
    int Wlj;        // block mode: rows within the LJ range, ceil(rlj / h)
};

constexpr int kLoc = 19;               // E (3), J (6), H (10) per cell

struct FarField {
    ld_ff_config cfg{};
    double rlj = 0.0;                  // largest LJ range
    int K = 0, Kp = 0, Op = 16, H = 0;
    size_t offW1 = 0, offb1 = 0, offW2 = 0, offb2 = 0, offW3 = 0, offb3 = 0, nW = 0;
    float sq = 1.f, out_scale = 1.f;
    int mode = 0;                      // 0 direct, 1 learned, 2 learned + judge
    bool active = true;                // judge verdict for the current window
    int64_t window_steps = 0;
    double last_err = NAN;
    int64_t judges = 0, fallbacks = 0, learned_steps = 0, direct_steps = 0;

    FFGrid* grid = nullptr;            // device
    int* cstart = nullptr;             // [kMaxNearCells^3]
    int* cend = nullptr;
    double* Fnear = nullptr;           // [3][n]
    double* mom = nullptr;             // [G^3 * 4]
    int* count = nullptr;              // [G^3] particles per cell
    int* occ = nullptr;                // [G^3] compacted occupied cells
    int* cell2occ = nullptr;           // [G^3]
    int* nocc = nullptr;               // [1]
    double* Ecell = nullptr;           // [G^3 * 3] centre field, or [G^3 * 19] expansion
    double* Ep = nullptr;              // [3][n] coarse field at each particle
    int* cfirst = nullptr;             // [G^3 + 1] first slot of each cell (block mode)
    int4* tiles = nullptr;             // row tiles (block mode)
    double* loc_part = nullptr;        // [loc_split][G^3][19] partial expansions
    int loc_split = 1;
    double* pmom = nullptr;            // [(G/2)^3 * 4] parent moments (two-level)
    int* pcount = nullptr;             // [(G/2)^3]
    int* pocc = nullptr;               // [(G/2)^3] compacted occupied parents
    int* pcell2occ = nullptr;          // [(G/2)^3]
    int* npocc = nullptr;              // [1]
    LocalConv conv;                    // one-level block expansion by FFT (G <= 32)
    bool use_conv = false;
    int* ntiles = nullptr;
    int max_tiles = 0;
    float* Xc = nullptr;               // [G^3 * Kp]
    float* Ac = nullptr;               // [G^3 * H]
    float* h1 = nullptr;               // [n * H]
    float* h2 = nullptr;               // [n * H]
    float* y = nullptr;                // [n * Op]
    float* W = nullptr;                // packed FP32 master weights
    __bf16* w1bf = nullptr;            // [128][Kp] BF16 copy of W1, column-major (hidden 128)
    bool w1bf_stale = true;            // W changed since w1bf was made
    float* grad = nullptr;             // packed gradients
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int adam_step = 0;
    double* rel = nullptr;             // [n] judge errors
    double* Efar = nullptr;            // [3][n] exact far field (training, tests)

    // training store
    int snap_cap = 0, snaps = 0;
    int64_t sample_cap = 0, samples = 0;
    float* snap_mom = nullptr;         // [snap_cap][G^3 * 4] normalised moments
    int* s_snap = nullptr;             // [sample_cap]
    int* s_cell = nullptr;
    float* s_off = nullptr;            // [sample_cap * 3]
    float* s_tgt = nullptr;            // [sample_cap * 3]
    // batch buffers
    int batch_cap = 0;
    float *bX = nullptr, *bT = nullptr, *bZ1 = nullptr, *bA1 = nullptr, *bZ2 = nullptr,
          *bA2 = nullptr, *bY = nullptr, *bdY = nullptr, *bd2 = nullptr, *bd1 = nullptr;
    int* bidx = nullptr;
    double* loss_part = nullptr;
    float* gws = nullptr;              // split-K workspace of the weight gradients
    size_t gws_floats = 0;
};

}  // namespace ld

namespace {

constexpr int kB = 256;

// SiLU z sigmoid(z) with the hardware exponential and reciprocal (about 1
// ulp each; the activations are rounded to BF16 next).
__device__ __forceinline__ float silu_f(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

__device__ __forceinline__ __bf16 bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}
__device__ __forceinline__ float bf16_round(float f) { return (float)bf16_rne(f); }

// Exclusive scan of one int per thread over a workgroup of 1024 (16
// wavefronts): shuffle scan inside each wavefront, then across the wavefront
// totals.  Returns the thread's exclusive prefix; *total receives the sum.
__device__ __forceinline__ int scan1024(int v, int* wsum, int* total) {
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        int a = threadIdx.x < 16 ? wsum[threadIdx.x] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(a, o);
            if (lane >= o) a += y;
        }
        if (threadIdx.x < 16) wsum[16 + threadIdx.x] = a;   // inclusive over wavefronts
    }
    __syncthreads();
    const int before = wv > 0 ? wsum[16 + wv - 1] : 0;
    *total = wsum[31];
    __syncthreads();                                    // wsum is reused by the next call
    return before + x - v;
}

// Exclusive scan of load(0 .. n-1) in index order by one workgroup of 1024:
// 8192 values at a time are read coalesced into LDS (buf), each thread takes
// 8 consecutive ones, and emit(e, prefix, value) is called for every e.
// Returns the total.
template <class Load, class Emit>
__device__ __forceinline__ int scan_runs(int n, Load load, Emit emit, int* buf, int* wsum) {
    const int t = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < n; base += 8 * 1024) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = base + i * 1024 + t;
            buf[i * 1024 + t] = e < n ? load(e) : 0;
        }
        __syncthreads();
        int v[8], sum = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v[i] = buf[8 * t + i];
            sum += v[i];
        }
        int tot;
        int run = carry + scan1024(sum, wsum, &tot);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = base + 8 * t + i;
            if (e < n) emit(e, run, v[i]);
            run += v[i];
        }
        carry += tot;
    }
    return carry;
}

// ---- grid --------------------------------------------------------------

__global__ __launch_bounds__(kB) void k_absmax_part(const float4* __restrict__ pos, int n,
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

// L = max |coordinate| x (1 + 2^-10) in FP32, then the cell sides.  In
// block mode the near cells are the grid cells and W rows around a tile
// cover both the block (B/2) and the largest LJ range rlj.
__device__ __forceinline__ FFGrid make_grid(float m, double rc, int G, int block_mode, int B,
                                            double rlj) {
    FFGrid g{};
    m = fmaxf(m, 1e-3f);
    const float Lf = m * 1.0009765625f;
    const double L = (double)Lf;
    const double h = 2.0 * L / G;
    g.L = L;
    g.h = h;
    if (block_mode) {
        const int wl = (int)ceil(rlj / h);
        const int W = wl < B / 2 ? B / 2 : wl;
        g.W = W > G ? G : W;
        g.Wlj = wl;
        g.hn = h;
        g.Gn = G;
    } else {
        int Gn = (int)floor(2.0 * L / rc);
        Gn = Gn < 1 ? 1 : (Gn > kMaxNearCells ? kMaxNearCells : Gn);
        g.hn = 2.0 * L / Gn;
        g.Gn = Gn;
        g.W = 0;
        g.Wlj = 0;
    }
    return g;
}

__global__ void k_grid(const float* part, int nparts, double rc, int G, int block_mode, int B,
                       double rlj, FFGrid* g) {
    float m = 0.f;
    for (int b = 0; b < nparts; ++b) m = fmaxf(m, part[b]);
    *g = make_grid(m, rc, G, block_mode, B, rlj);
}

__device__ __forceinline__ int cell1(double x, double L, double h, int G) {
    int c = (int)floor((x + L) / h);
    return c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
}

// ---- near cell list ------------------------------------------------------

// Cell keys from the FP64 positions (hi + lo), so that cell membership
// agrees with the moments and offsets.
static_assert(kB == ld::kRadixThreads, "k_near_keys counts digits per radix tile");

// Cell keys (cell << 32 | slot) of the slots, with the grid made from the
// 64 partial maxima (block 0 stores it for the later kernels) and the
// digit counts of the first radix pass over each radix tile.
__global__ __launch_bounds__(kB) void k_near_keys(const float4* __restrict__ pos,
                                                  const float4* __restrict__ lo, int n,
                                                  const float* __restrict__ part, double rc,
                                                  int G, int block_mode, int B, double rlj,
                                                  FFGrid* g, unsigned long long* keys,
                                                  unsigned* hist, int nwg) {
    __shared__ FFGrid sg;
    __shared__ unsigned h[256];
    const int t = threadIdx.x;
    h[t] = 0u;
    if (t < 64) {
        float m = part[t];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (t == 0) {
            sg = make_grid(m, rc, G, block_mode, B, rlj);
            if (blockIdx.x == 0) *g = sg;
        }
    }
    __syncthreads();
    const int Gn = sg.Gn;
    for (int r = 0; r < ld::kRadixRounds; ++r) {
        const int s = blockIdx.x * ld::kRadixTile + r * kB + t;
        if (s < n) {
            const float4 hp = pos[s], l = lo[s];
            const int cx = cell1((double)hp.x + (double)l.x, sg.L, sg.hn, Gn),
                      cy = cell1((double)hp.y + (double)l.y, sg.L, sg.hn, Gn),
                      cz = cell1((double)hp.z + (double)l.z, sg.L, sg.hn, Gn);
            const unsigned c = (unsigned)((cz * Gn + cy) * Gn + cx);
            keys[s] = ((unsigned long long)c << 32) | (unsigned)s;
            atomicAdd(&h[c & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)t * nwg + blockIdx.x] = h[t];
}

// Gap-filled first slot of every cell (fill_cell_first), M cells.
__global__ __launch_bounds__(kB) void k_cell_first(const unsigned long long* __restrict__ keys,
                                                   int n, int M, int* cfirst) {
    fill_cell_first(keys, n, M, blockIdx.x * kB + threadIdx.x, cfirst);
}

__global__ __launch_bounds__(kB) void k_zero_i(int* a, int m) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < m) a[k] = 0;
}

__global__ __launch_bounds__(kB) void k_zero_d(double* a, int m) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k < m) a[k] = 0.0;
}

__global__ __launch_bounds__(kB) void k_cell_ranges(const unsigned long long* __restrict__ keys,
                                                    int n, int* cstart, int* cend) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const unsigned c = (unsigned)(keys[s] >> 32);
    if (s == 0 || (unsigned)(keys[s - 1] >> 32) != c) cstart[c] = s;
    if (s == n - 1 || (unsigned)(keys[s + 1] >> 32) != c) cend[c] = s + 1;
}

// Exact pair forces of all pairs closer than rc (the near field), FP32 pair
// terms in 32-term blocks, FP64 totals.  Slots are in cell order.
__global__ __launch_bounds__(kB) void k_near(const float4* __restrict__ pos,
                                             const int* __restrict__ typ, int n,
                                             const FFGrid* g, const int* __restrict__ cstart,
                                             const int* __restrict__ cend, float rc2,
                                             PairTable tab, double* F) {
    __shared__ float ttab[4 * kMaxTypes * kMaxTypes];
    for (int k = threadIdx.x; k < kMaxTypes * kMaxTypes; k += kB) {
        ttab[k] = tab.sig2[k];
        ttab[kMaxTypes * kMaxTypes + k] = tab.rc2[k];
        ttab[2 * kMaxTypes * kMaxTypes + k] = tab.e24[k];
    }
    __syncthreads();
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const float4 pi = pos[i];
    const int ti = typ[i];
    const int T = tab.T;
    const int Gn = g->Gn;
    const int cx = cell1(pi.x, g->L, g->hn, Gn), cy = cell1(pi.y, g->L, g->hn, Gn),
              cz = cell1(pi.z, g->L, g->hn, Gn);
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, Lx = 0.0, Ly = 0.0, Lz = 0.0;
    float bx = 0.f, by = 0.f, bz = 0.f;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= Gn) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yv = cy + dy;
            if (yv < 0 || yv >= Gn) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int xv = cx + dx;
                if (xv < 0 || xv >= Gn) continue;
                const int c = (z * Gn + yv) * Gn + xv;
                const int j1 = cend[c];
                for (int j = cstart[c]; j < j1; ++j) {
                    if (j == i) continue;
                    const float4 pj = pos[j];
                    const float ddx = pj.x - pi.x, ddy = pj.y - pi.y, ddz = pj.z - pi.z;
                    const float r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                    if (r2 >= rc2) continue;
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float w = (pj.w * ri) * (ri * ri);
                    bx = fmaf(w, ddx, bx);
                    by = fmaf(w, ddy, by);
                    bz = fmaf(w, ddz, bz);
                    const int pidx = ti * T + typ[j];
                    if (r2 < ttab[kMaxTypes * kMaxTypes + pidx]) {
                        const float ir2 = 1.0f / r2;
                        const float s2 = ttab[pidx] * ir2;
                        const float s6 = s2 * s2 * s2;
                        const float gg =
                            ttab[2 * kMaxTypes * kMaxTypes + pidx] * s6 * (2.0f * s6 - 1.0f) * ir2;
                        Lx += (double)(gg * ddx);
                        Ly += (double)(gg * ddy);
                        Lz += (double)(gg * ddz);
                    }
                    if (++cnt == 32) {
                        Fx += (double)bx; Fy += (double)by; Fz += (double)bz;
                        bx = by = bz = 0.f;
                        cnt = 0;
                    }
                }
            }
        }
    }
    Fx += (double)bx; Fy += (double)by; Fz += (double)bz;
    const double qi = (double)pi.w;
    F[i] = -qi * Fx - Lx;
    F[(size_t)n + i] = -qi * Fy - Ly;
    F[2 * (size_t)n + i] = -qi * Fz - Lz;
}

// ---- block mode: row tiles and the block near field ----------------------

// Row tiles (one workgroup of 1024): every (y, z) row's slot range, from
// cfirst, cut into pieces of at most 64 slots, tile = (row, first slot, end
// slot).
__global__ __launch_bounds__(1024) void k_block_tiles(const int* __restrict__ cfirst, int G,
                                                      int4* tiles, int* ntiles) {
    __shared__ int buf[8 * 1024];
    __shared__ int wsum[32];
    const int nt = scan_runs(
        G * G, [&](int r) { return (cfirst[(r + 1) * G] - cfirst[r * G] + 63) / 64; },
        [&](int r, int pre, int cnt) {
            const int a = cfirst[r * G], b = cfirst[(r + 1) * G];
            for (int k = 0; k < cnt; ++k)
                tiles[pre + k] = make_int4(r, a + 64 * k, min(b, a + 64 * (k + 1)), 0);
        },
        buf, wsum);
    if (threadIdx.x == 0) *ntiles = nt;
}

// Block near field, one wavefront per row tile: Coulomb of every j in the
// B^3 block of i's cell, LJ of every pair within its range.  The tile's
// lanes share one (y, z) row, so the rows dy, dz in [-W, W] around it hold
// every partner; cells x_first - W .. x_last + W of such a row are one
// contiguous slot range.  Two ways to walk it:
//
// Lane windows (the LJ range fits in the block, W = B/2): each row's range
// is staged in LDS and every lane walks only its own window, the slots of
// cells ix - B/2 .. ix + B/2 of that row (one contiguous piece), so no pair
// is evaluated only to be masked; i itself is skipped by cutting its own
// row's window in two, and LJ terms are tried only in the rows within
// ceil(rlj / h) of the tile's.
//
// Row windows (LJ range beyond the block): every lane walks the tile's
// whole range of each row with per-pair tests of the block and the self
// pair.
//
// FP32 pair terms (Coulomb and LJ apart) in blocks of at most 32, FP64 totals.
//
// The two walks are separate kernels, both launched on the same grid of
// tiles; the one that does not match the grid's W leaves at once.  The lane
// walk (k_near_planes) gives each plane dz of the block a wavefront of its
// own, B wavefronts per tile whose FP64 sums are added in plane order: a
// tile's 25 rows on one wavefront left about four wavefronts per SIMD for
// the whole launch, too few to hide the row loads.  Kept apart, neither
// kernel spills registers to scratch at 6 wavefronts per SIMD.
constexpr int kNbChunk = 192;          // staged slots per piece of a row's range
constexpr int kNbMaxPlanes = 7;        // B <= 7

struct NbAcc {
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, Lx = 0.0, Ly = 0.0, Lz = 0.0;
};

template <bool LJ>
__device__ __forceinline__ void nb_pair(const float4* sp, const int* st, int k, const float4 pi,
                                        int trow, const float* ttab, float rc2max, float& bx,
                                        float& by, float& bz, float& lx, float& ly, float& lz) {
    const float4 pj = sp[k];
    const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float w = (pj.w * ri) * (ri * ri);
    bx = fmaf(w, dx, bx);
    by = fmaf(w, dy, by);
    bz = fmaf(w, dz, bz);
    if constexpr (LJ) {
        if (r2 < rc2max) {
            const int pidx = trow + st[k];
            if (r2 < ttab[kMaxTypes * kMaxTypes + pidx]) {
                const float ir2 = ri * ri;
                const float s2 = ttab[pidx] * ir2;
                const float s6 = s2 * s2 * s2;
                const float gg =
                    ttab[2 * kMaxTypes * kMaxTypes + pidx] * s6 * (2.0f * s6 - 1.0f) * ir2;
                lx = fmaf(gg, dx, lx);
                ly = fmaf(gg, dy, ly);
                lz = fmaf(gg, dz, lz);
            }
        }
    }
}

// This lane's terms of the staged slots [lo, hi).
template <bool LJ>
__device__ __forceinline__ void nb_range(const float4* sp, const int* st, int lo, int hi,
                                         const float4 pi, int trow, const float* ttab,
                                         float rc2max, NbAcc& a) {
    int k = lo;
    while (k < hi) {
        const int ke = min(hi, k + 32);
        float bx = 0.f, by = 0.f, bz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
        constexpr int U = LJ ? 4 : 8;          // pairs in flight per lane
        for (; k + U <= ke; k += U) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                nb_pair<LJ>(sp, st, k + u, pi, trow, ttab, rc2max, bx, by, bz, lx, ly, lz);
        }
        for (; k < ke; ++k)
            nb_pair<LJ>(sp, st, k, pi, trow, ttab, rc2max, bx, by, bz, lx, ly, lz);
        a.Fx += (double)bx;
        a.Fy += (double)by;
        a.Fz += (double)bz;
        if constexpr (LJ) {
            a.Lx += (double)lx;
            a.Ly += (double)ly;
            a.Lz += (double)lz;
        }
    }
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane windows (W = B/2): workgroup of B wavefronts per row tile, wavefront
// p walks the B rows of plane dz = p - B/2 through its own LDS slice; the
// slices hold the plane sums at the end.
__global__ __launch_bounds__(64 * kNbMaxPlanes, 6) void k_near_planes(
    const float4* __restrict__ pos, const int* __restrict__ typ,
    const unsigned long long* __restrict__ keys, const FFGrid* g, int G, int half,
    const int* __restrict__ cfirst, const int4* __restrict__ tiles,
    const int* __restrict__ ntiles, int n, PairTable tab, double* F) {
    __shared__ float4 sp_all[kNbMaxPlanes][kNbChunk];   // reused for the plane sums
    __shared__ int st_all[kNbMaxPlanes][kNbChunk];
    __shared__ float ttab[3 * kMaxTypes * kMaxTypes];
    const int lane = threadIdx.x % 64;
    const int p = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));   // wave-uniform
    const int planes = 2 * half + 1;
    if ((int)blockIdx.x >= *ntiles) return;            // uniform per workgroup
    if (g->W != half) return;                          // the row walk's grid
    float4* sp = sp_all[p];
    int* st = st_all[p];
    for (int k = threadIdx.x; k < kMaxTypes * kMaxTypes; k += blockDim.x) {
        ttab[k] = tab.sig2[k];
        ttab[kMaxTypes * kMaxTypes + k] = tab.rc2[k];
        ttab[2 * kMaxTypes * kMaxTypes + k] = tab.e24[k];
    }
    __syncthreads();
    const int4 tl = tiles[blockIdx.x];
    const int row = tl.x, s0 = tl.y, s1 = tl.z;
    const int i = s0 + lane;
    const bool live = i < s1;
    const float4 pi = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = live ? typ[i] : 0;
    const int ix = (int)((unsigned)((live ? keys[i] : keys[s0]) >> 32) % (unsigned)G);
    const int x_first = (int)((unsigned)(keys[s0] >> 32) % (unsigned)G);
    const int x_last = (int)((unsigned)(keys[s1 - 1] >> 32) % (unsigned)G);
    const int ry = row % G, rz = row / G;
    const int T = tab.T;
    const float rc2max = tab.rc2max;
    const int wlj = g->Wlj;
    const int trow = ti * T;
    NbAcc a;
    const int dz = p - half;
    const int z = rz + dz;
    if (z >= 0 && z < G) {
        for (int dy = -half; dy <= half; ++dy) {
            const int y = ry + dy;
            if (y < 0 || y >= G) continue;
            const int base = (z * G + y) * G;
            const int J0 = cfirst[base + max(0, x_first - half)];
            const int J1 = cfirst[base + min(G - 1, x_last + half) + 1];
            int ja = J0, jb = J0;
            if (live) {
                ja = cfirst[base + max(0, ix - half)];
                jb = cfirst[base + min(G - 1, ix + half) + 1];
            }
            const bool lj = abs(dy) <= wlj && abs(dz) <= wlj;
            const bool own = dy == 0 && dz == 0;
            for (int c0 = J0; c0 < J1; c0 += kNbChunk) {
                const int S = min(kNbChunk, J1 - c0);
                wave_sync_lds();
                for (int t = lane; t < S; t += 64) {
                    sp[t] = pos[c0 + t];
                    st[t] = typ[c0 + t];
                }
                wave_sync_lds();
                const int lo = min(max(ja - c0, 0), S), hi = min(max(jb - c0, 0), S);
                int m1 = hi, m2 = hi;                // [lo, m1) and [m2, hi): i skipped
                const int si = i - c0;
                if (own && si >= lo && si < hi) {
                    m1 = si;
                    m2 = si + 1;
                }
                if (lj) {
                    nb_range<true>(sp, st, lo, m1, pi, trow, ttab, rc2max, a);
                    nb_range<true>(sp, st, m2, hi, pi, trow, ttab, rc2max, a);
                } else {
                    nb_range<false>(sp, st, lo, m1, pi, trow, ttab, rc2max, a);
                    nb_range<false>(sp, st, m2, hi, pi, trow, ttab, rc2max, a);
                }
            }
        }
    }
    // plane sums, added in plane order (the slices are free after this barrier)
    __syncthreads();
    static_assert(sizeof(sp_all) >= kNbMaxPlanes * 6 * 64 * sizeof(double), "plane sums");
    double* red = reinterpret_cast<double*>(&sp_all[0][0]);   // [planes][6][64]
    double* r = red + (size_t)p * 6 * 64 + lane;
    r[0] = a.Fx;
    r[64] = a.Fy;
    r[128] = a.Fz;
    r[192] = a.Lx;
    r[256] = a.Ly;
    r[320] = a.Lz;
    __syncthreads();
    if (p != 0 || !live) return;
    const double qi = (double)pi.w;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double fc = 0.0, lc = 0.0;
#pragma unroll 1
        for (int q = 0; q < planes; ++q) {
            fc += red[(size_t)q * 6 * 64 + c * 64 + lane];
            lc += red[(size_t)q * 6 * 64 + (c + 3) * 64 + lane];
        }
        F[(size_t)c * n + i] = -qi * fc - lc;
    }
}

// Row windows (W > B/2): one wavefront per row tile.
__global__ __launch_bounds__(64, 6) void k_near_block(const float4* __restrict__ pos,
                                                   const int* __restrict__ typ,
                                                   const unsigned long long* __restrict__ keys,
                                                   const FFGrid* g, int G, int half,
                                                   const int* __restrict__ cfirst,
                                                   const int4* __restrict__ tiles,
                                                   const int* __restrict__ ntiles, int n,
                                                   PairTable tab, double* F) {
    __shared__ float4 sp[kNbChunk];
    __shared__ int st[kNbChunk];
    __shared__ float ttab[3 * kMaxTypes * kMaxTypes];
    const int lane = threadIdx.x;
    if ((int)blockIdx.x >= *ntiles) return;            // uniform per workgroup
    const int W = g->W;
    if (W == half) return;                             // the lane walk's grid
    for (int k = lane; k < kMaxTypes * kMaxTypes; k += 64) {
        ttab[k] = tab.sig2[k];
        ttab[kMaxTypes * kMaxTypes + k] = tab.rc2[k];
        ttab[2 * kMaxTypes * kMaxTypes + k] = tab.e24[k];
    }
    const int4 tl = tiles[blockIdx.x];
    const int row = tl.x, s0 = tl.y, s1 = tl.z;
    const int i = s0 + lane;
    const bool live = i < s1;
    const float4 pi = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = live ? typ[i] : 0;
    const int ix = (int)((unsigned)((live ? keys[i] : keys[s0]) >> 32) % (unsigned)G);
    const int x_first = (int)((unsigned)(keys[s0] >> 32) % (unsigned)G);
    const int x_last = (int)((unsigned)(keys[s1 - 1] >> 32) % (unsigned)G);
    const int ry = row % G, rz = row / G;
    const int T = tab.T;
    const float rc2max = tab.rc2max;
    NbAcc a;
    {
        for (int dz = -W; dz <= W; ++dz) {
            const int z = rz + dz;
            if (z < 0 || z >= G) continue;
            for (int dy = -W; dy <= W; ++dy) {
                const int y = ry + dy;
                if (y < 0 || y >= G) continue;
                // Coulomb partners of this row: cell x within half of the
                // lane's own (an empty window when the row is outside the block)
                const bool row_in = abs(dy) <= half && abs(dz) <= half;
                const int xlo = row_in ? ix - half : (1 << 20);
                const int xhi = row_in ? ix + half : -(1 << 20);
                const int base = (z * G + y) * G;
                const int j0 = cfirst[base + max(0, x_first - W)];
                const int j1 = cfirst[base + min(G - 1, x_last + W) + 1];
                for (int jt = j0; jt < j1; jt += 64) {
                    __syncthreads();
                    const int j = jt + lane;
                    if (j < j1) {
                        sp[lane] = pos[j];
                        st[lane] = (int)((unsigned)(keys[j] >> 32) % (unsigned)G) | (typ[j] << 16);
                    } else {
                        sp[lane] = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
                        st[lane] = 0xFFFF;
                    }
                    __syncthreads();
                    const int cnt = min(64, j1 - jt);
                    const int self = i - jt;           // LDS index of i itself, if present
                    for (int kb = 0; kb < cnt; kb += 32) {
                        const int ke = min(cnt, kb + 32);
                        float bx = 0.f, by = 0.f, bz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
#pragma unroll 4
                        for (int k = kb; k < ke; ++k) {
                            const float4 pj = sp[k];
                            const int info = st[k];
                            const int jx = info & 0xFFFF;
                            const float ddx = pj.x - pi.x, ddy = pj.y - pi.y, ddz = pj.z - pi.z;
                            const float r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                            const float ri = __builtin_amdgcn_rsqf(r2);
                            const bool inb = jx >= xlo && jx <= xhi && k != self;
                            const float w = inb ? (pj.w * ri) * (ri * ri) : 0.f;
                            bx = fmaf(w, ddx, bx);
                            by = fmaf(w, ddy, by);
                            bz = fmaf(w, ddz, bz);
                            if (r2 < rc2max && k != self) {
                                const int pidx = ti * T + (info >> 16);
                                if (r2 < ttab[kMaxTypes * kMaxTypes + pidx]) {
                                    const float ir2 = ri * ri;
                                    const float s2 = ttab[pidx] * ir2;
                                    const float s6 = s2 * s2 * s2;
                                    const float gg = ttab[2 * kMaxTypes * kMaxTypes + pidx] * s6 *
                                                     (2.0f * s6 - 1.0f) * ir2;
                                    lx = fmaf(gg, ddx, lx);
                                    ly = fmaf(gg, ddy, ly);
                                    lz = fmaf(gg, ddz, lz);
                                }
                            }
                        }
                        a.Fx += (double)bx;
                        a.Fy += (double)by;
                        a.Fz += (double)bz;
                        a.Lx += (double)lx;
                        a.Ly += (double)ly;
                        a.Lz += (double)lz;
                    }
                }
            }
        }
    }
    if (live) {
        const double qi = (double)pi.w;
        F[i] = -qi * a.Fx - a.Lx;
        F[(size_t)n + i] = -qi * a.Fy - a.Ly;
        F[2 * (size_t)n + i] = -qi * a.Fz - a.Lz;
    }
}

// ---- moments, occupancy, coarse field -----------------------------------

__global__ __launch_bounds__(kB) void k_moments(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo, int n, int G,
                                                const FFGrid* g, double* mom, int* count) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y,
                 z = (double)h.z + (double)l.z;
    const double L = g->L, hh = g->h;
    const int cx = cell1(x, L, hh, G), cy = cell1(y, L, hh, G), cz = cell1(z, L, hh, G);
    const int c = (cz * G + cy) * G + cx;
    const double q = (double)h.w;
    atomicAdd(&mom[4 * c], q);
    atomicAdd(&mom[4 * c + 1], q * (x - (-L + (cx + 0.5) * hh)));
    atomicAdd(&mom[4 * c + 2], q * (y - (-L + (cy + 0.5) * hh)));
    atomicAdd(&mom[4 * c + 3], q * (z - (-L + (cz + 0.5) * hh)));
    atomicAdd(&count[c], 1);
}

// Block mode: the slots are sorted by grid cell, so each cell's moments are a
// sum over its slot range (one work-item per cell, fixed order, no atomics);
// nm (optional) receives (Q / sq, P / (sq h)).
__global__ __launch_bounds__(kB) void k_moments_sorted(const float4* __restrict__ pos,
                                                       const float4* __restrict__ lo, int M,
                                                       int G, const FFGrid* g,
                                                       const int* __restrict__ cfirst,
                                                       double* mom, int* count, float sq,
                                                       float4* nm) {
    const int c = blockIdx.x * kB + threadIdx.x;
    if (c >= M) return;
    const int a = cfirst[c], b = cfirst[c + 1];
    const double L = g->L, hh = g->h;
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    const double ox = -L + (cx + 0.5) * hh, oy = -L + (cy + 0.5) * hh, oz = -L + (cz + 0.5) * hh;
    double Q = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
    for (int s = a; s < b; ++s) {
        const float4 h = pos[s], l = lo[s];
        const double q = (double)h.w;
        Q += q;
        Px += q * (((double)h.x + (double)l.x) - ox);
        Py += q * (((double)h.y + (double)l.y) - oy);
        Pz += q * (((double)h.z + (double)l.z) - oz);
    }
    mom[4 * (size_t)c] = Q;
    mom[4 * (size_t)c + 1] = Px;
    mom[4 * (size_t)c + 2] = Py;
    mom[4 * (size_t)c + 3] = Pz;
    count[c] = b - a;
    if (nm) {   // the network's normalised moments, as the training snapshots store them
        const double sh = (double)sq * hh;
        nm[c] = make_float4((float)(Q / sq), (float)(Px / sh), (float)(Py / sh), (float)(Pz / sh));
    }
}

// Deterministic compaction of occupied cells in cell order (one workgroup
// of 1024).
__global__ __launch_bounds__(1024) void k_compact(const int* __restrict__ count, int M, int* occ,
                                                  int* cell2occ, int* nocc) {
    __shared__ int buf[8 * 1024];
    __shared__ int wsum[32];
    const int tot = scan_runs(
        M, [&](int c) { return count[c] > 0 ? 1 : 0; },
        [&](int c, int pre, int f) {
            if (f) occ[pre] = c;
            cell2occ[c] = f ? pre : -1;
        },
        buf, wsum);
    if (threadIdx.x == 0) *nocc = tot;
}

// Field at every occupied cell centre from the monopole + dipole of every
// occupied cell outside its B^3 block.  FP32 terms, FP64 totals; the sources
// are split over gridDim.y workgroups (partials reduced by k_coarse_reduce).
__global__ __launch_bounds__(kB) void k_coarse(const double* __restrict__ mom,
                                               const int* __restrict__ occ,
                                               const int* __restrict__ nocc, int G, int B,
                                               const FFGrid* g, int M, double* part) {
    __shared__ float4 sm[kB];          // (Q, Px, Py, Pz)
    __shared__ float4 sc[kB];          // cell index (x, y, z) as floats
    const int no = *nocc;
    if ((int)blockIdx.x * kB >= no) return;            // uniform per workgroup
    const int nsplit = gridDim.y;
    const int per = ((no + nsplit - 1) / nsplit + kB - 1) / kB * kB;
    const int jb = blockIdx.y * per, je = min(no, jb + per);
    const int t = blockIdx.x * kB + threadIdx.x;
    const bool live = t < no;
    const int tc = live ? occ[t] : 0;
    const float tx = (float)(tc % G), ty = (float)((tc / G) % G), tz = (float)(tc / (G * G));
    const float h = (float)g->h;
    const float half = (float)(B / 2) + 0.5f;
    double Ex = 0.0, Ey = 0.0, Ez = 0.0;
    for (int j0 = jb; j0 < je; j0 += kB) {
        __syncthreads();
        const int j = j0 + threadIdx.x;
        if (j < je) {
            const int c = occ[j];
            sm[threadIdx.x] = make_float4((float)mom[4 * c], (float)mom[4 * c + 1],
                                          (float)mom[4 * c + 2], (float)mom[4 * c + 3]);
            sc[threadIdx.x] = make_float4((float)(c % G), (float)((c / G) % G),
                                          (float)(c / (G * G)), 0.f);
        } else {
            sm[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
            sc[threadIdx.x] = make_float4(1e6f, 1e6f, 1e6f, 0.f);
        }
        __syncthreads();
        float ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll 4
        for (int k = 0; k < kB; ++k) {
            const float4 cs = sc[k];
            const float dx = tx - cs.x, dy = ty - cs.y, dz = tz - cs.z;
            // cells of the B^3 block (and the padding) contribute nothing
            const bool outside = fmaxf(fabsf(dx), fmaxf(fabsf(dy), fabsf(dz))) > half;
            const float4 q = sm[k];
            const float rx = dx * h, ry = dy * h, rz = dz * h;
            const float r2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
            const float ri = outside ? __builtin_amdgcn_rsqf(r2) : 0.f;
            const float ri2 = ri * ri, ri3 = ri2 * ri;
            const float pr3 = 3.0f * fmaf(q.w, rz, fmaf(q.z, ry, q.y * rx)) * ri2;
            const float a = q.x + pr3;
            ex = fmaf(fmaf(a, rx, -q.y), ri3, ex);
            ey = fmaf(fmaf(a, ry, -q.z), ri3, ey);
            ez = fmaf(fmaf(a, rz, -q.w), ri3, ez);
        }
        Ex += (double)ex; Ey += (double)ey; Ez += (double)ez;
    }
    if (live) {
        double* o = part + ((size_t)blockIdx.y * M + tc) * 3;
        o[0] = Ex;
        o[1] = Ey;
        o[2] = Ez;
    }
}

// Block mode: second-order local expansion at every occupied cell centre of
// the monopole + dipole field of every occupied cell outside its B^3 block.
// With R = c_t - c_s, u = 1/|R|, p = P.R, the field of one source cell and
// its first and second derivatives at c_t are
//   E_c   = a R_c - u^3 P_c,                         a = Q u^3 + 3 p u^5
//   J_cd  = b R_c R_d + 3u^5 (P_c R_d + P_d R_c) + a delta_cd,
//                                                    b = -3 Q u^5 - 15 p u^7
//   H_cde = c R_c R_d R_e - 15 u^7 (P_c R_d R_e + P_d R_c R_e + P_e R_c R_d)
//           + delta_cd U_e + delta_ce U_d + delta_de U_c,
//                                                    c = 15 Q u^7 + 105 p u^9,
//                                                    U = b R + 3 u^5 P
// (E = -grad of Q/|R| + P.R/|R|^3; J and H its derivatives).  Stored per
// cell: E (3), J (xx xy xz yy yz zz), H (xxx xxy xxz xyy xyz xzz yyy yyz yzz
// zzz).  The field is harmonic outside its sources, so J and H are traceless:
// J_zz, H_xzz, H_yzz and H_zzz are not accumulated here but follow from the
// other components where the expansion is evaluated.  FP32 terms summed over
// one LDS tile, FP64 totals.  The sources are
// split over gridDim.y workgroups (one partial sum each, reduced in a fixed
// order by k_loc_reduce) so that a few hundred target tiles still fill the
// chip.
constexpr int kLB = 128;

// One source cell (moments Q, P about its centre) seen from a target centre
// at R = target - source: adds its E, J and H (the 12 accumulated components)
// to f.  valid = false adds nothing (u = 0 zeroes every term).
__device__ __forceinline__ void loc_add(float* f, float Rx, float Ry, float Rz, float Q, float Px,
                                        float Py, float Pz, bool valid) {
    const float r2 = fmaf(Rz, Rz, fmaf(Ry, Ry, Rx * Rx));
    const float u = valid ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float u2 = u * u, u3 = u2 * u, u5 = u3 * u2, u7 = u5 * u2, u9 = u7 * u2;
    const float p = fmaf(Pz, Rz, fmaf(Py, Ry, Px * Rx));
    const float a = fmaf(3.0f * p, u5, Q * u3);
    const float b = fmaf(-15.0f * p, u7, -3.0f * Q * u5);
    const float c = fmaf(105.0f * p, u9, 15.0f * Q * u7);
    const float t5 = 3.0f * u5, c2 = 15.0f * u7;
    // E
    f[0] = fmaf(a, Rx, fmaf(-u3, Px, f[0]));
    f[1] = fmaf(a, Ry, fmaf(-u3, Py, f[1]));
    f[2] = fmaf(a, Rz, fmaf(-u3, Pz, f[2]));
    // J: (b R_c + 3u^5 P_c) R_d + 3u^5 P_d R_c (+ a on the diagonal)
    const float Tx = t5 * Px, Ty = t5 * Py, Tz = t5 * Pz;
    const float Ux = fmaf(b, Rx, Tx), Uy = fmaf(b, Ry, Ty), Uz = fmaf(b, Rz, Tz);
    f[3] += fmaf(Ux, Rx, fmaf(Tx, Rx, a));
    f[4] += fmaf(Ux, Ry, Ty * Rx);
    f[5] += fmaf(Ux, Rz, Tz * Rx);
    f[6] += fmaf(Uy, Ry, fmaf(Ty, Ry, a));
    f[7] += fmaf(Uy, Rz, Tz * Ry);
    // zz follows from the trace (k_coarse_eval)
    // H: S_cd Y_e - W_c S_de - W_d S_ce + delta terms, S = R R^T,
    // W = 15 u^7 P, Y = c R - W
    const float Wx = c2 * Px, Wy = c2 * Py, Wz = c2 * Pz;
    const float Yx = fmaf(c, Rx, -Wx), Yy = fmaf(c, Ry, -Wy), Yz = fmaf(c, Rz, -Wz);
    const float Sxx = Rx * Rx, Sxy = Rx * Ry, Sxz = Rx * Rz, Syy = Ry * Ry, Syz = Ry * Rz;
    f[9] += fmaf(Sxx, Yx, fmaf(-2.0f * Wx, Sxx, 3.0f * Ux));            // xxx
    f[10] += fmaf(Sxx, Yy, fmaf(-2.0f * Wx, Sxy, Uy));                 // xxy
    f[11] += fmaf(Sxx, Yz, fmaf(-2.0f * Wx, Sxz, Uz));                 // xxz
    f[12] += fmaf(Sxy, Yy, fmaf(-Wx, Syy, fmaf(-Wy, Sxy, Ux)));        // xyy
    f[13] += fmaf(Sxy, Yz, fmaf(-Wx, Syz, -Wy * Sxz));                 // xyz
    f[15] += fmaf(Syy, Yy, fmaf(-2.0f * Wy, Syy, 3.0f * Uy));          // yyy
    f[16] += fmaf(Syy, Yz, fmaf(-2.0f * Wy, Syz, Uz));                 // yyz
    // xzz, yzz, zzz follow from the traces (k_coarse_eval)
}


__global__ __launch_bounds__(kLB) void k_coarse_local(const double* __restrict__ mom,
                                                      const int* __restrict__ occ,
                                                      const int* __restrict__ nocc, int G, int B,
                                                      const FFGrid* g, int M, double* part) {
    __shared__ float4 sm[kLB];         // (Q, Px, Py, Pz)
    __shared__ float4 sc[kLB];         // cell index (x, y, z) as floats
    const int no = *nocc;
    if ((int)blockIdx.x * kLB >= no) return;           // uniform per workgroup
    const int nsplit = gridDim.y;
    const int per = ((no + nsplit - 1) / nsplit + kLB - 1) / kLB * kLB;
    const int jb = blockIdx.y * per, je = min(no, jb + per);
    const int t = blockIdx.x * kLB + threadIdx.x;
    const bool live = t < no;
    const int tc = live ? occ[t] : 0;
    const float tx = (float)(tc % G), ty = (float)((tc / G) % G), tz = (float)(tc / (G * G));
    const float h = (float)g->h;
    const float half = (float)(B / 2) + 0.5f;
    double acc[kLoc];
#pragma unroll
    for (int k = 0; k < kLoc; ++k) acc[k] = 0.0;
    for (int j0 = jb; j0 < je; j0 += kLB) {
        __syncthreads();
        const int j = j0 + threadIdx.x;
        if (j < je) {
            const int c = occ[j];
            sm[threadIdx.x] = make_float4((float)mom[4 * c], (float)mom[4 * c + 1],
                                          (float)mom[4 * c + 2], (float)mom[4 * c + 3]);
            sc[threadIdx.x] = make_float4((float)(c % G), (float)((c / G) % G),
                                          (float)(c / (G * G)), 0.f);
        } else {
            sm[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
            sc[threadIdx.x] = make_float4(1e6f, 1e6f, 1e6f, 0.f);
        }
        __syncthreads();
        float f[kLoc];
#pragma unroll
        for (int k = 0; k < kLoc; ++k) f[k] = 0.f;
        const int cnt = min(kLB, je - j0);
        for (int k = 0; k < cnt; ++k) {
            const float4 cs = sc[k];
            const float dx = tx - cs.x, dy = ty - cs.y, dz = tz - cs.z;
            const bool outside = fmaxf(fabsf(dx), fmaxf(fabsf(dy), fabsf(dz))) > half;
            const float4 m = sm[k];
            loc_add(f, dx * h, dy * h, dz * h, m.x, m.y, m.z, m.w, outside);
        }
#pragma unroll
        for (int k = 0; k < kLoc; ++k) acc[k] += (double)f[k];
    }
    if (live) {
        double* o = part + ((size_t)blockIdx.y * M + tc) * kLoc;
#pragma unroll
        for (int k = 0; k < kLoc; ++k) o[k] = acc[k];
    }
}

// Two-level version of k_coarse_local (G even).  Parent cells are the
// 2x2x2 blocks of cells; pmom holds their monopole and dipole about the
// parent centre.  For a target whose parent is T, parents farther than D
// (Chebyshev, parent cells) from T enter through pmom, streamed through LDS
// over the occupied-parent list; the children of the (2D+1)^3 parents around
// T are gathered per lane (cells outside the grid or inside the target's
// block add nothing).  Both parts are shared out over gridDim.y source splits
// like the one-level kernel; partials are reduced by k_loc_reduce.
__global__ __launch_bounds__(kLB) void k_coarse_local2(
    const double* __restrict__ mom, const int* __restrict__ occ, const int* __restrict__ nocc,
    int G, int B, const double* __restrict__ pmom, const int* __restrict__ pocc,
    const int* __restrict__ npocc, int D, const FFGrid* g, int M, double* part) {
    __shared__ float4 sm[kLB];         // parent (Q, Px, Py, Pz)
    __shared__ float4 sc[kLB];         // parent index (x, y, z) as floats
    const int no = *nocc;
    if ((int)blockIdx.x * kLB >= no) return;           // uniform per workgroup
    const int nsplit = gridDim.y, split = blockIdx.y;
    const int t = blockIdx.x * kLB + threadIdx.x;
    const bool live = t < no;
    const int tc = live ? occ[t] : 0;
    const int tx = tc % G, ty = (tc / G) % G, tz = tc / (G * G);
    const int Gp = G / 2;
    const int Tx = tx / 2, Ty = ty / 2, Tz = tz / 2;
    const float h = (float)g->h;
    const int half = B / 2;
    double acc[kLoc];
#pragma unroll
    for (int k = 0; k < kLoc; ++k) acc[k] = 0.0;
    float f[kLoc];
    // far parents
    const int np = *npocc;
    const int per = ((np + nsplit - 1) / nsplit + kLB - 1) / kLB * kLB;
    const int jb = split * per, je = min(np, jb + per);
    for (int j0 = jb; j0 < je; j0 += kLB) {
        __syncthreads();
        const int j = j0 + threadIdx.x;
        if (j < je) {
            const int p = pocc[j];
            sm[threadIdx.x] = make_float4((float)pmom[4 * p], (float)pmom[4 * p + 1],
                                          (float)pmom[4 * p + 2], (float)pmom[4 * p + 3]);
            sc[threadIdx.x] = make_float4((float)(p % Gp), (float)((p / Gp) % Gp),
                                          (float)(p / (Gp * Gp)), 0.f);
        } else {
            sm[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
            sc[threadIdx.x] = make_float4(-1e6f, -1e6f, -1e6f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kLoc; ++k) f[k] = 0.f;
        const int cnt = min(kLB, je - j0);
        for (int k = 0; k < cnt; ++k) {
            const float4 cs = sc[k];
            const bool far = fmaxf(fabsf((float)Tx - cs.x),
                                   fmaxf(fabsf((float)Ty - cs.y), fabsf((float)Tz - cs.z))) >
                             (float)D + 0.5f;
            const float4 m = sm[k];
            // child centre minus parent centre: (t + 1/2 - 2 (p + 1/2)) h
            loc_add(f, ((float)tx - 2.f * cs.x - 0.5f) * h, ((float)ty - 2.f * cs.y - 0.5f) * h,
                    ((float)tz - 2.f * cs.z - 0.5f) * h, m.x, m.y, m.z, m.w, far);
        }
#pragma unroll
        for (int k = 0; k < kLoc; ++k) acc[k] += (double)f[k];
    }
    // children of the near parents, this split's share of them
    const int side = 2 * D + 1, nnear = side * side * side;
    for (int kp = split; kp < nnear; kp += nsplit) {
        const int px = Tx + kp % side - D, py = Ty + (kp / side) % side - D,
                  pz = Tz + kp / (side * side) - D;
        const bool pin = px >= 0 && py >= 0 && pz >= 0 && px < Gp && py < Gp && pz < Gp;
#pragma unroll
        for (int k = 0; k < kLoc; ++k) f[k] = 0.f;
#pragma unroll 2
        for (int ch = 0; ch < 8; ++ch) {
            const int sx = 2 * px + (ch & 1), sy = 2 * py + ((ch >> 1) & 1), sz = 2 * pz + (ch >> 2);
            const bool use = live && pin &&
                             (abs(sx - tx) > half || abs(sy - ty) > half || abs(sz - tz) > half);
            float Q = 0.f, Px = 0.f, Py = 0.f, Pz = 0.f;
            if (use) {
                const size_t c = ((size_t)sz * G + sy) * G + sx;
                Q = (float)mom[4 * c];
                Px = (float)mom[4 * c + 1];
                Py = (float)mom[4 * c + 2];
                Pz = (float)mom[4 * c + 3];
            }
            loc_add(f, (float)(tx - sx) * h, (float)(ty - sy) * h, (float)(tz - sz) * h, Q, Px, Py,
                    Pz, use);
        }
#pragma unroll
        for (int k = 0; k < kLoc; ++k) acc[k] += (double)f[k];
    }
    if (live) {
        double* o = part + ((size_t)blockIdx.y * M + tc) * kLoc;
#pragma unroll
        for (int k = 0; k < kLoc; ++k) o[k] = acc[k];
    }
}

// Parent cells (2x2x2 blocks of cells): the children's moments moved to the
// parent centre, Q_p = sum Q_c, P_p = sum (P_c + Q_c (c_c - c_p)), and the
// particle count.
__global__ __launch_bounds__(kB) void k_parent_moments(const double* __restrict__ mom,
                                                       const int* __restrict__ count, int G,
                                                       const FFGrid* g, double* pmom,
                                                       int* pcount) {
    const int Gp = G / 2, Mp = Gp * Gp * Gp;
    const int p = blockIdx.x * kB + threadIdx.x;
    if (p >= Mp) return;
    const int px = p % Gp, py = (p / Gp) % Gp, pz = p / (Gp * Gp);
    const double h = g->h;
    double Q = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
    int n = 0;
    for (int ch = 0; ch < 8; ++ch) {
        const int dx = ch & 1, dy = (ch >> 1) & 1, dz = ch >> 2;
        const size_t c = ((size_t)(2 * pz + dz) * G + (2 * py + dy)) * G + (2 * px + dx);
        const double q = mom[4 * c];
        Q += q;
        // child centre - parent centre = (d - 1/2) h per axis
        Px += mom[4 * c + 1] + q * (dx - 0.5) * h;
        Py += mom[4 * c + 2] + q * (dy - 0.5) * h;
        Pz += mom[4 * c + 3] + q * (dz - 0.5) * h;
        n += count[c];
    }
    pmom[4 * (size_t)p] = Q;
    pmom[4 * (size_t)p + 1] = Px;
    pmom[4 * (size_t)p + 2] = Py;
    pmom[4 * (size_t)p + 3] = Pz;
    pcount[p] = n;
}

// out[cell] = sum over the source splits of the partial expansions, in split
// order, for every occupied cell.
__global__ __launch_bounds__(kB) void k_loc_reduce(const double* __restrict__ part,
                                                   const int* __restrict__ occ,
                                                   const int* __restrict__ nocc, int M, int nsplit,
                                                   double* out) {
    const int e = blockIdx.x * kB + threadIdx.x;
    if (e >= *nocc * kLoc) return;
    const size_t c = (size_t)occ[e / kLoc];
    const int k = e % kLoc;
    double v = 0.0;
    for (int p = 0; p < nsplit; ++p) v += part[((size_t)p * M + c) * kLoc + k];
    out[c * kLoc + k] = v;
}

// Coarse field at every particle: the centre value of its cell (radial mode)
// or the cell's local expansion at its offset d = x - centre (block mode):
// E_a + J_ab d_b + (1/2) H_abe d_b d_e.  Out: [3][n] slot order.
__global__ __launch_bounds__(kB) void k_coarse_eval(const float4* __restrict__ pos,
                                                    const float4* __restrict__ lo, int n, int G,
                                                    const FFGrid* g, const double* __restrict__ Ec,
                                                    int block_mode, double* Ep) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const float4 hv = pos[s], l = lo[s];
    const double x = (double)hv.x + (double)l.x, y = (double)hv.y + (double)l.y,
                 z = (double)hv.z + (double)l.z;
    const double L = g->L, hh = g->h;
    const int cx = cell1(x, L, hh, G), cy = cell1(y, L, hh, G), cz = cell1(z, L, hh, G);
    const size_t c = ((size_t)cz * G + cy) * G + cx;
    double E[3];
    if (!block_mode) {
        E[0] = Ec[3 * c]; E[1] = Ec[3 * c + 1]; E[2] = Ec[3 * c + 2];
    } else {
        double o[kLoc];
        for (int k = 0; k < kLoc; ++k) o[k] = Ec[kLoc * c + k];
        // the components the expansion kernel leaves to Laplace's equation
        o[8] = -(o[3] + o[6]);             // J_zz
        o[14] = -(o[9] + o[12]);           // H_xzz = -(H_xxx + H_xyy)
        o[17] = -(o[10] + o[15]);          // H_yzz = -(H_xxy + H_yyy)
        o[18] = -(o[11] + o[16]);          // H_zzz = -(H_xxz + H_yyz)
        const double dx = x - (-L + (cx + 0.5) * hh), dy = y - (-L + (cy + 0.5) * hh),
                     dz = z - (-L + (cz + 0.5) * hh);
        const double xx = 0.5 * dx * dx, yy = 0.5 * dy * dy, zz = 0.5 * dz * dz;
        const double xy = dx * dy, xz = dx * dz, yz = dy * dz;
        // J: 3 xx, 4 xy, 5 xz, 6 yy, 7 yz, 8 zz
        // H: 9 xxx, 10 xxy, 11 xxz, 12 xyy, 13 xyz, 14 xzz, 15 yyy, 16 yyz, 17 yzz, 18 zzz
        E[0] = o[0] + o[3] * dx + o[4] * dy + o[5] * dz + o[9] * xx + o[12] * yy + o[14] * zz +
               o[10] * xy + o[11] * xz + o[13] * yz;
        E[1] = o[1] + o[4] * dx + o[6] * dy + o[7] * dz + o[10] * xx + o[15] * yy + o[17] * zz +
               o[12] * xy + o[13] * xz + o[16] * yz;
        E[2] = o[2] + o[5] * dx + o[7] * dy + o[8] * dz + o[11] * xx + o[16] * yy + o[18] * zz +
               o[13] * xy + o[14] * xz + o[17] * yz;
    }
    Ep[s] = E[0];
    Ep[(size_t)n + s] = E[1];
    Ep[2 * (size_t)n + s] = E[2];
}

// E[cell] = sum over the source splits of k_coarse's partial fields, in split
// order, for every occupied cell.
__global__ __launch_bounds__(kB) void k_coarse_reduce(const double* __restrict__ part,
                                                      const int* __restrict__ occ,
                                                      const int* __restrict__ nocc, int M,
                                                      int nsplit, double* E) {
    const int e = blockIdx.x * kB + threadIdx.x;
    if (e >= *nocc * 3) return;
    const size_t c = (size_t)occ[e / 3];
    const int k = e % 3;
    double v = 0.0;
    for (int p = 0; p < nsplit; ++p) v += part[((size_t)p * M + c) * 3 + k];
    E[c * 3 + k] = v;
}

// Moment rows of the B^3 block around each occupied cell (first 4 B^3
// features of every particle in that cell), zero-padded to Kp.
__global__ __launch_bounds__(kB) void k_cell_features(const double* __restrict__ mom,
                                                      const int* __restrict__ occ,
                                                      const int* __restrict__ nocc, int G, int B,
                                                      const FFGrid* g, float sq, int Kp,
                                                      float* Xc) {
    const int oc = blockIdx.x;
    if (oc >= *nocc) return;
    const int c = occ[oc];
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    const int half = B / 2;
    const double sh = (double)sq * g->h;
    float* row = Xc + (size_t)oc * Kp;
    for (int f = threadIdx.x; f < Kp; f += kB) {
        float v = 0.f;
        if (f < 4 * B * B * B) {
            const int cell = f / 4, comp = f % 4;
            const int dx = cell % B - half, dy = (cell / B) % B - half, dz = cell / (B * B) - half;
            const int x = cx + dx, y = cy + dy, z = cz + dz;
            if (x >= 0 && y >= 0 && z >= 0 && x < G && y < G && z < G) {
                const double m = mom[4 * ((z * G + y) * G + x) + comp];
                v = (float)(comp == 0 ? m / sq : m / sh);
            }
        }
        row[f] = v;
    }
}

__device__ __forceinline__ void particle_cell(const float4 h, const float4 l, int G,
                                              const FFGrid* g, int* c, float off[3]) {
    const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y,
                 z = (double)h.z + (double)l.z;
    const double L = g->L, hh = g->h;
    const int cx = cell1(x, L, hh, G), cy = cell1(y, L, hh, G), cz = cell1(z, L, hh, G);
    *c = (cz * G + cy) * G + cx;
    off[0] = (float)((x - (-L + (cx + 0.5) * hh)) / hh);
    off[1] = (float)((y - (-L + (cy + 0.5) * hh)) / hh);
    off[2] = (float)((z - (-L + (cz + 0.5) * hh)) / hh);
}

// First layer finished per particle: z1 = A_cell + W1[offset rows] o + b1;
// one work-item per (particle, hidden unit).
__global__ __launch_bounds__(kB) void k_layer1(const float4* __restrict__ pos,
                                               const float4* __restrict__ lo, int n, int G,
                                               const FFGrid* g, const int* __restrict__ cell2occ,
                                               const float* __restrict__ Ac,
                                               const float* __restrict__ W1o,
                                               const float* __restrict__ b1, int H, float* h1) {
    const size_t e = (size_t)blockIdx.x * kB + threadIdx.x;
    if (e >= (size_t)n * H) return;
    const int s = (int)(e / H), j = (int)(e % H);
    int c;
    float off[3];
    particle_cell(pos[s], lo[s], G, g, &c, off);
    const int oc = cell2occ[c];
    if (oc < 0) {   // cannot happen: the particle's own cell is occupied
        h1[e] = 0.f;
        return;
    }
    const float z = Ac[(size_t)oc * H + j] + bf16_round(off[0]) * bf16_round(W1o[j]) +
                    bf16_round(off[1]) * bf16_round(W1o[H + j]) +
                    bf16_round(off[2]) * bf16_round(W1o[2 * H + j]) + b1[j];
    h1[e] = silu_f(z);
}

// The network's per-particle part fused into one kernel for hidden width 128:
// finish layer 1 (A_cell + W1_offset o + b1, SiLU), layer 2 (128 x 128,
// SiLU) and layer 3 (128 x 16) on the matrix cores, and
// F = F_near + q (E_coarse + scale y).  W2 and W3 are staged once per
// workgroup in LDS as BF16, column-major (the B operand of
// v_mfma_f32_16x16x32_bf16: 8 consecutive K values of one column per lane).
// Every wavefront then walks 16-particle tiles on its own: the tile's
// activations (16 x 128, layer 1 and then layer 2 in the same rows) live in
// the wavefront's own LDS rows, so a tile needs no workgroup barrier.
// Activations are rounded to BF16 where the unfused path rounds them (as the
// next product stages them), so the two paths compute the same products.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int kMW = 16;                 // particles per wavefront tile (one MFMA row block)
constexpr int kFW = 8;                  // wavefronts per workgroup
constexpr int kFH = 128;                // hidden width of the fused kernel
constexpr int kFHP = kFH + 8;           // padded LDS row (BF16 elements)

__global__ __launch_bounds__(kFW * 64) void k_mlp_fused(
    const float4* __restrict__ pos, const float4* __restrict__ lo, int n, int G,
    const FFGrid* g, const float* __restrict__ Ac, const float* __restrict__ W1o,
    const float* __restrict__ b1, const float* __restrict__ W2, const float* __restrict__ b2,
    const float* __restrict__ W3, const float* __restrict__ b3, float scale,
    const double* __restrict__ Fn, const double* __restrict__ Ep, double* Fpart, double* Fc,
    double* Fm) {
    __shared__ __attribute__((aligned(16))) __bf16 sW2[kFH][kFHP];        // [out column][k]
    __shared__ __attribute__((aligned(16))) __bf16 sW3[16][kFHP];         // [out column][k]
    __shared__ __attribute__((aligned(16))) __bf16 sAct[kFW][kMW][kFHP];  // per wavefront
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    for (int e = t; e < kFH * kFH; e += kFW * 64) sW2[e % kFH][e / kFH] = bf16_rne(W2[e]);
    for (int e = t; e < kFH * 16; e += kFW * 64) sW3[e % 16][e / 16] = bf16_rne(W3[e]);
    // this lane's layer-1 columns l and l + 64: offset weights and bias
    float wo[2][3], bias1[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const int col = l + 64 * hh;
        wo[hh][0] = bf16_round(W1o[col]);
        wo[hh][1] = bf16_round(W1o[kFH + col]);
        wo[hh][2] = bf16_round(W1o[2 * kFH + col]);
        bias1[hh] = b1[col];
    }
    __syncthreads();
    __bf16 (*act)[kFHP] = sAct[w];
    const int ntiles = (n + kMW - 1) / kMW;
    for (int tile = blockIdx.x * kFW + w; tile < ntiles; tile += gridDim.x * kFW) {
        const int s0 = tile * kMW;
        // lanes 0..15: the tile's particles (cell, offset)
        int oc = -1;
        float o0 = 0.f, o1 = 0.f, o2 = 0.f;
        if (l < kMW && s0 + l < n) {
            float off[3];
            particle_cell(pos[s0 + l], lo[s0 + l], G, g, &oc, off);
            o0 = bf16_round(off[0]);
            o1 = bf16_round(off[1]);
            o2 = bf16_round(off[2]);
        }
        // layer 1: the 16 rows, columns l and l + 64; every row's cell term
        // is loaded before the arithmetic so the gathers overlap
        float av[kMW][2];
#pragma unroll
        for (int r = 0; r < kMW; ++r) {
            const int ocr = __shfl(oc, r);
            av[r][0] = ocr >= 0 ? Ac[(size_t)ocr * kFH + l] : 0.f;
            av[r][1] = ocr >= 0 ? Ac[(size_t)ocr * kFH + l + 64] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < kMW; ++r) {
            const int ocr = __shfl(oc, r);
            const float f0 = __shfl(o0, r), f1 = __shfl(o1, r), f2 = __shfl(o2, r);
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int col = l + 64 * hh;
                float a = 0.f;
                if (ocr >= 0) {
                    const float z = av[r][hh] + f0 * wo[hh][0] + f1 * wo[hh][1] +
                                    f2 * wo[hh][2] + bias1[hh];
                    a = silu_f(z);
                }
                act[r][col] = bf16_rne(a);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // layer 2: 16 rows x 128 columns
        f32x4_t acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kFH / 32; ++ks) {
            const int kk = ks * 32 + 8 * (l / 16);
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&act[l % 16][kk]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(&sW2[j * 16 + l % 16][kk]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = j * 16 + l % 16;
            const float bb = b2[c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                act[4 * (l / 16) + r][c] = bf16_rne(silu_f(acc[j][r] + bb));
        }
        __builtin_amdgcn_wave_barrier();
        // layer 3: 16 rows x 16 output columns (3 used)
        f32x4_t y = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kFH / 32; ++ks) {
            const int kk = ks * 32 + 8 * (l / 16);
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&act[l % 16][kk]);
            const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(&sW3[l % 16][kk]);
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, y, 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
        // lane (k = l % 16 < 3, l / 16) holds output k of rows 4 (l / 16) + 0..3
        const int k = l % 16;
        if (k < 3) {
            const float bb = b3[k];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = s0 + 4 * (l / 16) + r;
                if (s < n) {
                    const double q = (double)pos[s].w;
                    const double ec = q * Ep[(size_t)k * n + s];
                    const double em = q * (double)scale * (double)(y[r] + bb);
                    Fpart[(size_t)k * n + s] = Fn[(size_t)k * n + s] + ec + em;
                    if (Fc) Fc[(size_t)k * n + s] = ec;
                    if (Fm) Fm[(size_t)k * n + s] = em;
                }
            }
        }
    }
}

// W1 of hidden width 128 as BF16, column-major: wbf[col][k] (k < Kp), the
// B operand layout of the cell layer (8 consecutive K of one column = 16 B).
__global__ __launch_bounds__(kB) void k_w1_bf16(const float* __restrict__ W1, int Kp,
                                                __bf16* __restrict__ wbf) {
    const int e = blockIdx.x * kB + threadIdx.x;
    if (e >= kFH * Kp) return;
    const int col = e / Kp, k = e % Kp;
    wbf[e] = bf16_rne(W1[(size_t)k * kFH + col]);
}

// Layer 1, moment part, for hidden width 128: Ac[c][col] = sum over the
// B^3 block's features k = 4 b + comp of bf16(nm[cell b][comp])
// bf16(W1[k][col]) (zero outside the grid), one row per grid cell, on the
// matrix cores.  The features are gathered from the normalised moment grid
// nm as the A operand is formed (8 consecutive features = two neighbour
// cells per lane), a chunk of 128 K ahead of the LDS staging of the BF16
// W1 copy wbf (column-major, 128 K at a time), so the gathers and the
// staging overlap.  Workgroup: 64 cells (4 wavefronts x 16 rows) x 128
// columns.
__global__ __launch_bounds__(256) void k_cell_layer(const float4* __restrict__ nm, int G, int B,
                                                    const __bf16* __restrict__ wbf, int Kp,
                                                    float* __restrict__ Ac) {
    __shared__ __attribute__((aligned(16))) __bf16 sB[kFH][kFHP];   // [column][k - k0]
    __shared__ int nb[7 * 7 * 7];                                   // block offsets, packed
    const int no = G * G * G;
    const int m0 = blockIdx.x * 64;
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    const int B3 = B * B * B, half = B / 2;
    for (int b = t; b < B3; b += 256)
        nb[b] = (b % B - half + 8) | (((b / B) % B - half + 8) << 8) | ((b / (B * B) - half + 8) << 16);
    __syncthreads();
    const int row = m0 + w * 16 + l % 16;
    const bool live = row < no;
    const int c = live ? row : m0;
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    f32x4_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Kp; k0 += kFH) {
        // this lane's features of the chunk: 4 steps x 2 cells
        float4 v[4][2];
#pragma unroll
        for (int ks = 0; ks < kFH / 32; ++ks) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int b = (k0 + ks * 32 + 8 * (l / 16)) / 4 + hh;
                v[ks][hh] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (live && b < B3) {
                    const int o = nb[b];
                    const int x = cx + (o & 255) - 8, y = cy + ((o >> 8) & 255) - 8,
                              z = cz + (o >> 16) - 8;
                    if (x >= 0 && y >= 0 && z >= 0 && x < G && y < G && z < G)
                        v[ks][hh] = nm[(z * G + y) * G + x];
                }
            }
        }
        __syncthreads();                                // sB of the previous chunk is free
        for (int e = t; e < kFH * kFH / 8; e += 256) {
            const int col = e / (kFH / 8), q = e % (kFH / 8);
            bf16x8_t x = {};
            if (k0 + 8 * q < Kp)
                x = *reinterpret_cast<const bf16x8_t*>(wbf + (size_t)col * Kp + k0 + 8 * q);
            *reinterpret_cast<bf16x8_t*>(&sB[col][8 * q]) = x;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kFH / 32; ++ks) {
            bf16x8_t a;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                a[4 * hh] = bf16_rne(v[ks][hh].x);
                a[4 * hh + 1] = bf16_rne(v[ks][hh].y);
                a[4 * hh + 2] = bf16_rne(v[ks][hh].z);
                a[4 * hh + 3] = bf16_rne(v[ks][hh].w);
            }
            const int kl = ks * 32 + 8 * (l / 16);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bf16x8_t bv = *reinterpret_cast<const bf16x8_t*>(&sB[j * 16 + l % 16][kl]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = m0 + w * 16 + 4 * (l / 16) + r;
            if (rr < no) Ac[(size_t)rr * kFH + j * 16 + l % 16] = acc[j][r];
        }
    }
}

// F = F_near + q (E_coarse + scale y) into Fpart (slot order) and optional
// parts.
__global__ __launch_bounds__(kB) void k_combine(const float4* __restrict__ pos, int n,
                                                const double* __restrict__ Fn,
                                                const double* __restrict__ Ep,
                                                const float* __restrict__ y, int Op, float scale,
                                                double* Fpart, double* Fc, double* Fm) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const double q = (double)pos[s].w;
    for (int k = 0; k < 3; ++k) {
        const double ec = q * Ep[(size_t)k * n + s];
        const double em = q * (double)scale * (double)y[(size_t)s * Op + k];
        Fpart[(size_t)k * n + s] = Fn[(size_t)k * n + s] + ec + em;
        if (Fc) Fc[(size_t)k * n + s] = ec;
        if (Fm) Fm[(size_t)k * n + s] = em;
    }
}

// Exact far field sum_{j: r >= rc} q_j (x_i - x_j) / r^3 (no q_i factor).
__global__ __launch_bounds__(kB) void k_far_exact(const float4* __restrict__ pos, int n,
                                                  float rc2, double* E) {
    __shared__ float4 sp[kB];
    const int i = blockIdx.x * kB + threadIdx.x;
    const float4 pi = i < n ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    double Ex = 0.0, Ey = 0.0, Ez = 0.0;
    for (int j0 = 0; j0 < n; j0 += kB) {
        __syncthreads();
        const int j = j0 + threadIdx.x;
        sp[threadIdx.x] = j < n ? pos[j] : make_float4(kFarAway, kFarAway, kFarAway, 0.f);
        __syncthreads();
        float ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll 8
        for (int k = 0; k < kB; ++k) {
            const float4 pj = sp[k];
            const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float w = r2 >= rc2 ? (pj.w * ri) * (ri * ri) : 0.f;
            ex = fmaf(w, dx, ex);
            ey = fmaf(w, dy, ey);
            ez = fmaf(w, dz, ez);
        }
        Ex += (double)ex; Ey += (double)ey; Ez += (double)ez;
    }
    if (i < n) {
        E[i] = -Ex;
        E[(size_t)n + i] = -Ey;
        E[2 * (size_t)n + i] = -Ez;
    }
}

// Exact Coulomb field of the particles outside the B^3 block of each
// particle's cell (no q_i factor); cells from the sorted keys.
__global__ __launch_bounds__(kB) void k_far_exact_block(const float4* __restrict__ pos,
                                                        const unsigned long long* __restrict__ keys,
                                                        int n, int G, int half, double* E) {
    __shared__ float4 sp[kB];
    __shared__ int4 sc[kB];
    const int i = blockIdx.x * kB + threadIdx.x;
    const float4 pi = i < n ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const unsigned ci = i < n ? (unsigned)(keys[i] >> 32) : 0u;
    const int ix = (int)(ci % G), iy = (int)((ci / G) % G), iz = (int)(ci / (G * G));
    double Ex = 0.0, Ey = 0.0, Ez = 0.0;
    for (int j0 = 0; j0 < n; j0 += kB) {
        __syncthreads();
        const int j = j0 + threadIdx.x;
        if (j < n) {
            const unsigned cj = (unsigned)(keys[j] >> 32);
            sp[threadIdx.x] = pos[j];
            sc[threadIdx.x] = make_int4((int)(cj % G), (int)((cj / G) % G), (int)(cj / (G * G)), 0);
        } else {
            sp[threadIdx.x] = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            sc[threadIdx.x] = make_int4(-(1 << 20), -(1 << 20), -(1 << 20), 0);
        }
        __syncthreads();
        float ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll 8
        for (int k = 0; k < kB; ++k) {
            const float4 pj = sp[k];
            const int4 cj = sc[k];
            const bool far = abs(cj.x - ix) > half || abs(cj.y - iy) > half || abs(cj.z - iz) > half;
            const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float w = far ? (pj.w * ri) * (ri * ri) : 0.f;
            ex = fmaf(w, dx, ex);
            ey = fmaf(w, dy, ey);
            ez = fmaf(w, dz, ez);
        }
        Ex += (double)ex; Ey += (double)ey; Ez += (double)ez;
    }
    if (i < n) {
        E[i] = -Ex;
        E[(size_t)n + i] = -Ey;
        E[2 * (size_t)n + i] = -Ez;
    }
}

// Training samples of the current snapshot: (snapshot, cell, offset,
// target = E_far - E_coarse) appended at base.
__global__ __launch_bounds__(kB) void k_collect(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo, int n, int G,
                                                const FFGrid* g, const double* __restrict__ Efar,
                                                const double* __restrict__ Ep, int snap,
                                                int64_t base, int* s_snap, int* s_cell,
                                                float* s_off, float* s_tgt) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    int c;
    float off[3];
    particle_cell(pos[s], lo[s], G, g, &c, off);
    const int64_t k = base + s;
    s_snap[k] = snap;
    s_cell[k] = c;
    for (int d = 0; d < 3; ++d) {
        s_off[3 * k + d] = off[d];
        s_tgt[3 * k + d] = (float)(Efar[(size_t)d * n + s] - Ep[(size_t)d * n + s]);
    }
}

// Normalised moment grid of a snapshot (for feature gathers at train time).
__global__ __launch_bounds__(kB) void k_snap_mom(const double* __restrict__ mom, int M,
                                                 const FFGrid* g, float sq, float* out) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= 4 * M) return;
    const double sh = (double)sq * g->h;
    out[k] = (float)((k % 4 == 0) ? mom[k] / sq : mom[k] / sh);
}

// Batch features and scaled targets from the sample store.
__global__ __launch_bounds__(kB) void k_gather_batch(const int* __restrict__ idx, int B_,
                                                     const int* __restrict__ s_snap,
                                                     const int* __restrict__ s_cell,
                                                     const float* __restrict__ s_off,
                                                     const float* __restrict__ s_tgt,
                                                     const float* __restrict__ snap_mom, int G,
                                                     int Bk, int Kp, float inv_scale, float* X,
                                                     float* T) {
    const int b = blockIdx.x;
    if (b >= B_) return;
    const int64_t k = idx[b];
    const int snap = s_snap[k], c = s_cell[k];
    const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
    const int half = Bk / 2;
    const float* mg = snap_mom + (size_t)snap * 4 * G * G * G;
    float* row = X + (size_t)b * Kp;
    const int nm = 4 * Bk * Bk * Bk;
    for (int f = threadIdx.x; f < Kp; f += kB) {
        float v = 0.f;
        if (f < nm) {
            const int cell = f / 4, comp = f % 4;
            const int x = cx + cell % Bk - half, y = cy + (cell / Bk) % Bk - half,
                      z = cz + cell / (Bk * Bk) - half;
            if (x >= 0 && y >= 0 && z >= 0 && x < G && y < G && z < G)
                v = mg[4 * ((z * G + y) * G + x) + comp];
        } else if (f < nm + 3) {
            v = s_off[3 * k + (f - nm)];
        }
        row[f] = v;
    }
    if (threadIdx.x < 3) T[3 * b + threadIdx.x] = s_tgt[3 * k + threadIdx.x] * inv_scale;
}

// Copy rows of m x K features (host layout, K = 4B^3+3) into a Kp-wide buffer.
__global__ __launch_bounds__(kB) void k_pad_rows(const float* __restrict__ X, int m, int K,
                                                 int Kp, float* out) {
    const int r = blockIdx.x;
    if (r >= m) return;
    for (int f = threadIdx.x; f < Kp; f += kB) out[(size_t)r * Kp + f] = f < K ? X[(size_t)r * K + f] : 0.f;
}

// F = q E (slot order [3][n]).
__global__ __launch_bounds__(kB) void k_q_times(const float4* __restrict__ pos, int n,
                                                const double* __restrict__ E, double* F) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const double q = (double)pos[s].w;
    for (int k = 0; k < 3; ++k) F[(size_t)k * n + s] = q * E[(size_t)k * n + s];
}

__global__ __launch_bounds__(kB) void k_rel_err(const double* __restrict__ Fa,
                                                const double* __restrict__ Fb, int n,
                                                double* rel) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    double d2 = 0.0, b2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double a = Fa[(size_t)k * n + s], b = Fb[(size_t)k * n + s];
        d2 += (a - b) * (a - b);
        b2 += b * b;
    }
    rel[s] = b2 > 0.0 ? sqrt(d2 / b2) : (d2 > 0.0 ? INFINITY : 0.0);
}

__global__ __launch_bounds__(kB) void k_sum_parts(const double* __restrict__ F, int parts, int n,
                                                  double* out) {
    const int e = blockIdx.x * kB + threadIdx.x;
    if (e >= 3 * n) return;
    double v = 0.0;
    for (int p = 0; p < parts; ++p) v += F[(size_t)p * 3 * n + e];
    out[e] = v;
}

__global__ __launch_bounds__(kB) void k_to_orig(const double* __restrict__ F, const int* oid,
                                                int n, double* out) {
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= n) return;
    const size_t o = (size_t)oid[s];
    for (int k = 0; k < 3; ++k) out[3 * o + k] = F[(size_t)k * n + s];
}

// ---- host side ------------------------------------------------------------

FarField* FF(ld_ctx* c) { return c->ff; }

template <class T>
bool dalloc(T** p, size_t count) {
    return hipMalloc(p, sizeof(T) * (count > 0 ? count : 1)) == hipSuccess;
}

void ff_free_bufs(FarField* f) {
    void* b[] = {f->grid, f->cstart, f->cend, f->Fnear, f->mom, f->count, f->occ, f->cell2occ,
                 f->nocc, f->Ecell, f->Ep, f->cfirst, f->tiles, f->ntiles, f->loc_part, f->pmom,
                 f->pcount, f->pocc, f->pcell2occ, f->npocc, f->Xc, f->Ac, f->h1, f->h2, f->y, f->W, f->w1bf, f->grad, f->adam_m,
                 f->adam_v, f->rel, f->Efar, f->snap_mom, f->s_snap, f->s_cell, f->s_off,
                 f->s_tgt, f->bX, f->bT, f->bZ1, f->bA1, f->bZ2, f->bA2, f->bY, f->bdY, f->bd2,
                 f->bd1, f->bidx, f->loss_part, f->gws};
    for (void* p : b)
        if (p) (void)hipFree(p);
    conv_free(&f->conv);
}

#define KLAUNCH(kernel, grid, block, ...)                                                 \
    do {                                                                                  \
        hipLaunchKernelGGL(kernel, grid, block, 0, __VA_ARGS__);                          \
        HIP_TRY(hipGetLastError());                                                       \
    } while (0)

// Moments, occupancy and coarse field at the current positions (after ff_near).
ld_status ff_grid_and_coarse(ld_ctx* c, hipStream_t s) {
    FarField* f = FF(c);
    const int n = (int)c->n;
    const int G = f->cfg.grid, M = G * G * G;
    // the grid is the one ff_near set for these positions
    if (f->cfg.near_mode == 1) {
        // slots are in grid-cell order (ff_near ran first): per-cell sums
        KLAUNCH(k_moments_sorted, dim3((M + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, M, G,
                f->grid, f->cfirst, f->mom, f->count, f->sq,
                f->H == kFH ? reinterpret_cast<float4*>(f->Xc) : nullptr);
    } else {
        KLAUNCH(k_zero_d, dim3((4 * M + kB - 1) / kB), dim3(kB), s, f->mom, 4 * M);
        KLAUNCH(k_zero_i, dim3((M + kB - 1) / kB), dim3(kB), s, f->count, M);
        KLAUNCH(k_moments, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, n, G, f->grid,
                f->mom, f->count);
    }
    // the occupied-cell list serves the direct coarse sums and the unfused
    // network (the FFT expansion and the hidden-128 kernels work per cell)
    if (!(f->cfg.near_mode == 1 && f->use_conv && f->H == kFH))
        KLAUNCH(k_compact, dim3(1), dim3(1024), s, f->count, M, f->occ, f->cell2occ, f->nocc);
    if (f->cfg.near_mode == 1 && f->cfg.parent_reach > 0) {
        const int Mp = (G / 2) * (G / 2) * (G / 2);
        KLAUNCH(k_parent_moments, dim3((Mp + kB - 1) / kB), dim3(kB), s, f->mom, f->count, G,
                f->grid, f->pmom, f->pcount);
        KLAUNCH(k_compact, dim3(1), dim3(1024), s, f->pcount, Mp, f->pocc, f->pcell2occ, f->npocc);
        KLAUNCH(k_coarse_local2, dim3((M + kLB - 1) / kLB, f->loc_split), dim3(kLB), s, f->mom,
                f->occ, f->nocc, G, f->cfg.block, f->pmom, f->pocc, f->npocc,
                f->cfg.parent_reach, f->grid, M, f->loc_part);
        KLAUNCH(k_loc_reduce, dim3((M * kLoc + kB - 1) / kB), dim3(kB), s, f->loc_part, f->occ,
                f->nocc, M, f->loc_split, f->Ecell);
    } else if (f->cfg.near_mode == 1 && f->use_conv) {
        const double* h = (const double*)((const char*)f->grid + offsetof(FFGrid, h));
        HIP_TRY(conv_local(&f->conv, f->mom, G, h, f->Ecell, s));
    } else if (f->cfg.near_mode == 1) {
        KLAUNCH(k_coarse_local, dim3((M + kLB - 1) / kLB, f->loc_split), dim3(kLB), s, f->mom,
                f->occ, f->nocc, G, f->cfg.block, f->grid, M, f->loc_part);
        KLAUNCH(k_loc_reduce, dim3((M * kLoc + kB - 1) / kB), dim3(kB), s, f->loc_part, f->occ,
                f->nocc, M, f->loc_split, f->Ecell);
    } else {
        KLAUNCH(k_coarse, dim3((M + kB - 1) / kB, f->loc_split), dim3(kB), s, f->mom, f->occ,
                f->nocc, G, f->cfg.block, f->grid, M, f->loc_part);
        KLAUNCH(k_coarse_reduce, dim3((M * 3 + kB - 1) / kB), dim3(kB), s, f->loc_part, f->occ,
                f->nocc, M, f->loc_split, f->Ecell);
    }
    KLAUNCH(k_coarse_eval, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, n, G, f->grid,
            f->Ecell, f->cfg.near_mode, f->Ep);
    return LD_OK;
}

// Near cell list (re-sorts the slots by cell) and the exact near forces.
ld_status ff_near(ld_ctx* c, hipStream_t s) {
    FarField* f = FF(c);
    const int n = (int)c->n;
    const int G = f->cfg.grid, M = G * G * G;
    const bool block = f->cfg.near_mode == 1;
    KLAUNCH(k_absmax_part, dim3(64), dim3(kB), s, c->pos, n, c->sb.bounds_part);
    const int nwg = ld::radix_tiles(n);
    KLAUNCH(k_near_keys, dim3(nwg), dim3(kB), s, c->pos, c->lo, n, c->sb.bounds_part,
            f->cfg.near_cut, G, f->cfg.near_mode, f->cfg.block, f->rlj, f->grid, c->sb.keys,
            c->sb.hist, nwg);
    const int NC = kMaxNearCells * kMaxNearCells * kMaxNearCells;
    {
        // cell indices stay below G^3 (block) or 64^3 (radial near cells)
        const int cells = block ? M : NC;
        int bits = 1;
        while ((1 << bits) < cells) ++bits;
        HIP_TRY(ld::launch_radix_by_high(c->sb.keys,
                                         reinterpret_cast<unsigned long long*>(c->sb.tmp4), n,
                                         bits, c->sb.hist, s, true));
        // permute into the second slot arrays and swap (no copy back); a
        // captured step graph holds the old addresses and is recaptured
        if (!c->pos2) {
            if (!(dalloc(&c->pos2, (size_t)n) && dalloc(&c->lo2, (size_t)n) &&
                  dalloc(&c->typ2, (size_t)n) && dalloc(&c->oid2, (size_t)n)))
                return fail(LD_ENOMEM, "cannot allocate the second slot arrays");
        }
        HIP_TRY(ld::permute_slots_into(c->sb.keys, n, c->pos, c->lo, c->typ, c->oid, c->pos2,
                                       c->lo2, c->typ2, c->oid2, s));
        std::swap(c->pos, c->pos2);
        std::swap(c->lo, c->lo2);
        std::swap(c->typ, c->typ2);
        std::swap(c->oid, c->oid2);
        c->graph_len = -1;
    }
    // timed: the near-field pair kernels alone
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && !ld::timing_events(c, ld::kTimedNear, &e0, &e1))
        return fail(LD_EHIP, "cannot create timing events");
    if (block) {
        KLAUNCH(k_cell_first, dim3((n + kB - 1) / kB), dim3(kB), s, c->sb.keys, n, M, f->cfirst);
        KLAUNCH(k_block_tiles, dim3(1), dim3(1024), s, f->cfirst, G, f->tiles, f->ntiles);
        if (e0) HIP_TRY(hipEventRecord(e0, s));
        // both walks on the same grid of tiles; the one that does not match
        // the grid's W (known on the device only) leaves at once
        KLAUNCH(k_near_planes, dim3(f->max_tiles), dim3(64 * f->cfg.block), s, c->pos, c->typ,
                c->sb.keys, f->grid, G, f->cfg.block / 2, f->cfirst, f->tiles, f->ntiles, n,
                c->tab, f->Fnear);
        KLAUNCH(k_near_block, dim3(f->max_tiles), dim3(64), s, c->pos, c->typ, c->sb.keys,
                f->grid, G, f->cfg.block / 2, f->cfirst, f->tiles, f->ntiles, n, c->tab, f->Fnear);
        if (e1) HIP_TRY(hipEventRecord(e1, s));
    } else {
        KLAUNCH(k_zero_i, dim3((NC + kB - 1) / kB), dim3(kB), s, f->cstart, NC);
        KLAUNCH(k_zero_i, dim3((NC + kB - 1) / kB), dim3(kB), s, f->cend, NC);
        KLAUNCH(k_cell_ranges, dim3((n + kB - 1) / kB), dim3(kB), s, c->sb.keys, n, f->cstart,
                f->cend);
        const float rc2 = (float)(f->cfg.near_cut * f->cfg.near_cut);
        if (e0) HIP_TRY(hipEventRecord(e0, s));
        KLAUNCH(k_near, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->typ, n, f->grid,
                f->cstart, f->cend, rc2, c->tab, f->Fnear);
        if (e1) HIP_TRY(hipEventRecord(e1, s));
    }
    c->steps_since_sort = 0;
    return LD_OK;
}

// Exact far field into f->Efar for the current slot order (the cell keys of
// the last ff_near sort in block mode).
ld_status ff_far_exact(ld_ctx* c, hipStream_t s) {
    FarField* f = FF(c);
    const int n = (int)c->n;
    if (f->cfg.near_mode == 1) {
        ld_status st = ff_near(c, s);
        if (st != LD_OK) return st;
        KLAUNCH(k_far_exact_block, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->sb.keys, n,
                f->cfg.grid, f->cfg.block / 2, f->Efar);
    } else {
        const float rc2 = (float)(f->cfg.near_cut * f->cfg.near_cut);
        KLAUNCH(k_far_exact, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, n, rc2, f->Efar);
    }
    return LD_OK;
}

ld_status gemm(hipStream_t s, const float* A, int lda, int tA, const float* B, int ldb, int tB,
               float* C, int ldc, int M, int N, int K, const float* bias, int act, float* Z,
               int ldz, int acc, const int* M_dev, float* work = nullptr,
               size_t work_floats = 0, float* colsum_B = nullptr) {
    ld::GemmArgs g{};
    g.work = work; g.work_floats = work_floats;
    g.colsum_B = colsum_B;
    g.A = A; g.lda = lda; g.transA = tA;
    g.B = B; g.ldb = ldb; g.transB = tB;
    g.C = C; g.ldc = ldc;
    g.bias = bias; g.Z = Z; g.ldz = ldz;
    g.M = M; g.N = N; g.K = K;
    g.act = act; g.accumulate = acc; g.M_dev = M_dev;
    HIP_TRY(ld::launch_gemm(g, s));
    return LD_OK;
}

// The learned pair forces of every slot into Fpart[0] (and optional parts).
// boxes: refresh the 64-slot group boxes for the new slot order (not needed
// when the update, which rewrites them, follows).
ld_status ff_learned_forces(ld_ctx* c, hipStream_t s, double* Fc, double* Fm, bool boxes) {
    FarField* f = FF(c);
    const int n = (int)c->n;
    const int G = f->cfg.grid, M = G * G * G, H = f->H;
    ld_status st = ff_near(c, s);
    if (st != LD_OK) return st;
    st = ff_grid_and_coarse(c, s);
    if (st != LD_OK) return st;
    // layer 1, moment part, once per cell (no bias: added per particle)
    if (H == kFH) {
        // normalised moments (as the training snapshots store them) in Xc;
        // block mode: k_moments_sorted wrote them
        if (f->cfg.near_mode != 1)
            KLAUNCH(k_snap_mom, dim3((4 * M + kB - 1) / kB), dim3(kB), s, f->mom, M, f->grid,
                    f->sq, f->Xc);
        if (f->w1bf_stale) {
            KLAUNCH(k_w1_bf16, dim3((kFH * f->Kp + kB - 1) / kB), dim3(kB), s, f->W + f->offW1,
                    f->Kp, f->w1bf);
            f->w1bf_stale = false;
        }
        KLAUNCH(k_cell_layer, dim3((M + 63) / 64), dim3(256), s,
                reinterpret_cast<const float4*>(f->Xc), G, f->cfg.block, f->w1bf, f->Kp, f->Ac);
    } else {
        KLAUNCH(k_cell_features, dim3(M), dim3(kB), s, f->mom, f->occ, f->nocc, G, f->cfg.block,
                f->grid, f->sq, f->Kp, f->Xc);
        st = gemm(s, f->Xc, f->Kp, 0, f->W + f->offW1, H, 0, f->Ac, H, M, H, f->Kp, nullptr, 0,
                  nullptr, 0, 0, f->nocc);
        if (st != LD_OK) return st;
    }
    if (H == kFH) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int groups = (n + kMW * kFW - 1) / (kMW * kFW);
        KLAUNCH(k_mlp_fused, dim3(std::max(1, std::min(groups, 2 * cus))), dim3(kFW * 64), s,
                c->pos,
                c->lo, n, G, f->grid, f->Ac, f->W + f->offW1 + (size_t)(f->K - 3) * H,
                f->W + f->offb1, f->W + f->offW2, f->W + f->offb2, f->W + f->offW3,
                f->W + f->offb3, f->out_scale, f->Fnear, f->Ep, c->Fpart, Fc, Fm);
        if (boxes) HIP_TRY(ld::launch_boxes(c->pos, n, c->box, s));
        return LD_OK;
    }
    KLAUNCH(k_layer1, dim3((unsigned)(((size_t)n * H + kB - 1) / kB)), dim3(kB), s, c->pos, c->lo,
            n, G, f->grid, f->cell2occ, f->Ac,
            f->W + f->offW1 + (size_t)(f->K - 3) * H, f->W + f->offb1, H, f->h1);
    st = gemm(s, f->h1, H, 0, f->W + f->offW2, H, 0, f->h2, H, n, H, H, f->W + f->offb2, 1,
              nullptr, 0, 0, nullptr);
    if (st != LD_OK) return st;
    st = gemm(s, f->h2, H, 0, f->W + f->offW3, f->Op, 0, f->y, f->Op, n, f->Op, H,
              f->W + f->offb3, 0, nullptr, 0, 0, nullptr);
    if (st != LD_OK) return st;
    KLAUNCH(k_combine, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, n, f->Fnear, f->Ep, f->y,
            f->Op, f->out_scale, c->Fpart, Fc, Fm);
    if (boxes) HIP_TRY(ld::launch_boxes(c->pos, n, c->box, s));
    return LD_OK;
}

// Direct pair forces summed into one slot-order array dst [3][n].
ld_status ff_direct_total(ld_ctx* c, hipStream_t s, double* dst) {
    ld::PairLaunch L{};
    L.pos = c->pos; L.lo = c->lo; L.typ = c->typ; L.box = c->box; L.n = (int)c->n;
    L.block = c->tune.block; L.j_split = c->tune.j_split; L.comp = c->tune.comp;
    L.cull = c->tune.cull; L.Fpart = c->Fpart;
    L.nearbits = c->nearbits; L.nb_words = c->nb_words;
    HIP_TRY(ld::launch_pair(L, c->tab, s));
    KLAUNCH(k_sum_parts, dim3((3 * (int)c->n + kB - 1) / kB), dim3(kB), s, c->Fpart,
            c->tune.j_split, (int)c->n, dst);
    return LD_OK;
}

// Median relative error of the learned pair forces against direct summation.
ld_status ff_judge_now(ld_ctx* c, double* med) {
    FarField* f = FF(c);
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    ld_status st = ff_learned_forces(c, s, nullptr, nullptr, true);   // re-sorts, Fpart[0]
    if (st != LD_OK) return st;
    double* Fl = c->work;                  // [3][n]
    double* Fd = c->work + 3 * (size_t)n;  // [3][n]
    HIP_TRY(hipMemcpyAsync(Fl, c->Fpart, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    st = ff_direct_total(c, s, Fd);
    if (st != LD_OK) return st;
    KLAUNCH(k_rel_err, dim3((n + kB - 1) / kB), dim3(kB), s, Fl, Fd, n, f->rel);
    std::vector<double> h(n);
    HIP_TRY(hipMemcpyAsync(h.data(), f->rel, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::nth_element(h.begin(), h.begin() + n / 2, h.end());
    *med = h[n / 2];
    f->last_err = *med;
    ++f->judges;
    return LD_OK;
}

void init_layout(FarField* f) {
    const int B = f->cfg.block;
    f->H = f->cfg.hidden;
    f->K = 4 * B * B * B + 3;
    f->Kp = (f->K + 31) / 32 * 32;
    f->Op = 16;
    size_t o = 0;
    f->offW1 = o; o += (size_t)f->Kp * f->H;
    f->offb1 = o; o += f->H;
    f->offW2 = o; o += (size_t)f->H * f->H;
    f->offb2 = o; o += f->H;
    f->offW3 = o; o += (size_t)f->H * f->Op;
    f->offb3 = o; o += f->Op;
    f->nW = o;
}

ld_status ensure_batch(FarField* f, int B_) {
    if (B_ <= f->batch_cap) return LD_OK;
    float** bufs[] = {&f->bX, &f->bT, &f->bZ1, &f->bA1, &f->bZ2, &f->bA2, &f->bY, &f->bdY,
                      &f->bd2, &f->bd1};
    for (float** b : bufs)
        if (*b) { (void)hipFree(*b); *b = nullptr; }
    if (f->bidx) { (void)hipFree(f->bidx); f->bidx = nullptr; }
    if (f->loss_part) { (void)hipFree(f->loss_part); f->loss_part = nullptr; }
    if (f->gws) { (void)hipFree(f->gws); f->gws = nullptr; }
    const size_t H = f->H;
    // split-K pieces of the largest weight gradient (Kp x H), at most 64
    f->gws_floats = (size_t)64 * f->Kp * H;
    bool ok = dalloc(&f->gws, f->gws_floats) &&
              dalloc(&f->bX, (size_t)B_ * f->Kp) && dalloc(&f->bT, (size_t)B_ * 3) &&
              dalloc(&f->bZ1, B_ * H) && dalloc(&f->bA1, B_ * H) && dalloc(&f->bZ2, B_ * H) &&
              dalloc(&f->bA2, B_ * H) && dalloc(&f->bY, (size_t)B_ * f->Op) &&
              dalloc(&f->bdY, (size_t)B_ * f->Op) && dalloc(&f->bd2, B_ * H) &&
              dalloc(&f->bd1, B_ * H) && dalloc(&f->bidx, (size_t)B_) &&
              dalloc(&f->loss_part, (size_t)B_ * f->Op / kB + 8);
    if (!ok) return fail(LD_ENOMEM, "cannot allocate training batch of %d", B_);
    f->batch_cap = B_;
    return LD_OK;
}

// Forward (saving activations) + loss + backward into f->grad for the batch
// in bX / bT (B_ rows, targets already scaled).  Returns the loss.
ld_status fwd_bwd(FarField* f, int B_, hipStream_t s, double* loss) {
    const int H = f->H, Op = f->Op, Kp = f->Kp;
    float* W = f->W;
    float* gW = f->grad;
    ld_status st;
#define TRY(x) do { st = (x); if (st != LD_OK) return st; } while (0)
    TRY(gemm(s, f->bX, Kp, 0, W + f->offW1, H, 0, f->bA1, H, B_, H, Kp, W + f->offb1, 1, f->bZ1,
             H, 0, nullptr));
    TRY(gemm(s, f->bA1, H, 0, W + f->offW2, H, 0, f->bA2, H, B_, H, H, W + f->offb2, 1, f->bZ2,
             H, 0, nullptr));
    TRY(gemm(s, f->bA2, H, 0, W + f->offW3, Op, 0, f->bY, Op, B_, Op, H, W + f->offb3, 0,
             nullptr, 0, 0, nullptr));
    int nparts = 0;
    HIP_TRY(ld::launch_mse(f->bY, Op, f->bT, B_, 3, f->bdY, f->loss_part, &nparts, s));
    // layer 3: weight and bias gradients in one product (the bias gradient
    // is the column sums of dY), then dA2 times SiLU'(Z2) in its epilogue
    TRY(gemm(s, f->bA2, H, 1, f->bdY, Op, 0, gW + f->offW3, Op, H, Op, B_, nullptr, 0, nullptr, 0,
             0, nullptr, f->gws, f->gws_floats, gW + f->offb3));
    TRY(gemm(s, f->bdY, Op, 0, W + f->offW3, Op, 1, f->bd2, H, B_, H, Op, nullptr, 2, f->bZ2, H, 0,
             nullptr));
    // layer 2
    TRY(gemm(s, f->bA1, H, 1, f->bd2, H, 0, gW + f->offW2, H, H, H, B_, nullptr, 0, nullptr, 0, 0,
             nullptr, f->gws, f->gws_floats, gW + f->offb2));
    TRY(gemm(s, f->bd2, H, 0, W + f->offW2, H, 1, f->bd1, H, B_, H, H, nullptr, 2, f->bZ1, H, 0,
             nullptr));
    // layer 1
    TRY(gemm(s, f->bX, Kp, 1, f->bd1, H, 0, gW + f->offW1, H, Kp, H, B_, nullptr, 0, nullptr, 0, 0,
             nullptr, f->gws, f->gws_floats, gW + f->offb1));
#undef TRY
    if (loss) {
        std::vector<double> parts(nparts);
        HIP_TRY(hipMemcpyAsync(parts.data(), f->loss_part, sizeof(double) * nparts,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double l = 0.0;
        for (double v : parts) l += v;
        *loss = l;
    }
    return LD_OK;
}

// Philox4x32-10 on the host for training shuffles (stream tag 3).
uint32_t philox_word(uint64_t seed, uint64_t ctr, int word) {
    uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = 0u, c3 = 3u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    const uint32_t w[4] = {c0, c1, c2, c3};
    return w[word & 3];
}

}  // namespace

namespace ld {

void ff_free(ld_ctx* c) {
    if (!c->ff) return;
    ff_free_bufs(c->ff);
    delete c->ff;
    c->ff = nullptr;
}

bool ff_active(const ld_ctx* c) { return c->ff && c->ff->mode != 0; }

ld_status ff_step_forces(ld_ctx* c, hipStream_t s, int* j_split_used) {
    FarField* f = c->ff;
    if (f->mode == 2 && f->window_steps % f->cfg.judge_every == 0) {
        double med = 0.0;
        ld_status st = ff_judge_now(c, &med);
        if (st != LD_OK) return st;
        f->active = med <= f->cfg.judge_tol;
        if (!f->active) ++f->fallbacks;
    }
    ++f->window_steps;
    if (f->mode == 1 || f->active) {
        // the update that follows rewrites the group boxes
        ld_status st = ff_learned_forces(c, s, nullptr, nullptr, false);
        if (st != LD_OK) return st;
        *j_split_used = 1;
        ++f->learned_steps;
    } else {
        ld::PairLaunch L{};
        L.pos = c->pos; L.lo = c->lo; L.typ = c->typ; L.box = c->box; L.n = (int)c->n;
        L.block = c->tune.block; L.j_split = c->tune.j_split; L.comp = c->tune.comp;
        L.cull = c->tune.cull; L.Fpart = c->Fpart;
        HIP_TRY(ld::launch_pair(L, c->tab, s));
        *j_split_used = c->tune.j_split;
        ++f->direct_steps;
    }
    return LD_OK;
}

}  // namespace ld

extern "C" {

ld_status ld_ff_enable(ld_ctx* c, const ld_ff_config* cfg) {
    g_err.clear();
    if (!c || !cfg) return fail(LD_EINVAL, "ctx and cfg are required");
    if (c->pm) return fail(LD_ESTATE, "the paper's scheme is enabled (ld_paper_disable first)");
    if (!(cfg->near_cut > 0.0)) return fail(LD_EINVAL, "near_cut must be positive");
    if (cfg->grid < 4 || cfg->grid > 64) return fail(LD_EINVAL, "grid must be in [4, 64]");
    if (cfg->block < 1 || cfg->block > 7 || cfg->block % 2 == 0)
        return fail(LD_EINVAL, "block must be odd, 1..7");
    if (cfg->hidden < 16 || cfg->hidden > 256 || cfg->hidden % 16)
        return fail(LD_EINVAL, "hidden must be a multiple of 16 in [16, 256]");
    if (cfg->judge_every < 1) return fail(LD_EINVAL, "judge_every must be >= 1");
    if (!(cfg->judge_tol > 0.0)) return fail(LD_EINVAL, "judge_tol must be positive");
    if (cfg->near_mode != 0 && cfg->near_mode != 1)
        return fail(LD_EINVAL, "near_mode must be 0 (radial) or 1 (block)");
    if (cfg->parent_reach < 0 || cfg->parent_reach > 31)
        return fail(LD_EINVAL, "parent_reach must be in [0, 31]");
    if (cfg->near_mode == 1 && cfg->parent_reach > 0 && cfg->grid % 2)
        return fail(LD_EINVAL, "the two-level expansion (parent_reach > 0) needs an even grid");
    double maxlj = 0.0;
    for (int a = 0; a < c->p.n_types; ++a)
        for (int b = 0; b < c->p.n_types; ++b)
            maxlj = std::max(maxlj, c->p.lj_cut * 0.5 * (c->p.sigma[a] + c->p.sigma[b]));
    if (cfg->near_mode == 0 && cfg->near_cut < maxlj)
        return fail(LD_EINVAL, "near_cut %.3g is below the largest LJ range %.3g", cfg->near_cut,
                    maxlj);
    HIP_TRY(hipStreamSynchronize(c->stream));
    ld::ff_free(c);
    FarField* f = new (std::nothrow) FarField();
    if (!f) return fail(LD_ENOMEM, "host allocation failed");
    f->cfg = *cfg;
    f->rlj = maxlj;
    init_layout(f);
    // source splits of the local expansion: up to 16, partials within 128 MB
    {
        const size_t Mc = (size_t)cfg->grid * cfg->grid * cfg->grid;
        const size_t cap = ((size_t)128 << 20) / (sizeof(double) * kLoc * Mc);
        f->loc_split = (int)std::max<size_t>(1, std::min<size_t>(16, cap));
    }
    const size_t n = (size_t)c->n;
    const size_t M = (size_t)cfg->grid * cfg->grid * cfg->grid;
    const size_t NC = (size_t)kMaxNearCells * kMaxNearCells * kMaxNearCells;
    double qmax = 0.0;
    {
        std::vector<float4> h(n);
        HIP_TRY(hipMemcpy(h.data(), c->pos, sizeof(float4) * n, hipMemcpyDeviceToHost));
        for (const float4& v : h) qmax = std::max(qmax, (double)std::fabs(v.w));
    }
    f->sq = (float)(qmax > 0.0 ? qmax : 1.0);
    bool ok = dalloc(&f->grid, 1) && dalloc(&f->cstart, NC) && dalloc(&f->cend, NC) &&
              dalloc(&f->Fnear, 3 * n) && dalloc(&f->mom, 4 * M) && dalloc(&f->count, M) &&
              dalloc(&f->occ, M) && dalloc(&f->cell2occ, M) && dalloc(&f->nocc, 1) &&
              dalloc(&f->Ecell, kLoc * M) && dalloc(&f->Ep, 3 * n) && dalloc(&f->cfirst, M + 1) &&
              dalloc(&f->tiles, (n + 63) / 64 + (size_t)cfg->grid * cfg->grid) &&
              dalloc(&f->ntiles, 1) &&
              dalloc(&f->loc_part, (size_t)f->loc_split * M * kLoc) &&
              dalloc(&f->pmom, 4 * (M / 8 + 1)) && dalloc(&f->pcount, M / 8 + 1) &&
              dalloc(&f->pocc, M / 8 + 1) && dalloc(&f->pcell2occ, M / 8 + 1) &&
              dalloc(&f->npocc, 1) &&
              dalloc(&f->Xc, M * f->Kp) && dalloc(&f->Ac, M * f->H) &&
              dalloc(&f->h1, n * f->H) && dalloc(&f->h2, n * f->H) && dalloc(&f->y, n * f->Op) &&
              dalloc(&f->W, f->nW) && dalloc(&f->grad, f->nW) && dalloc(&f->adam_m, f->nW) &&
              dalloc(&f->adam_v, f->nW) && dalloc(&f->rel, n) && dalloc(&f->Efar, 3 * n) &&
              dalloc(&f->w1bf, f->H == kFH ? (size_t)kFH * f->Kp : 1);
    if (ok && cfg->near_mode == 1 && cfg->parent_reach == 0 && cfg->grid <= kConvMaxGrid) {
        ok = conv_setup(&f->conv, cfg->block, c->stream) == hipSuccess;
        f->use_conv = ok;
    }
    if (!ok) {
        ff_free_bufs(f);
        delete f;
        return fail(LD_ENOMEM, "cannot allocate the learned far field");
    }
    // deterministic small initial weights (Philox, tag 3), zero biases
    std::vector<float> w(f->nW, 0.f);
    auto init = [&](size_t off, int rows, int valid_rows, int cols, int valid_cols, double sc) {
        for (int r = 0; r < valid_rows; ++r)
            for (int q = 0; q < valid_cols; ++q) {
                const uint64_t k = off + (size_t)r * cols + q;
                const double u = ((philox_word(0x5EEDull, k, 0) >> 9) + 0.5) / 8388608.0;
                w[off + (size_t)r * cols + q] = (float)((2.0 * u - 1.0) * sc);
            }
        (void)rows;
    };
    init(f->offW1, f->Kp, f->K, f->H, f->H, std::sqrt(3.0 / f->K));
    init(f->offW2, f->H, f->H, f->H, f->H, std::sqrt(3.0 / f->H));
    init(f->offW3, f->H, f->H, f->Op, 3, std::sqrt(3.0 / f->H) * 0.1);
    HIP_TRY(hipMemcpy(f->W, w.data(), sizeof(float) * f->nW, hipMemcpyHostToDevice));
    std::vector<float> zero(f->nW, 0.f);
    HIP_TRY(hipMemcpy(f->adam_m, zero.data(), sizeof(float) * f->nW, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->adam_v, zero.data(), sizeof(float) * f->nW, hipMemcpyHostToDevice));
    f->max_tiles = (int)((n + 63) / 64 + (size_t)cfg->grid * cfg->grid);
    f->out_scale = 1.f;
    f->mode = 0;
    c->ff = f;
    return LD_OK;
}

ld_status ld_ff_mode(ld_ctx* c, int32_t mode) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (mode < 0 || mode > 2) return fail(LD_EINVAL, "mode must be 0, 1 or 2");
    if (mode != 0 && !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (mode != 0 && c->pm) return fail(LD_ESTATE, "the paper's scheme is enabled");
    if (c->ff) {
        c->ff->mode = mode;
        c->ff->window_steps = 0;
        c->ff->active = true;
    }
    return LD_OK;
}

int64_t ld_ff_weights_size(ld_ctx* c) { return (c && c->ff) ? (int64_t)c->ff->nW : 0; }

ld_status ld_ff_set_weights(ld_ctx* c, const float* w, int64_t count, double sq,
                            double out_scale) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (!w || count != (int64_t)c->ff->nW)
        return fail(LD_EINVAL, "weights need exactly %lld floats", (long long)c->ff->nW);
    if (!(sq > 0.0) || !(out_scale >= 0.0) || !std::isfinite(out_scale))
        return fail(LD_EINVAL, "sq must be positive and out_scale >= 0 (0: network off)");
    HIP_TRY(copy_in(c->ff->W, w, sizeof(float) * count, c->stream));
    c->ff->w1bf_stale = true;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ff->sq = (float)sq;
    c->ff->out_scale = (float)out_scale;
    return LD_OK;
}

ld_status ld_ff_get_weights(ld_ctx* c, float* w, int64_t count, double* sq, double* out_scale) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (w) {
        if (count != (int64_t)c->ff->nW)
            return fail(LD_EINVAL, "weights need exactly %lld floats", (long long)c->ff->nW);
        HIP_TRY(copy_out(w, c->ff->W, sizeof(float) * count, c->stream));
    }
    if (sq) *sq = c->ff->sq;
    if (out_scale) *out_scale = c->ff->out_scale;
    return LD_OK;
}

// Model file: "LDFFW001", int32 grid, block, hidden, near_mode, parent_reach,
// reserved; FP64 near_cut, sq, out_scale; int64 count; FP32 weights[count].
ld_status ld_ff_save(ld_ctx* c, const char* path) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (!path) return fail(LD_EINVAL, "path is NULL");
    FarField* f = c->ff;
    std::vector<float> w(f->nW);
    HIP_TRY(copy_out(w.data(), f->W, sizeof(float) * w.size(), c->stream));
    const int32_t hdr[6] = {f->cfg.grid, f->cfg.block, f->cfg.hidden, f->cfg.near_mode,
                            f->cfg.parent_reach, 0};
    const double dv[3] = {f->cfg.near_cut, (double)f->sq, (double)f->out_scale};
    const int64_t count = (int64_t)w.size();
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(LD_EINVAL, "cannot open %s for writing", path);
    const bool ok = std::fwrite("LDFFW001", 1, 8, fp) == 8 && std::fwrite(hdr, 4, 6, fp) == 6 &&
                    std::fwrite(dv, 8, 3, fp) == 3 && std::fwrite(&count, 8, 1, fp) == 1 &&
                    std::fwrite(w.data(), 4, w.size(), fp) == w.size();
    const bool closed = std::fclose(fp) == 0;
    if (!ok || !closed) return fail(LD_EINVAL, "writing %s failed", path);
    return LD_OK;
}

ld_status ld_ff_load(ld_ctx* c, const char* path) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (!path) return fail(LD_EINVAL, "path is NULL");
    FarField* f = c->ff;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(LD_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t hdr[6];
    double dv[3];
    int64_t count = 0;
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "LDFFW001", 8) == 0 &&
              std::fread(hdr, 4, 6, fp) == 6 && std::fread(dv, 8, 3, fp) == 3 &&
              std::fread(&count, 8, 1, fp) == 1;
    if (!ok) {
        std::fclose(fp);
        return fail(LD_EINVAL, "%s is not a model file", path);
    }
    if (hdr[0] != f->cfg.grid || hdr[1] != f->cfg.block || hdr[2] != f->cfg.hidden ||
        hdr[3] != f->cfg.near_mode || hdr[4] != f->cfg.parent_reach ||
        (f->cfg.near_mode == 0 && dv[0] != f->cfg.near_cut) || count != (int64_t)f->nW) {
        std::fclose(fp);
        return fail(LD_EINVAL,
                    "%s holds a model for grid %d, block %d, hidden %d, near mode %d, parent "
                    "reach %d (near cut %g), not this configuration",
                    path, hdr[0], hdr[1], hdr[2], hdr[3], hdr[4], dv[0]);
    }
    std::vector<float> w((size_t)count);
    ok = std::fread(w.data(), 4, w.size(), fp) == w.size();
    std::fclose(fp);
    if (!ok) return fail(LD_EINVAL, "%s is truncated", path);
    return ld_ff_set_weights(c, w.data(), count, dv[1], dv[2]);
}

ld_status ld_ff_grid(ld_ctx* c, double* L, int32_t* near_cells) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    hipStream_t s = c->stream;
    KLAUNCH(k_absmax_part, dim3(64), dim3(kB), s, c->pos, (int)c->n, c->sb.bounds_part);
    KLAUNCH(k_grid, dim3(1), dim3(1), s, c->sb.bounds_part, 64, c->ff->cfg.near_cut,
            c->ff->cfg.grid, c->ff->cfg.near_mode, c->ff->cfg.block, c->ff->rlj, c->ff->grid);
    FFGrid g;
    HIP_TRY(copy_out(&g, c->ff->grid, sizeof g, s));
    if (L) *L = g.L;
    if (near_cells) *near_cells = g.Gn;
    return LD_OK;
}

ld_status ld_ff_forces(ld_ctx* c, int32_t part, double* out) {
    g_err.clear();
    if (!c || !c->ff || !out) return fail(LD_EINVAL, "ctx (with ld_ff_enable) and out required");
    if (part < 0 || part > 4) return fail(LD_EINVAL, "part must be 0..4");
    FarField* f = c->ff;
    hipStream_t s = c->stream;
    const int n = (int)c->n;
    double* Fc = c->work;                    // [3][n]
    double* Fm = c->work + 3 * (size_t)n;    // [3][n]
    double* dst = c->work + 6 * (size_t)n;   // [3n] original order
    const double* src = nullptr;
    if (part == 4) {
        ld_status st = ff_far_exact(c, s);
        if (st != LD_OK) return st;
        KLAUNCH(k_q_times, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, n, f->Efar, Fc);
        src = Fc;
    } else {
        ld_status st = ff_learned_forces(c, s, Fc, Fm, true);
        if (st != LD_OK) return st;
        src = part == 0 ? f->Fnear : part == 1 ? Fc : part == 2 ? Fm : c->Fpart;
    }
    KLAUNCH(k_to_orig, dim3((n + kB - 1) / kB), dim3(kB), s, src, c->oid, n, dst);
    HIP_TRY(copy_out(out, dst, sizeof(double) * 3 * n, s));
    return LD_OK;
}

ld_status ld_ff_mlp(ld_ctx* c, const float* X, int64_t m, float* Y) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (!X || !Y || m < 1 || m > (1 << 22)) return fail(LD_EINVAL, "X, Y and 1 <= m <= 2^22");
    FarField* f = c->ff;
    hipStream_t s = c->stream;
    ld_status st = ensure_batch(f, (int)m);
    if (st != LD_OK) return st;
    // stage the caller's m x K rows, then pad to Kp
    float* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, sizeof(float) * (size_t)m * f->K));
    hipError_t e = copy_in(tmp, X, sizeof(float) * (size_t)m * f->K, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)m), dim3(kB), 0, s, tmp, (int)m, f->K, f->Kp,
                           f->bX);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(LD_EHIP, "staging features: %s", hipGetErrorString(e));
    const int H = f->H, Op = f->Op;
    st = gemm(s, f->bX, f->Kp, 0, f->W + f->offW1, H, 0, f->bA1, H, (int)m, H, f->Kp,
              f->W + f->offb1, 1, nullptr, 0, 0, nullptr);
    if (st == LD_OK)
        st = gemm(s, f->bA1, H, 0, f->W + f->offW2, H, 0, f->bA2, H, (int)m, H, H, f->W + f->offb2,
                  1, nullptr, 0, 0, nullptr);
    if (st == LD_OK)
        st = gemm(s, f->bA2, H, 0, f->W + f->offW3, Op, 0, f->bY, Op, (int)m, Op, H,
                  f->W + f->offb3, 0, nullptr, 0, 0, nullptr);
    if (st != LD_OK) return st;
    std::vector<float> y((size_t)m * Op), o((size_t)m * 3);
    HIP_TRY(hipMemcpyAsync(y.data(), f->bY, sizeof(float) * y.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t r = 0; r < m; ++r)
        for (int k = 0; k < 3; ++k) o[3 * r + k] = y[r * Op + k];
    HIP_TRY(put_out(Y, o.data(), sizeof(float) * o.size(), s));
    return LD_OK;
}

ld_status ld_ff_grads(ld_ctx* c, const float* X, const float* T, int64_t m, float* grads,
                      double* loss) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (!X || !T || !grads || m < 1 || m > (1 << 20))
        return fail(LD_EINVAL, "X, T, grads and 1 <= m <= 2^20 required");
    FarField* f = c->ff;
    hipStream_t s = c->stream;
    ld_status st = ensure_batch(f, (int)m);
    if (st != LD_OK) return st;
    float* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, sizeof(float) * (size_t)m * f->K));
    hipError_t e = copy_in(tmp, X, sizeof(float) * (size_t)m * f->K, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)m), dim3(kB), 0, s, tmp, (int)m, f->K, f->Kp,
                           f->bX);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = copy_in(f->bT, T, sizeof(float) * (size_t)m * 3, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(LD_EHIP, "staging batch: %s", hipGetErrorString(e));
    st = fwd_bwd(f, (int)m, s, loss);
    if (st != LD_OK) return st;
    HIP_TRY(copy_out(grads, f->grad, sizeof(float) * f->nW, s));
    return LD_OK;
}

ld_status ld_ff_collect(ld_ctx* c, int32_t reset, int32_t max_snapshots) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    FarField* f = c->ff;
    hipStream_t s = c->stream;
    const int n = (int)c->n;
    const int G = f->cfg.grid, M = G * G * G;
    if (reset || !f->s_snap) {
        const int cap = std::max(1, max_snapshots);
        if (f->snap_mom) { (void)hipFree(f->snap_mom); f->snap_mom = nullptr; }
        int** ib[] = {&f->s_snap, &f->s_cell};
        for (int** b : ib)
            if (*b) { (void)hipFree(*b); *b = nullptr; }
        float** fb[] = {&f->s_off, &f->s_tgt};
        for (float** b : fb)
            if (*b) { (void)hipFree(*b); *b = nullptr; }
        f->snap_cap = cap;
        f->sample_cap = (int64_t)cap * n;
        if (!(dalloc(&f->snap_mom, (size_t)cap * 4 * M) && dalloc(&f->s_snap, f->sample_cap) &&
              dalloc(&f->s_cell, f->sample_cap) && dalloc(&f->s_off, 3 * f->sample_cap) &&
              dalloc(&f->s_tgt, 3 * f->sample_cap)))
            return fail(LD_ENOMEM, "cannot allocate %d training snapshots", cap);
        f->snaps = 0;
        f->samples = 0;
    }
    if (f->snaps >= f->snap_cap) return fail(LD_ESTATE, "training store is full");
    // the far field is judged on the same cell assignment as inference
    ld_status st = ff_near(c, s);
    if (st != LD_OK) return st;
    st = ff_grid_and_coarse(c, s);
    if (st != LD_OK) return st;
    st = ff_far_exact(c, s);
    if (st != LD_OK) return st;
    KLAUNCH(k_snap_mom, dim3((4 * M + kB - 1) / kB), dim3(kB), s, f->mom, M, f->grid, f->sq,
            f->snap_mom + (size_t)f->snaps * 4 * M);
    KLAUNCH(k_collect, dim3((n + kB - 1) / kB), dim3(kB), s, c->pos, c->lo, n, G, f->grid,
            f->Efar, f->Ep, f->snaps, f->samples, f->s_snap, f->s_cell, f->s_off, f->s_tgt);
    HIP_TRY(hipStreamSynchronize(s));
    f->snaps += 1;
    f->samples += n;
    return LD_OK;
}

ld_status ld_ff_train(ld_ctx* c, const ld_ff_train_cfg* tc, ld_ff_train_report* rep) {
    g_err.clear();
    if (!c || !c->ff || !tc) return fail(LD_EINVAL, "ctx (with ld_ff_enable) and cfg required");
    FarField* f = c->ff;
    if (f->samples < 2) return fail(LD_ESTATE, "collect training snapshots first");
    if (tc->epochs < 0 || tc->batch < 16 || tc->batch > (1 << 16) || !(tc->lr > 0.0))
        return fail(LD_EINVAL, "epochs >= 0, 16 <= batch <= 65536, lr > 0");
    if (!(tc->val_fraction >= 0.0 && tc->val_fraction < 0.9))
        return fail(LD_EINVAL, "val_fraction in [0, 0.9)");
    hipStream_t s = c->stream;
    const int B_ = tc->batch;
    ld_status st = ensure_batch(f, B_);
    if (st != LD_OK) return st;
    // output scale: RMS of the targets
    std::vector<float> tg(3 * (size_t)f->samples);
    HIP_TRY(hipMemcpyAsync(tg.data(), f->s_tgt, sizeof(float) * tg.size(), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    double ss = 0.0;
    for (float v : tg) ss += (double)v * v;
    const double rms = std::sqrt(ss / (double)tg.size());
    if (tc->reset_scale || f->out_scale == 1.f || !(f->out_scale > 0.f))
        f->out_scale = (float)(rms > 0.0 ? rms : 1.0);
    const float inv_scale = 1.0f / f->out_scale;
    // split: the last val_fraction of the samples is held out
    const int64_t nval = (int64_t)(tc->val_fraction * (double)f->samples);
    const int64_t ntr = f->samples - nval;
    std::vector<int> perm(ntr);
    for (int64_t k = 0; k < ntr; ++k) perm[k] = (int)k;
    // Each epoch's permutation is uploaded from one of two pinned host
    // buffers into one of two device buffers, stream-ordered before the
    // epoch's batches, so the host shuffles epoch e + 1 while the GPU trains
    // on epoch e; a host buffer is refilled only after its last copy ended.
    const size_t pcount = (size_t)std::max<int64_t>(std::max<int64_t>(ntr, 1), B_);
    int* dperm_buf[2] = {nullptr, nullptr};
    int* hperm[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    auto release = [&]() {
        for (int k = 0; k < 2; ++k) {
            if (dperm_buf[k]) (void)hipFree(dperm_buf[k]);
            if (hperm[k]) (void)hipHostFree(hperm[k]);
            if (copied[k]) (void)hipEventDestroy(copied[k]);
        }
    };
    for (int k = 0; k < 2; ++k) {
        if (hipMalloc(&dperm_buf[k], sizeof(int) * pcount) != hipSuccess ||
            hipHostMalloc(&hperm[k], sizeof(int) * pcount) != hipSuccess ||
            hipEventCreateWithFlags(&copied[k], hipEventDisableTiming) != hipSuccess) {
            release();
            return fail(LD_ENOMEM, "cannot allocate the batch permutations");
        }
    }
    int* dperm = dperm_buf[0];
    double last = 0.0;
    int64_t iters = 0;
    const int G = f->cfg.grid;
    for (int ep = 0; ep < tc->epochs && st == LD_OK; ++ep) {
        // Fisher-Yates with Philox words (stream tag 3), applied to the
        // previous epoch's order
        for (int64_t k = ntr - 1; k > 0; --k) {
            const uint64_t ctr = ((uint64_t)ep << 40) ^ (uint64_t)k;
            const int64_t j = (int64_t)(philox_word(tc->seed, ctr, 0) % (uint64_t)(k + 1));
            std::swap(perm[k], perm[j]);
        }
        const int slot = ep & 1;
        if (hipEventSynchronize(copied[slot]) != hipSuccess) {     // its last copy is done
            st = fail(LD_EHIP, "wait for a permutation copy");
            break;
        }
        std::memcpy(hperm[slot], perm.data(), sizeof(int) * ntr);
        dperm = dperm_buf[slot];
        if (hipMemcpyAsync(dperm, hperm[slot], sizeof(int) * ntr, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipEventRecord(copied[slot], s) != hipSuccess) {
            st = fail(LD_EHIP, "upload permutation");
            break;
        }
        double ep_loss = 0.0;
        int nb = 0;
        for (int64_t b0 = 0; b0 + B_ <= ntr && st == LD_OK; b0 += B_) {
            hipLaunchKernelGGL(k_gather_batch, dim3(B_), dim3(kB), 0, s, dperm + b0, B_, f->s_snap,
                               f->s_cell, f->s_off, f->s_tgt, f->snap_mom, G, f->cfg.block, f->Kp,
                               inv_scale, f->bX, f->bT);
            if (hipGetLastError() != hipSuccess) { st = fail(LD_EHIP, "gather"); break; }
            double l = 0.0;
            // the reported loss is the last batch's of the last epoch (reading
            // it waits for the GPU, so no other batch reads it back)
            const bool want = ep + 1 == tc->epochs && b0 + 2 * B_ > ntr;
            st = fwd_bwd(f, B_, s, want ? &l : nullptr);
            if (st != LD_OK) break;
            ++f->adam_step;
            f->w1bf_stale = true;
            if (ld::launch_adam(f->W, f->grad, f->adam_m, f->adam_v, (int)f->nW, (float)tc->lr,
                                f->adam_step, s) != hipSuccess) {
                st = fail(LD_EHIP, "adam");
                break;
            }
            if (want) { ep_loss = l; nb = 1; }
            ++iters;
        }
        if (nb) last = ep_loss;
    }
    // validation: relative RMS error of the residual on the held-out samples,
    // and the least-squares gain of the output there (sums of y t, y y, t t)
    double val_rel = NAN, val_raw = NAN, gain = 1.0;
    if (st == LD_OK && nval >= 16) {
        double num = 0.0, den = 0.0, sty = 0.0, syy = 0.0;
        std::vector<int> vidx;
        for (int64_t k = ntr; k < f->samples; ++k) vidx.push_back((int)k);
        for (size_t v0 = 0; v0 + 16 <= vidx.size() && st == LD_OK; v0 += B_) {
            const int bsz = (int)std::min<size_t>(B_, vidx.size() - v0);
            if (hipMemcpyAsync(dperm, vidx.data() + v0, sizeof(int) * bsz, hipMemcpyHostToDevice,
                               s) != hipSuccess) { st = fail(LD_EHIP, "upload"); break; }
            hipLaunchKernelGGL(k_gather_batch, dim3(bsz), dim3(kB), 0, s, dperm, bsz, f->s_snap,
                               f->s_cell, f->s_off, f->s_tgt, f->snap_mom, G, f->cfg.block, f->Kp,
                               inv_scale, f->bX, f->bT);
            const int H = f->H, Op = f->Op;
            st = gemm(s, f->bX, f->Kp, 0, f->W + f->offW1, H, 0, f->bA1, H, bsz, H, f->Kp,
                      f->W + f->offb1, 1, nullptr, 0, 0, nullptr);
            if (st == LD_OK)
                st = gemm(s, f->bA1, H, 0, f->W + f->offW2, H, 0, f->bA2, H, bsz, H, H,
                          f->W + f->offb2, 1, nullptr, 0, 0, nullptr);
            if (st == LD_OK)
                st = gemm(s, f->bA2, H, 0, f->W + f->offW3, Op, 0, f->bY, Op, bsz, Op, H,
                          f->W + f->offb3, 0, nullptr, 0, 0, nullptr);
            if (st != LD_OK) break;
            std::vector<float> y((size_t)bsz * Op), t((size_t)bsz * 3);
            if (hipMemcpyAsync(y.data(), f->bY, sizeof(float) * y.size(), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipMemcpyAsync(t.data(), f->bT, sizeof(float) * t.size(), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) { st = fail(LD_EHIP, "readback"); break; }
            for (int r = 0; r < bsz; ++r)
                for (int k = 0; k < 3; ++k) {
                    const double yv = (double)y[(size_t)r * Op + k], tv = t[3 * r + k];
                    const double d = yv - tv;
                    num += d * d;
                    den += tv * tv;
                    sty += yv * tv;
                    syy += yv * yv;
                }
        }
        if (den > 0.0) {
            val_raw = std::sqrt(num / den);
            val_rel = val_raw;
            if (tc->calibrate) {
                gain = syy > 0.0 ? std::min(1.0, std::max(0.0, sty / syy)) : 0.0;
                val_rel = std::sqrt(std::max(0.0, den - 2.0 * gain * sty + gain * gain * syy) / den);
                f->out_scale = (float)((double)f->out_scale * gain);
            }
        }
    }
    (void)hipStreamSynchronize(s);
    release();
    if (st != LD_OK) return st;
    if (rep) {
        rep->samples = f->samples;
        rep->iterations = iters;
        rep->final_loss = last;
        rep->val_rel_rms = val_rel;
        rep->out_scale = f->out_scale;
        rep->gain = gain;
        rep->val_rel_rms_raw = val_raw;
    }
    return LD_OK;
}

ld_status ld_ff_judge(ld_ctx* c, double* median_rel_err) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    double med = 0.0;
    ld_status st = ff_judge_now(c, &med);
    if (st != LD_OK) return st;
    if (median_rel_err) *median_rel_err = med;
    return LD_OK;
}

ld_status ld_ff_stats(ld_ctx* c, int64_t out[4], double* last_err) {
    g_err.clear();
    if (!c || !c->ff) return fail(LD_ESTATE, "ld_ff_enable first");
    if (out) {
        out[0] = c->ff->judges;
        out[1] = c->ff->fallbacks;
        out[2] = c->ff->learned_steps;
        out[3] = c->ff->direct_steps;
    }
    if (last_err) *last_err = c->ff->last_err;
    return LD_OK;
}

}  // extern "C"
