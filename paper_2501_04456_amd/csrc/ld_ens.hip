// Ensembles of independent droplets in one persistent launch.
//
// Every droplet d owns a contiguous slot range [off[d], off[d+1]) with its own
// parameters, radius schedule and noise seed.  The pair sum is split into
// work items (droplet, 64-particle i tile); an item costs 64 x N_d pairs.
// Items are ordered longest first and pulled from one atomic counter by
// resident wavefronts, so a few large droplets cannot leave the chip idle at
// the end of the step.  Each wavefront stages j tiles of its item's droplet
// in its own LDS slice.  The update runs over all slots of all droplets in
// one launch.  A droplet's noise is keyed by its seed and the particle's
// index inside the droplet, so each droplet follows exactly the stream it
// would follow alone.
//
// Every sort interval each droplet's slots are re-ordered along a Hilbert
// curve over the droplet's own bounding cube (uncharged particles last), and
// every step each 64-slot tile of a droplet gets a bounding box and a charged
// flag.  The pair kernel then treats a pair of tiles like the single-droplet
// kernel treats a pair of groups: careful loop when the boxes come within the
// largest LJ range, Coulomb-only loop when they do not, nothing when one
// side is uncharged.  In the careful loop both sides' positions are taken
// relative to the centre of the i tile's box, (hi - c) + lo rounded to FP32,
// so a pair difference carries the rounding of a coordinate tens of sigma
// from c rather than of |x|.  Outputs are mapped back to the original order
// through the per-droplet index, which travels with the particle.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <new>

#include "ld_host.h"
#include "ld_pair_core.h"
#include "ld_update_core.h"

using namespace ld;
using namespace ld::host;

namespace {

constexpr int kWaves = 4;                 // wavefronts per workgroup
constexpr int kEnsBlock = kWaves * kGroup;
constexpr int kEnsSortEvery = 50;         // sort interval without graphs

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void k_ens_reset(unsigned* counter) { *counter = 0u; }

// The careful loop works on positions relative to the tile box's centre when
// the box is compact (half-extent below kRelReach sigma: |x - c| < 256 sigma,
// so (hi - c) + lo carries at most two FP32 roundings of 2^-17 sigma); a box
// stretched by NPs thrown far out keeps the exact (hi, lo) differences.
constexpr float kRelReach = 255.f;

__device__ __forceinline__ bool tile_compact(const Box& b) {
    const float ext = fmaxf(fmaxf(b.hi.x - b.lo.x, b.hi.y - b.lo.y), b.hi.z - b.lo.z);
    return ext < 2.f * kRelReach;           // false for NaN or infinite boxes too
}

template <int COMP, bool CULL, int UNROLL>
__global__ __launch_bounds__(kEnsBlock, 5) void k_ens_pair(
    const float4* __restrict__ pos, const float4* __restrict__ lo, const int* __restrict__ typ,
    const int* __restrict__ off, const int2* __restrict__ items, int W, unsigned* counter, const PairTable* __restrict__ tabs,
    const Box* __restrict__ box, const int* __restrict__ tbase, double* __restrict__ F,
    int total, unsigned* __restrict__ nearbits, int nb_words) {
    __shared__ float4 sp[kWaves][kGroup];
    __shared__ float4 sl[kWaves][kGroup];          // low words (stretched tiles only)
    const int w = threadIdx.x / kGroup;
    const int lane = threadIdx.x % kGroup;
    for (;;) {
        unsigned item = 0u;
        if (lane == 0) item = atomicAdd(counter, 1u);
        item = (unsigned)__shfl((int)item, 0);
        if (item >= (unsigned)W) break;
        const int2 it = items[item];
        const int d = it.x;
        const int o = off[d];
        const int nd = off[d + 1] - o;
        const float rc2max = tabs[d].rc2max;
        const int i = it.y + lane;
        const bool live = i < nd;
        const float4 pi = live ? pos[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 li = live ? lo[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        pair::Acc a;
        Box bi;
        const int t0 = tbase[d];
        // origin of the near tiles' positions: the centre of the tile's box,
        // else its first particle
        float4 c = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.x))),
                               __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.y))),
                               __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.z))),
                               0.f);
        bool rel = false;
        if constexpr (CULL) {
            bi = box[t0 + it.y / kGroup];
            c = make_float4(0.5f * (bi.lo.x + bi.hi.x), 0.5f * (bi.lo.y + bi.hi.y),
                            0.5f * (bi.lo.z + bi.hi.z), 0.f);
            rel = tile_compact(bi);
        }
        const float4 pr = make_float4((pi.x - c.x) + li.x, (pi.y - c.y) + li.y,
                                      (pi.z - c.z) + li.z, pi.w);
        const float cull2 = rc2max * 1.0001f;
        for (int jt = 0; jt < nd; jt += kGroup) {
            bool near = true;
            if constexpr (CULL) {
                // box values are uniform across the wavefront
                const Box bj = box[t0 + jt / kGroup];
                near = __builtin_amdgcn_readfirstlane((int)(pair::box_dist2(bi, bj) < cull2));
                const bool coulomb =
                    __builtin_amdgcn_readfirstlane((int)(bi.lo.w != 0.f && bj.lo.w != 0.f));
                if (!near && !coulomb) continue;
            }
            wave_sync();
            const int j = jt + lane;
            float4 pj = j < nd ? pos[o + j] : make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            if (near && j < nd) {              // near tiles: relative to c, or low words apart
                const float4 lj = lo[o + j];
                if (rel)
                    pj = make_float4((pj.x - c.x) + lj.x, (pj.y - c.y) + lj.y,
                                     (pj.z - c.z) + lj.z, pj.w);
                else
                    sl[w][lane] = lj;
            } else if (near && !rel) {
                sl[w][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            sp[w][lane] = pj;
            wave_sync();
            if (near) {
                const bool lj =
                    rel ? pair::group_near_rel<COMP, false>(sp[w], jt, i, pr, cull2, a)
                        : pair::group_near<COMP, false>(sp[w], sl[w], jt, i, pi, li, cull2, a);
                // tile pairs with a Lennard-Jones candidate, for k_ens_lj
                if (__ballot(lj && live) && lane == 0) {
                    const int gj = jt / kGroup;
                    atomicOr(&nearbits[(size_t)(t0 + it.y / kGroup) * nb_words + (gj >> 5)],
                             1u << (gj & 31));
                }
            } else
                pair::group_far<COMP, UNROLL>(sp[w], pi, a);
        }
        if constexpr (COMP == 1) {
            a.Fx = (double)a.sx - (double)a.cx;
            a.Fy = (double)a.sy - (double)a.cy;
            a.Fz = (double)a.sz - (double)a.cz;
        }
        if (live) {
            const double qi = (double)pi.w;
            const size_t s = (size_t)(o + i);
            F[s] = -qi * a.Fx;
            F[(size_t)total + s] = -qi * a.Fy;
            F[2 * (size_t)total + s] = -qi * a.Fz;
        }
    }
}

// The same sums with 256-slot work items (droplet, block of four tiles): the
// workgroup's four wavefronts own the four tiles and share each staged tile
// of 256 j (high and low words), so a staging wait serves 4 x 256 pairs per
// lane instead of 64.  A near j group is restaged by its wavefront alone, relative
// to the centre of that wavefront's own tile box, exactly as in k_ens_pair;
// every lane sees the same j groups in the same order with the same inputs,
// so the forces are bit for bit those of k_ens_pair.
template <int COMP, bool CULL, int UNROLL>
__global__ __launch_bounds__(kEnsBlock, 5) void k_ens_pair_b(
    const float4* __restrict__ pos, const float4* __restrict__ lo, const int* __restrict__ off,
    const int2* __restrict__ items, int W, unsigned* counter,
    const PairTable* __restrict__ tabs, const Box* __restrict__ box,
    const int* __restrict__ tbase, double* __restrict__ F, int total,
    unsigned* __restrict__ nearbits, int nb_words) {
    __shared__ float4 sp[kEnsBlock];                 // shared j tile (high words)
    __shared__ float4 sl[kEnsBlock];                 // and its low words
    __shared__ float4 sr[kWaves][kGroup];            // a wavefront's near group, relative
    __shared__ unsigned item_s;
    const int w = threadIdx.x / kGroup;
    const int lane = threadIdx.x % kGroup;
    for (;;) {
        __syncthreads();                             // item_s free to overwrite
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned item = item_s;
        if (item >= (unsigned)W) break;              // uniform per workgroup
        const int2 it = items[item];
        const int d = it.x;
        const int o = off[d];
        const int nd = off[d + 1] - o;
        const float rc2max = tabs[d].rc2max;
        const int i0 = it.y + w * kGroup;            // this wavefront's tile
        const bool wlive = i0 < nd;
        const int i = i0 + lane;
        const bool live = i < nd;
        const float4 pi = live ? pos[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 li = live ? lo[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        pair::Acc a;
        Box bi;
        const int t0 = tbase[d];
        float4 c = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.x))),
                               __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.y))),
                               __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pi.z))),
                               0.f);
        bool rel = false;
        if constexpr (CULL) {
            if (wlive) {
                bi = box[t0 + i0 / kGroup];
                c = make_float4(0.5f * (bi.lo.x + bi.hi.x), 0.5f * (bi.lo.y + bi.hi.y),
                                0.5f * (bi.lo.z + bi.hi.z), 0.f);
                rel = tile_compact(bi);
            }
        }
        const float4 pr = make_float4((pi.x - c.x) + li.x, (pi.y - c.y) + li.y,
                                      (pi.z - c.z) + li.z, pi.w);
        const float cull2 = rc2max * 1.0001f;
        for (int jt = 0; jt < nd; jt += kEnsBlock) {
            __syncthreads();
            const int js = jt + (int)threadIdx.x;
            sp[threadIdx.x] = js < nd ? pos[o + js] : make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            sl[threadIdx.x] = js < nd ? lo[o + js] : make_float4(0.f, 0.f, 0.f, 0.f);
            __syncthreads();
            if (!wlive) continue;
#pragma unroll 1
            for (int g = 0; g < kWaves; ++g) {
                const int jg = jt + g * kGroup;
                if (jg >= nd) break;
                bool near = true;
                if constexpr (CULL) {
                    const Box bj = box[t0 + jg / kGroup];
                    near = __builtin_amdgcn_readfirstlane((int)(pair::box_dist2(bi, bj) < cull2));
                    const bool coulomb =
                        __builtin_amdgcn_readfirstlane((int)(bi.lo.w != 0.f && bj.lo.w != 0.f));
                    if (!near && !coulomb) continue;
                }
                if (near) {
                    bool lj;
                    if (rel) {
                        const int j = jg + lane;
                        float4 pj = sp[g * kGroup + lane];
                        if (j < nd) {
                            const float4 lw = sl[g * kGroup + lane];
                            pj = make_float4((pj.x - c.x) + lw.x, (pj.y - c.y) + lw.y,
                                             (pj.z - c.z) + lw.z, pj.w);
                        }
                        wave_sync();
                        sr[w][lane] = pj;
                        wave_sync();
                        lj = pair::group_near_rel<COMP, false>(sr[w], jg, i, pr, cull2, a);
                    } else {
                        lj = pair::group_near<COMP, false>(sp + g * kGroup, sl + g * kGroup, jg,
                                                           i, pi, li, cull2, a);
                    }
                    if (__ballot(lj && live) && lane == 0) {
                        const int gj = jg / kGroup;
                        atomicOr(&nearbits[(size_t)(t0 + i0 / kGroup) * nb_words + (gj >> 5)],
                                 1u << (gj & 31));
                    }
                } else {
                    pair::group_far<COMP, UNROLL>(sp + g * kGroup, pi, a);
                }
            }
        }
        if constexpr (COMP == 1) {
            a.Fx = (double)a.sx - (double)a.cx;
            a.Fy = (double)a.sy - (double)a.cy;
            a.Fz = (double)a.sz - (double)a.cz;
        }
        if (live) {
            const double qi = (double)pi.w;
            const size_t sl = (size_t)(o + i);
            F[sl] = -qi * a.Fx;
            F[(size_t)total + sl] = -qi * a.Fy;
            F[2 * (size_t)total + sl] = -qi * a.Fz;
        }
    }
}

// Lennard-Jones forces of every tile of every droplet, in FP64, added into F
// after k_ens_pair.  One workgroup per 64-slot tile: its four wavefronts
// share round-robin the j tiles in which k_ens_pair found a pair within the
// largest LJ range (a bitmap row per tile, cleared here); each stages its j
// tiles in its own LDS slice, and the partial sums are added in wavefront
// order.
__global__ __launch_bounds__(kEnsBlock) void k_ens_lj(
    const float4* __restrict__ pos, const float4* __restrict__ lo, const int* __restrict__ typ,
    const int* __restrict__ off, const int2* __restrict__ tiles, int ntiles,
    const PairTable* __restrict__ tabs, const Box* __restrict__ box,
    const int* __restrict__ tbase, double* __restrict__ F, int total,
    unsigned* __restrict__ nearbits, int nb_words) {
    __shared__ float4 sh[kWaves][kGroup];
    __shared__ float4 sl[kWaves][kGroup];
    __shared__ int st[kWaves][kGroup];
    __shared__ double red[kWaves][3][kGroup];
    const int w = threadIdx.x / kGroup;
    const int lane = threadIdx.x % kGroup;
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    const int d = tl.x;
    const int o = off[d];
    const int nd = off[d + 1] - o;
    const int i = tl.y - o + lane;
    const bool live = i < nd;
    const PairTable* tb = tabs + d;
    const double* t64 = tb->sig2d;           // sig2d, e24d, e4d, rc2d follow each other
    const int T = tb->T;
    const float4 pi = live ? pos[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 li = live ? lo[o + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = live ? typ[o + i] : 0;
    Box bi;
    if (box) bi = box[t];
    const float cull2 = tb->rc2max * 1.0001f;
    const int ng = (nd + kGroup - 1) / kGroup;
    const int t0 = tbase[d];
    double L[3] = {0.0, 0.0, 0.0};
    double S = 0.0, U = 0.0;
    int rank = 0;
    unsigned* row = nearbits + (size_t)t * nb_words;   // tiles k_ens_pair found an LJ candidate in
    for (int c0 = 0; c0 < ng; c0 += kGroup) {
        const int gj = c0 + lane;
        const bool nb = gj < ng && ((row[gj >> 5] >> (gj & 31)) & 1u);
        unsigned long long m = __ballot(nb);
        while (m) {
            const int g = c0 + __builtin_ctzll(m);
            m &= m - 1ull;
            if ((rank++ & (kWaves - 1)) != w) continue;
            const int j = g * kGroup + lane;
            wave_sync();
            sh[w][lane] = j < nd ? pos[o + j] : make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            sl[w][lane] = j < nd ? lo[o + j] : make_float4(0.f, 0.f, 0.f, 0.f);
            st[w][lane] = j < nd ? typ[o + j] : 0;
            wave_sync();
#pragma unroll 2
            for (int k = 0; k < kGroup; ++k) {
                const float4 pj = sh[w][k];
                const float4 lj = sl[w][k];
                const float dx = (pj.x - pi.x) + (lj.x - li.x);
                const float dy = (pj.y - pi.y) + (lj.y - li.y);
                const float dz = (pj.z - pi.z) + (lj.z - li.z);
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                if (r2 < cull2 && live && g * kGroup + k != i)
                    pair::lj_pair64<false>(pj, lj, pi, li, t64, ti * T + st[w][k], L, S, U);
            }
        }
    }
    red[w][0][lane] = L[0];
    red[w][1][lane] = L[1];
    red[w][2][lane] = L[2];
    __syncthreads();
    for (int k = threadIdx.x; k < nb_words; k += kEnsBlock) row[k] = 0u;   // all zero at rest
    if (w != 0 || !live) return;
    double Ls[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < kWaves; ++v)
        for (int c = 0; c < 3; ++c) Ls[c] += red[v][c][lane];
    const size_t s = (size_t)(o + i);
    F[s] -= Ls[0];
    F[(size_t)total + s] -= Ls[1];
    F[2 * (size_t)total + s] -= Ls[2];
}

__global__ __launch_bounds__(256) void k_ens_update(float4* pos, float4* lo,
                                                    const int* __restrict__ typ,
                                                    const int* __restrict__ did,
                                                    const int* __restrict__ lid,
                                                    const double* __restrict__ F, int total,
                                                    const ExtParams* __restrict__ ext,
                                                    const unsigned long long* __restrict__ seeds,
                                                    double dt, DevState* st) {
    const long long step = st->step;
    const double tn = st->t + dt;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < total) {
        const int d = did[s];
        const ExtParams& P = ext[d];
        const double R = radius_at(P.R, tn);
        float4 h = pos[s], l = lo[s];
        const double Fs[3] = {F[s], F[(size_t)total + s], F[2 * (size_t)total + s]};
        if (!upd::advance(h, l, Fs, typ[s], R, dt, P, (uint32_t)lid[s],
                          (unsigned long long)step, seeds[d]))
            atomicMin(&st->bad_step, (unsigned long long)step);
        pos[s] = h;
        lo[s] = l;
    }
}

// Bounding box and charged flag of every 64-slot tile (one wavefront each).
__global__ __launch_bounds__(256) void k_ens_boxes(const float4* __restrict__ pos,
                                                   const int* __restrict__ off,
                                                   const int2* __restrict__ tiles, int ntiles,
                                                   Box* box) {
    const int g = blockIdx.x * 4 + threadIdx.x / kGroup;
    if (g >= ntiles) return;                           // uniform per wavefront
    const int2 t = tiles[g];
    const int s = t.y + (int)(threadIdx.x % kGroup);
    const bool live = s < off[t.x + 1];
    const float4 h = live ? pos[s] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float lx = upd::wave_min(live ? h.x : INFINITY), hx = upd::wave_max(live ? h.x : -INFINITY);
    const float ly = upd::wave_min(live ? h.y : INFINITY), hy = upd::wave_max(live ? h.y : -INFINITY);
    const float lz = upd::wave_min(live ? h.z : INFINITY), hz = upd::wave_max(live ? h.z : -INFINITY);
    const bool charged = __any(live && h.w != 0.f);
    if (threadIdx.x % kGroup == 0) {
        Box b;
        b.lo = make_float4(lx, ly, lz, charged ? 1.f : 0.f);
        b.hi = make_float4(hx, hy, hz, 0.f);
        box[g] = b;
    }
}

// Bounding box of every droplet (one workgroup each), [n_drop][6].
__global__ __launch_bounds__(256) void k_ens_bounds(const float4* __restrict__ pos,
                                                    const int* __restrict__ off, float* out) {
    __shared__ float red[6][256];
    const int d = blockIdx.x;
    float m[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int s = off[d] + threadIdx.x; s < off[d + 1]; s += 256) {
        const float4 h = pos[s];
        m[0] = fminf(m[0], h.x); m[1] = fminf(m[1], h.y); m[2] = fminf(m[2], h.z);
        m[3] = fmaxf(m[3], h.x); m[4] = fmaxf(m[4], h.y); m[5] = fmaxf(m[5], h.z);
    }
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = m[c];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; ++c)
                red[c][threadIdx.x] = c < 3 ? fminf(red[c][threadIdx.x], red[c][threadIdx.x + w])
                                            : fmaxf(red[c][threadIdx.x], red[c][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 6) out[6 * d + threadIdx.x] = red[threadIdx.x][0];
}

// Sort keys: droplet (bits 51..63), uncharged flag (50), 18-bit Hilbert
// index over the droplet's bounding cube (32..49), slot (0..31; the permute
// kernels read the source slot from the low 32 bits).
__global__ __launch_bounds__(256) void k_ens_keys(const float4* __restrict__ pos,
                                                  const int* __restrict__ did,
                                                  const float* __restrict__ bounds, int total,
                                                  int n_pow2, unsigned long long* keys) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_pow2) return;
    if (s >= total) {
        keys[s] = ~0ull;
        return;
    }
    const int d = did[s];
    const float* b = bounds + 6 * d;
    const float ext = fmaxf(fmaxf(b[3] - b[0], b[4] - b[1]), fmaxf(b[5] - b[2], 1e-30f));
    const float scale = 63.0f / ext;
    const float4 h = pos[s];
    const unsigned qx = (unsigned)fminf(63.f, fmaxf(0.f, (h.x - b[0]) * scale));
    const unsigned qy = (unsigned)fminf(63.f, fmaxf(0.f, (h.y - b[1]) * scale));
    const unsigned qz = (unsigned)fminf(63.f, fmaxf(0.f, (h.z - b[2]) * scale));
    const unsigned long long code = hilbert_index<6>(qx, qy, qz);
    const unsigned long long neutral = h.w == 0.f ? 1ull : 0ull;
    keys[s] = ((unsigned long long)d << 51) | (neutral << 50) | (code << 32) | (unsigned)s;
}

// Positions and forces in the original order: slot s holds particle lid[s]
// of droplet did[s].
__global__ __launch_bounds__(256) void k_ens_gather(const float4* __restrict__ pos,
                                                    const float4* __restrict__ lo,
                                                    const int* __restrict__ did,
                                                    const int* __restrict__ lid,
                                                    const int* __restrict__ off, int total,
                                                    float* hi_out, float* lo_out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= total) return;
    const size_t o = (size_t)off[did[s]] + (size_t)lid[s];
    const float4 h = pos[s], l = lo[s];
    hi_out[3 * o] = h.x;
    hi_out[3 * o + 1] = h.y;
    hi_out[3 * o + 2] = h.z;
    lo_out[3 * o] = l.x;
    lo_out[3 * o + 1] = l.y;
    lo_out[3 * o + 2] = l.z;
}

__global__ __launch_bounds__(256) void k_ens_forces_aos(const double* __restrict__ F,
                                                        const int* __restrict__ did,
                                                        const int* __restrict__ lid,
                                                        const int* __restrict__ off, int total,
                                                        double* out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= total) return;
    const size_t o = (size_t)off[did[s]] + (size_t)lid[s];
    out[3 * o] = F[s];
    out[3 * o + 1] = F[(size_t)total + s];
    out[3 * o + 2] = F[2 * (size_t)total + s];
}

}  // namespace

struct ld_ens {
    int n_drop = 0;
    int total = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<int> off_h;
    float4* pos = nullptr;
    float4* lo = nullptr;
    int* typ = nullptr;
    int* did = nullptr;
    int* lid = nullptr;
    int* off = nullptr;
    int2* items = nullptr;               // (droplet, first slot) of every 64-slot tile
    int W = 0;
    int2* items_b = nullptr;             // (droplet, first slot) of every 256-slot block
    int W_b = 0;
    int rows = 64;                       // slots per work item: 64 (k_ens_pair) or 256 (k_ens_pair_b)
    unsigned* counter = nullptr;
    PairTable* tabs = nullptr;
    ExtParams* ext = nullptr;
    unsigned long long* seeds = nullptr;
    double* F = nullptr;
    double* work = nullptr;              // [3 * total] output staging
    DevState* st = nullptr;
    int workgroups = 0;
    int comp = 0;
    int graph_steps = 0;
    int unroll = 16;                     // Coulomb pairs in flight per lane (8, 16 or 32)
    unsigned* nearbits = nullptr;        // [ntiles][nb_words] tile pairs with an LJ candidate
    int nb_words = 0;
    hipGraphExec_t graph = nullptr;
    double graph_dt = 0.0;
    int graph_len = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    // spatial ordering and tile culling
    bool cull = false;                   // off when droplets or slots exceed the key fields
    Box* box = nullptr;                  // [ntiles]
    int* tbase = nullptr;                // [n_drop] first tile of each droplet
    int2* tiles = nullptr;               // [ntiles] (droplet, first slot)
    int ntiles = 0;
    float* dbounds = nullptr;            // [n_drop * 6]
    ld::SortBuffers sb{};
    int64_t steps_since_sort = 0;
};

namespace {

void ens_free(ld_ens* e) {
    void* bufs[] = {e->pos,   e->lo,   e->typ,   e->did,     e->lid,   e->off,
                    e->items, e->counter, e->tabs, e->ext,   e->seeds, e->F, e->items_b,
                    e->work,  e->st,   e->box,   e->tbase,   e->tiles, e->dbounds,
                    e->sb.keys, e->sb.tmp4, e->sb.tmp_i, e->nearbits};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (e->graph) (void)hipGraphExecDestroy(e->graph);
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    for (hipEvent_t v : e->ev) (void)hipEventDestroy(v);
}

// Sort interval: the graph chunk length when graphs are on (every chunk
// starts with a sort, so eager steps and replays sort at the same steps).
int sort_interval(const ld_ens* e) {
    return e->graph_steps > 0 ? e->graph_steps : kEnsSortEvery;
}

// Re-order every droplet's slots along its Hilbert curve.
ld_status enqueue_sort(ld_ens* e, hipStream_t s) {
    hipLaunchKernelGGL(k_ens_bounds, dim3(e->n_drop), dim3(256), 0, s, e->pos, e->off,
                       e->dbounds);
    hipLaunchKernelGGL(k_ens_keys, dim3((e->sb.n_pow2 + 255) / 256), dim3(256), 0, s, e->pos,
                       e->did, e->dbounds, e->total, e->sb.n_pow2, e->sb.keys);
    HIP_TRY(hipGetLastError());
    HIP_TRY(ld::launch_sort_by_keys(e->pos, e->lo, e->typ, e->lid, e->total, e->sb, s));
    return LD_OK;
}

// Work items a workgroup can run at once: four tiles, or one block.
int max_workgroups(const ld_ens* e) {
    return e->rows == 256 ? e->W_b : (e->W + kWaves - 1) / kWaves;
}

template <int COMP, int UNROLL>
void launch_ens_pair_u(ld_ens* e, hipStream_t s) {
    if (e->rows == 256) {
        if (e->cull)
            hipLaunchKernelGGL((k_ens_pair_b<COMP, true, UNROLL>), dim3(e->workgroups),
                               dim3(kEnsBlock), 0, s, e->pos, e->lo, e->off, e->items_b, e->W_b,
                               e->counter, e->tabs, e->box, e->tbase, e->F, e->total,
                               e->nearbits, e->nb_words);
        else
            hipLaunchKernelGGL((k_ens_pair_b<COMP, false, UNROLL>), dim3(e->workgroups),
                               dim3(kEnsBlock), 0, s, e->pos, e->lo, e->off, e->items_b, e->W_b,
                               e->counter, e->tabs, e->box, e->tbase, e->F, e->total,
                               e->nearbits, e->nb_words);
        return;
    }
    if (e->cull)
        hipLaunchKernelGGL((k_ens_pair<COMP, true, UNROLL>), dim3(e->workgroups), dim3(kEnsBlock),
                           0, s, e->pos, e->lo, e->typ, e->off, e->items, e->W, e->counter,
                           e->tabs, e->box, e->tbase, e->F, e->total, e->nearbits, e->nb_words);
    else
        hipLaunchKernelGGL((k_ens_pair<COMP, false, UNROLL>), dim3(e->workgroups),
                           dim3(kEnsBlock), 0, s, e->pos, e->lo, e->typ, e->off, e->items, e->W,
                           e->counter, e->tabs, e->box, e->tbase, e->F, e->total, e->nearbits,
                           e->nb_words);
}

template <int COMP>
void launch_ens_pair(ld_ens* e, hipStream_t s) {
    if (e->unroll == 8)
        launch_ens_pair_u<COMP, 8>(e, s);
    else if (e->unroll == 32)
        launch_ens_pair_u<COMP, 32>(e, s);
    else
        launch_ens_pair_u<COMP, 16>(e, s);
}

// Boxes, the persistent Coulomb kernel, then the FP64 Lennard-Jones kernel;
// t0 / t1 (or null) are recorded around the Coulomb kernel.
ld_status enqueue_pair(ld_ens* e, hipStream_t s, hipEvent_t t0 = nullptr,
                       hipEvent_t t1 = nullptr) {
    if (e->cull)
        hipLaunchKernelGGL(k_ens_boxes, dim3((e->ntiles + 3) / 4), dim3(256), 0, s, e->pos,
                           e->off, e->tiles, e->ntiles, e->box);
    hipLaunchKernelGGL(k_ens_reset, dim3(1), dim3(1), 0, s, e->counter);
    if (t0) HIP_TRY(hipEventRecord(t0, s));
    if (e->comp == 0)
        launch_ens_pair<0>(e, s);
    else
        launch_ens_pair<1>(e, s);
    HIP_TRY(hipGetLastError());
    if (t1) HIP_TRY(hipEventRecord(t1, s));
    hipLaunchKernelGGL(k_ens_lj, dim3(e->ntiles), dim3(kEnsBlock), 0, s,
                       e->pos, e->lo, e->typ, e->off, e->tiles, e->ntiles, e->tabs,
                       e->cull ? e->box : nullptr, e->tbase, e->F, e->total, e->nearbits,
                       e->nb_words);
    HIP_TRY(hipGetLastError());
    return LD_OK;
}

ld_status enqueue_step(ld_ens* e, double dt, hipStream_t s, bool timed) {
    if (e->cull && e->steps_since_sort >= sort_interval(e)) {
        ld_status st = enqueue_sort(e, s);
        if (st != LD_OK) return st;
        e->steps_since_sort = 0;
    }
    ++e->steps_since_sort;
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
        while (e->ev.size() < e->ev_used + 2) {
            hipEvent_t v;
            HIP_TRY(hipEventCreate(&v));
            e->ev.push_back(v);
        }
        a = e->ev[e->ev_used++];
        b = e->ev[e->ev_used++];
    }
    ld_status st = enqueue_pair(e, s, a, b);    // timed: the Coulomb kernel alone
    if (st != LD_OK) return st;
    hipLaunchKernelGGL(k_ens_update, dim3((e->total + 255) / 256), dim3(256), 0, s, e->pos,
                       e->lo, e->typ, e->did, e->lid, e->F, e->total, e->ext, e->seeds, dt,
                       e->st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(ld::launch_advance(e->st, dt, s));
    return LD_OK;
}

ld_status capture(ld_ens* e, double dt, int steps) {
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    if (!e->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking));
    // the chunk starts with a sort: it is replayed at sort boundaries only
    const int64_t saved = e->steps_since_sort;
    e->steps_since_sort = sort_interval(e);
    HIP_TRY(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
    ld_status st = LD_OK;
    for (int k = 0; k < steps && st == LD_OK; ++k) st = enqueue_step(e, dt, e->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t err = hipStreamEndCapture(e->cap_stream, &g);
    e->steps_since_sort = saved;
    if (st != LD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (err != hipSuccess) return fail(LD_EHIP, "stream capture: %s", hipGetErrorString(err));
    err = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return fail(LD_EHIP, "graph instantiate: %s", hipGetErrorString(err));
    e->graph_dt = dt;
    e->graph_len = steps;
    return LD_OK;
}

}  // namespace

extern "C" {

ld_status ld_ens_init(ld_ens** out, int32_t n_drop, const int64_t* offsets, const int32_t* type,
                      const double* charge, const float* pos, const ld_params* p,
                      const ld_radius* R, const uint64_t* seeds, void* stream) {
    g_err.clear();
    if (!out) return fail(LD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_drop < 1) return fail(LD_EINVAL, "n_drop must be >= 1");
    if (!offsets || !type || !charge || !pos || !p || !R || !seeds)
        return fail(LD_EINVAL, "offsets, type, charge, pos, p, R and seeds are required");
    std::vector<int64_t> offs((size_t)n_drop + 1);
    std::memcpy(offs.data(), offsets, sizeof(int64_t) * offs.size());
    if (offs[0] != 0) return fail(LD_EINVAL, "offsets[0] must be 0");
    for (int d = 0; d < n_drop; ++d) {
        if (offs[d + 1] - offs[d] < 2)
            return fail(LD_EINVAL, "droplet %d has fewer than 2 particles", d);
        ld_status st = check_params(&p[d]);
        if (st != LD_OK) return st;
        st = check_radius(&R[d]);
        if (st != LD_OK) return st;
    }
    const int64_t total = offs[n_drop];
    if (total > (1 << 27)) return fail(LD_EINVAL, "total particles %lld > 2^27", (long long)total);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ty;
    std::vector<double> q;
    std::vector<float> x;
    ld_status st;
    if ((st = read_host(ty, type, (size_t)total, s)) != LD_OK) return st;
    if ((st = read_host(q, charge, (size_t)total, s)) != LD_OK) return st;
    if ((st = read_host(x, pos, (size_t)total * 3, s)) != LD_OK) return st;

    ld_ens* e = new (std::nothrow) ld_ens();
    if (!e) return fail(LD_ENOMEM, "host allocation failed");
    e->n_drop = n_drop;
    e->total = (int)total;
    e->stream = s;
    e->off_h.assign(offs.begin(), offs.end());
    std::vector<float4> h4(total), l4(total);
    std::vector<int> dids(total), lids(total);
    std::vector<PairTable> tabs(n_drop);
    std::vector<ExtParams> exts(n_drop);
    std::vector<unsigned long long> sd(n_drop);
    std::vector<int2> items, items_b, tiles;
    std::vector<int> tbase(n_drop);
    for (int d = 0; d < n_drop; ++d) {
        make_tables(p[d], R[d], tabs[d], exts[d]);
        sd[d] = seeds[d];
        const double qs = std::sqrt(p[d].kT * p[d].bjerrum);
        for (int64_t i = offs[d]; i < offs[d + 1]; ++i) {
            if (ty[i] < 0 || ty[i] >= p[d].n_types) {
                ens_free(e);
                delete e;
                return fail(LD_EINVAL, "type[%lld] outside droplet %d's types", (long long)i, d);
            }
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(x[3 * i + k]) || !std::isfinite(q[i])) {
                    ens_free(e);
                    delete e;
                    return fail(LD_EINVAL, "particle %lld not finite", (long long)i);
                }
            h4[i] = make_float4(x[3 * i], x[3 * i + 1], x[3 * i + 2], (float)(q[i] * qs));
            l4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            dids[i] = d;
            lids[i] = (int)(i - offs[d]);
        }
        tbase[d] = (int)tiles.size();
        for (int64_t i0 = 0; i0 < offs[d + 1] - offs[d]; i0 += kGroup) {
            items.push_back(make_int2(d, (int)i0));
            tiles.push_back(make_int2(d, (int)(offs[d] + i0)));
        }
        for (int64_t i0 = 0; i0 < offs[d + 1] - offs[d]; i0 += kEnsBlock)
            items_b.push_back(make_int2(d, (int)i0));
    }
    // longest item first: an item costs N_d pairs per lane
    auto longer = [&](const int2& a, const int2& b) {
        return (offs[a.x + 1] - offs[a.x]) > (offs[b.x + 1] - offs[b.x]);
    };
    std::stable_sort(items.begin(), items.end(), longer);
    std::stable_sort(items_b.begin(), items_b.end(), longer);
    e->W = (int)items.size();
    e->W_b = (int)items_b.size();
    std::vector<int> off32(offs.begin(), offs.end());
    const size_t N = (size_t)total;
    bool ok = hipMalloc(&e->pos, sizeof(float4) * N) == hipSuccess &&
              hipMalloc(&e->lo, sizeof(float4) * N) == hipSuccess &&
              hipMalloc(&e->typ, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&e->did, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&e->lid, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&e->off, sizeof(int) * (n_drop + 1)) == hipSuccess &&
              hipMalloc(&e->items, sizeof(int2) * items.size()) == hipSuccess &&
              hipMalloc(&e->items_b, sizeof(int2) * items_b.size()) == hipSuccess &&
              hipMalloc(&e->counter, sizeof(unsigned)) == hipSuccess &&
              hipMalloc(&e->tabs, sizeof(PairTable) * n_drop) == hipSuccess &&
              hipMalloc(&e->ext, sizeof(ExtParams) * n_drop) == hipSuccess &&
              hipMalloc(&e->seeds, sizeof(unsigned long long) * n_drop) == hipSuccess &&
              hipMalloc(&e->F, sizeof(double) * 3 * N) == hipSuccess &&
              hipMalloc(&e->work, sizeof(double) * 3 * N) == hipSuccess &&
              hipMalloc(&e->st, sizeof(DevState)) == hipSuccess &&
              hipMalloc(&e->tbase, sizeof(int) * n_drop) == hipSuccess &&
              hipMalloc(&e->tiles, sizeof(int2) * tiles.size()) == hipSuccess;
    // spatial ordering needs the droplet index in 13 bits
    e->cull = n_drop <= (1 << 13);
    e->ntiles = (int)tiles.size();
    {
        int max_ng = 1;
        for (int d = 0; d < n_drop; ++d)
            max_ng = std::max(max_ng, (int)((offs[d + 1] - offs[d] + kGroup - 1) / kGroup));
        e->nb_words = (max_ng + 31) / 32;
        const size_t bytes = sizeof(unsigned) * tiles.size() * (size_t)e->nb_words;
        ok = ok && hipMalloc(&e->nearbits, bytes) == hipSuccess &&
             hipMemsetAsync(e->nearbits, 0, bytes, s) == hipSuccess;
    }
    int n_pow2 = 2048;                                   // the bitonic sort's smallest size
    while (n_pow2 < (int)total) n_pow2 <<= 1;
    e->sb.n_pow2 = n_pow2;
    if (ok && e->cull)
        ok = hipMalloc(&e->box, sizeof(Box) * tiles.size()) == hipSuccess &&
             hipMalloc(&e->dbounds, sizeof(float) * 6 * n_drop) == hipSuccess &&
             hipMalloc(&e->sb.keys, sizeof(unsigned long long) * n_pow2) == hipSuccess &&
             hipMalloc(&e->sb.tmp4, sizeof(float4) * N) == hipSuccess &&
             hipMalloc(&e->sb.tmp_i, sizeof(int) * N) == hipSuccess;
    if (!ok) {
        ens_free(e);
        delete e;
        return fail(LD_ENOMEM, "device allocation failed for %lld particles", (long long)total);
    }
    DevState ds{};
    ds.bad_step = ~0ull;
    const unsigned zero = 0u;
    hipError_t err = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (err == hipSuccess) err = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    up(e->pos, h4.data(), sizeof(float4) * N);
    up(e->lo, l4.data(), sizeof(float4) * N);
    up(e->typ, ty.data(), sizeof(int) * N);
    up(e->did, dids.data(), sizeof(int) * N);
    up(e->lid, lids.data(), sizeof(int) * N);
    up(e->off, off32.data(), sizeof(int) * (n_drop + 1));
    up(e->items, items.data(), sizeof(int2) * items.size());
    up(e->items_b, items_b.data(), sizeof(int2) * items_b.size());
    up(e->counter, &zero, sizeof zero);
    up(e->tabs, tabs.data(), sizeof(PairTable) * n_drop);
    up(e->ext, exts.data(), sizeof(ExtParams) * n_drop);
    up(e->seeds, sd.data(), sizeof(unsigned long long) * n_drop);
    up(e->st, &ds, sizeof ds);
    up(e->tbase, tbase.data(), sizeof(int) * n_drop);
    up(e->tiles, tiles.data(), sizeof(int2) * tiles.size());
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        ens_free(e);
        delete e;
        return fail(LD_EHIP, "upload failed: %s", hipGetErrorString(err));
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    e->workgroups = std::max(1, std::min(cus * 8, max_workgroups(e)));
    e->steps_since_sort = sort_interval(e);              // sort before the first step
    *out = e;
    return LD_OK;
}

void ld_ens_destroy(ld_ens* e) {
    if (!e) return;
    (void)hipStreamSynchronize(e->stream);
    ens_free(e);
    delete e;
}

ld_status ld_ens_set_tuning(ld_ens* e, int32_t workgroups, int32_t comp, int32_t graph_steps) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    if (workgroups < 0 || workgroups > 65536) return fail(LD_EINVAL, "workgroups in [0, 65536]");
    if (comp != 0 && comp != 1) return fail(LD_EINVAL, "comp must be 0 or 1");
    if (graph_steps < 0 || graph_steps > 4096) return fail(LD_EINVAL, "graph_steps in [0, 4096]");
    HIP_TRY(hipStreamSynchronize(e->stream));
    if (workgroups > 0) e->workgroups = workgroups;
    e->comp = comp;
    e->graph_steps = graph_steps;
    e->steps_since_sort = sort_interval(e);              // new interval: sort next step
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    return LD_OK;
}

ld_status ld_ens_get_tuning(ld_ens* e, int32_t out[5]) {
    g_err.clear();
    if (!e || !out) return fail(LD_EINVAL, "ensemble and out are required");
    out[0] = e->workgroups;
    out[1] = e->comp;
    out[2] = e->graph_steps;
    out[3] = e->unroll;
    out[4] = e->rows;
    return LD_OK;
}

ld_status ld_ens_set_unroll(ld_ens* e, int32_t unroll) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    if (unroll != 8 && unroll != 16 && unroll != 32)
        return fail(LD_EINVAL, "unroll must be 8, 16 or 32");
    HIP_TRY(hipStreamSynchronize(e->stream));
    e->unroll = unroll;
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    return LD_OK;
}

ld_status ld_ens_set_rows(ld_ens* e, int32_t rows) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    if (rows != 64 && rows != 256) return fail(LD_EINVAL, "rows must be 64 or 256");
    HIP_TRY(hipStreamSynchronize(e->stream));
    e->rows = rows;
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    return LD_OK;
}

ld_status ld_ens_autotune(ld_ens* e, const char* cache_path, int32_t force, int32_t out[5]) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    HIP_TRY(hipStreamSynchronize(e->stream));
    // cache key: architecture, droplet count, quarter-octave buckets of the
    // pair count sum_d N_d^2 and of the largest droplet, culling, compensation
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    char arch[64];
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* q = arch; *q; ++q)
        if (*q == ':' || *q == ' ') *q = '_';
    double pairs = 0.0;
    int64_t nmax = 0;
    for (int d = 0; d + 1 < (int)e->off_h.size(); ++d) {
        const int64_t nd = e->off_h[d + 1] - e->off_h[d];
        pairs += (double)nd * (double)nd;
        nmax = std::max(nmax, nd);
    }
    char key[192];
    std::snprintf(key, sizeof key, "ens2/%s/d%d/p%d/m%d/cull%d/comp%d", arch, e->n_drop,
                  (int)std::floor(std::log2(pairs) * 4.0),
                  (int)std::floor(std::log2((double)nmax) * 4.0), e->cull ? 1 : 0, e->comp);
    // Time the slot order the steps will use: a sort that is due (a new
    // ensemble sorts before its first step) is done now, as that step would
    // have done it, so the trajectory is unchanged; an unsorted ensemble
    // would have most tile pairs take the careful loop and rank the far
    // loop's settings wrongly.
    if (e->cull && e->steps_since_sort >= sort_interval(e)) {
        const ld_status st = enqueue_sort(e, e->stream);
        if (st != LD_OK) return st;
        e->steps_since_sort = 0;
    }
    int best_w = e->workgroups, best_u = e->unroll, best_r = e->rows;
    bool cached = false;
    if (cache_path && !force) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char k[192];
            int wg = 0, un = 0, ro = 0;
            double ms = 0.0;
            while (std::fscanf(f, "%191s %d %d %d %lf", k, &wg, &un, &ro, &ms) == 5)
                if (std::strcmp(k, key) == 0 && (ro == 64 || ro == 256) &&
                    (un == 8 || un == 16 || un == 32) && wg > 0) {
                    best_w = wg;
                    best_u = un;
                    best_r = ro;
                    cached = true;
                }
            std::fclose(f);
        }
    }
    double best_ms = INFINITY;
    if (!cached) {
        const bool saved_timing = e->timing;
        e->timing = false;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const int per_cu[] = {2, 3, 4, 5, 6, 7, 8};
        const int unrolls[] = {8, 16, 32};
        const int item_rows[] = {64, 256};
        ld_status st = LD_OK;
        // fastest of `reps` timed bursts of `burst` back-to-back launches
        // (after one warm-up burst) of a setting, per launch
        auto time_setting = [&](int w, int u, int r, int reps, int burst) {
            e->rows = r;
            e->unroll = u;
            e->workgroups = w;
            double ms_min = INFINITY;
            for (int rep = 0; rep <= reps && st == LD_OK; ++rep) {
                if (hipEventRecord(e0, e->stream) != hipSuccess) st = LD_EHIP;
                for (int b = 0; b < burst && st == LD_OK; ++b) st = enqueue_pair(e, e->stream);
                if (st == LD_OK && hipEventRecord(e1, e->stream) != hipSuccess) st = LD_EHIP;
                if (st == LD_OK && hipEventSynchronize(e1) != hipSuccess) st = LD_EHIP;
                float ms = 0.f;
                if (st == LD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    st = LD_EHIP;
                if (rep > 0 && ms / burst < ms_min) ms_min = ms / burst;
            }
            return ms_min;
        };
        struct Cand {
            double ms;
            int w, u, r;
        };
        std::vector<Cand> cands;
        for (int r : item_rows)
            for (int u : unrolls)
                for (int k : per_cu) {
                    if (st != LD_OK) break;
                    e->rows = r;
                    const int w = std::max(1, std::min(cus * k, max_workgroups(e)));
                    cands.push_back({time_setting(w, u, r, 3, 1), w, u, r});
                }
        // One pass of single launches leaves settings within a few per cent
        // of each other, in an order that the clock's state can decide and
        // that need not hold under sustained load: the four best are timed
        // again as bursts of launches in three interleaved rounds and
        // ranked by their summed times.
        std::sort(cands.begin(), cands.end(),
                  [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        const int top = std::min<int>(4, (int)cands.size());
        std::vector<double> sum(top, 0.0);
        for (int round = 0; round < 3 && st == LD_OK; ++round)
            for (int c = 0; c < top && st == LD_OK; ++c)
                sum[c] += time_setting(cands[c].w, cands[c].u, cands[c].r, 2, 6);
        for (int c = 0; c < top && st == LD_OK; ++c)
            if (sum[c] / 3.0 < best_ms) {
                best_ms = sum[c] / 3.0;
                best_w = cands[c].w;
                best_u = cands[c].u;
                best_r = cands[c].r;
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        e->timing = saved_timing;
        if (st != LD_OK) return fail(LD_EHIP, "ensemble autotune launch failed");
        if (cache_path) {
            if (FILE* f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s %d %d %d %.6f\n", key, best_w, best_u, best_r, best_ms);
                std::fclose(f);
            }
        }
    }
    e->workgroups = best_w;
    e->unroll = best_u;
    e->rows = best_r;
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    return out ? ld_ens_get_tuning(e, out) : LD_OK;
}

ld_status ld_ens_step(ld_ens* e, double dt, int64_t n_steps) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LD_EINVAL, "dt=%g must be positive", dt);
    if (n_steps < 0) return fail(LD_EINVAL, "n_steps must be >= 0");
    int64_t left = n_steps;
    const bool use_graph = e->graph_steps > 0 && !e->timing;
    const int len = e->graph_steps;
    while (left > 0) {
        // a captured chunk starts with a sort, so it is used at sort
        // boundaries only; eager steps fill up to the next boundary
        const bool at_chunk = !e->cull || e->steps_since_sort >= sort_interval(e);
        if (use_graph && at_chunk && left >= len) {
            if (!e->graph || e->graph_dt != dt || e->graph_len != len) {
                ld_status st = capture(e, dt, len);
                if (st != LD_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(e->graph, e->stream));
            e->steps_since_sort = len;
            left -= len;
            continue;
        }
        ld_status st = enqueue_step(e, dt, e->stream, e->timing);
        if (st != LD_OK) return st;
        --left;
    }
    return LD_OK;
}

ld_status ld_ens_forces(ld_ens* e, double* F_pair) {
    g_err.clear();
    if (!e || !F_pair) return fail(LD_EINVAL, "ensemble and F_pair are required");
    ld_status st = enqueue_pair(e, e->stream);
    if (st != LD_OK) return st;
    hipLaunchKernelGGL(k_ens_forces_aos, dim3((e->total + 255) / 256), dim3(256), 0, e->stream,
                       e->F, e->did, e->lid, e->off, e->total, e->work);
    HIP_TRY(hipGetLastError());
    HIP_TRY(copy_out(F_pair, e->work, sizeof(double) * 3 * (size_t)e->total, e->stream));
    return LD_OK;
}

ld_status ld_ens_get_positions(ld_ens* e, float* pos, float* pos_lo) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    const size_t N = (size_t)e->total;
    float* hi = reinterpret_cast<float*>(e->work);
    float* lo = hi + 3 * N;
    hipLaunchKernelGGL(k_ens_gather, dim3((e->total + 255) / 256), dim3(256), 0, e->stream,
                       e->pos, e->lo, e->did, e->lid, e->off, e->total, hi, lo);
    HIP_TRY(hipGetLastError());
    if (pos) HIP_TRY(copy_out(pos, hi, sizeof(float) * 3 * N, e->stream));
    if (pos_lo) HIP_TRY(copy_out(pos_lo, lo, sizeof(float) * 3 * N, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    return LD_OK;
}

ld_status ld_ens_get_state(ld_ens* e, int64_t* step, double* t) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    DevState ds;
    HIP_TRY(hipMemcpyAsync(&ds, e->st, sizeof ds, hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    if (step) *step = ds.step;
    if (t) *t = ds.t;
    return LD_OK;
}

ld_status ld_ens_sync(ld_ens* e) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    DevState ds;
    HIP_TRY(hipMemcpyAsync(&ds, e->st, sizeof ds, hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    if (ds.bad_step != ~0ull) {
        const unsigned long long none = ~0ull;
        HIP_TRY(hipMemcpy(&e->st->bad_step, &none, sizeof none, hipMemcpyHostToDevice));
        return fail(LD_ENONFINITE, "step %llu produced a non-finite or too large move",
                    (unsigned long long)ds.bad_step);
    }
    return LD_OK;
}

ld_status ld_ens_kernel_timing(ld_ens* e, int32_t enable) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    HIP_TRY(hipStreamSynchronize(e->stream));
    e->timing = enable != 0;
    if (enable) e->ev_used = 0;
    return LD_OK;
}

ld_status ld_ens_kernel_time(ld_ens* e, int64_t* launches, double* total_ms) {
    g_err.clear();
    if (!e) return fail(LD_EINVAL, "ensemble is NULL");
    HIP_TRY(hipStreamSynchronize(e->stream));
    double tot = 0.0;
    for (size_t k = 0; k + 1 < e->ev_used; k += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e->ev[k], e->ev[k + 1]));
        tot += ms;
    }
    if (launches) *launches = (int64_t)(e->ev_used / 2);
    if (total_ms) *total_ms = tot;
    return LD_OK;
}

}  // extern "C"
