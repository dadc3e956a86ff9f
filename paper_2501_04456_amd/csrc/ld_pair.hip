// All-pairs force kernels: the O(N^2) part of each step (section 2.2, step
// (ii): Lennard-Jones and Coulomb forces, both unshifted; Coulomb here runs
// over all pairs).
//
// k_pair: the Coulomb sum.  One work-item owns one particle i (slot order).
// A workgroup of BLOCK work-items streams the j range of its split through
// LDS one tile of BLOCK particles at a time; every lane reads the same LDS
// word per j (a broadcast), so the j stream costs one ds_read per wavefront
// per j and the VALU does the rest.  Per pair: 12 FP32 VALU operations plus
// one v_rsq_f32 (three subtractions, r^2 as mul+fma+fma, q_j r^-3 as three
// multiplications, three fma into the block accumulators).  With tile
// culling on, a 64-particle j group whose bounding box is farther than the
// largest LJ range from the wavefront's own box takes the plain loop on the
// FP32 high words; a nearer group takes the loop on positions relative to
// the centre c of the workgroup's box, (hi - c) + lo, staged beside the high
// words (same instruction count, and the rounding of |x - c| instead of
// |x|), which also leaves out the self pair and flags LJ candidates; a far
// pair of groups one of which is uncharged is skipped (no force at all).
//
// k_lj: the Lennard-Jones sum, which is short-ranged (lj_cut sigma_ij): one
// workgroup per 64-slot i group visits the j groups that k_pair found to
// hold a pair within the largest LJ range (a bitmap k_pair fills and k_lj
// clears; without it, the groups whose boxes come that close), stages each
// in LDS and evaluates the pairs inside the cutoff in FP64.  It adds its
// result into the first force partial of each slot after k_pair has
// written it (same stream, one writer per slot).
//
// Precision.  The Coulomb pair terms are FP32.  Each lane sums KB = 32 of
// them in an FP32 block accumulator and then moves the block into FP64
// totals (COMP=0) or into a blocked Kahan pair (COMP=1, flushed to FP64 at
// the end).  The worst-case rounding of a 32-term FP32 block is
// 31 u sum|f| ~ 1.8e-6 of the conditioning scale S_i = sum_j |f_ij|.  The
// Lennard-Jones terms are FP64 throughout.
#include "ld_pair_core.h"

namespace ld {
namespace {

using namespace pair;

// Wavefronts per SIMD the register allocation must allow (block 64 keeps a
// whole j tile in registers whatever the bound; it is left unconstrained).
#ifndef LD_PAIR_MIN_WAVES
#define LD_PAIR_MIN_WAVES 6
#endif

constexpr float kRelReach = 255.f;         // sigma; see the near-loop choice in k_pair
#ifndef LD_PAIR_REL_GUARD
#define LD_PAIR_REL_GUARD 1
#endif

// Workgroup -> (i tile, j split) on a one-dimensional grid.  Workgroups go
// to the eight XCDs in turn (linear id mod 8), so XCD k takes i tiles k,
// k + 8, k + 16, ... for every split, split after split: the i tiles one
// XCD serves (about an eighth of them) stay in its L2 across the splits
// instead of every tile being fetched again for each split.  Workgroups
// past the last tile of an XCD's share leave at once.
constexpr int kXcds = 8;
__host__ __device__ inline int pair_grid(int tiles, int j_split) {
    return kXcds * ((tiles + kXcds - 1) / kXcds) * j_split;
}

template <int BLOCK, int COMP, bool DIAG, bool CULL, bool REL>
__global__ __launch_bounds__(BLOCK, BLOCK == 64 ? 1 : LD_PAIR_MIN_WAVES) void k_pair(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo,
                                                const Box* __restrict__ box, int n,
                                                int j_per_split, float rc2max,
                                                double* __restrict__ Fpart,
                                                double* __restrict__ S_out,
                                                double* __restrict__ U_out,
                                                unsigned* __restrict__ nearbits, int nb_words) {
    __shared__ float4 sp[BLOCK];             // j tile, high words
    __shared__ float4 sr[BLOCK];             // near loop: positions relative to c, or low words

    const int tid = threadIdx.x;
    const int ngroups = (n + kGroup - 1) / kGroup;
    const int tiles = (n + BLOCK - 1) / BLOCK;
    const int per_xcd = (tiles + kXcds - 1) / kXcds;
    const int q = (int)blockIdx.x / kXcds;
    const int tx = (int)blockIdx.x % kXcds + kXcds * (q % per_xcd);   // i tile
    const int ty = q / per_xcd;                                         // j split
    if (tx >= tiles) return;                     // uniform per workgroup
    // A small margin covers FP32 rounding of box distances against r^2.
    const float cull2 = rc2max * 1.0001f;
    // Near loop on positions relative to c, the centre of the box of the
    // workgroup's BLOCK slots, when that box is compact (half-extent below
    // kRelReach: |x - c| < 256 sigma, so (hi - c) + lo carries at most two
    // FP32 roundings of 2^-17 sigma, 1.5e-5 sigma, and in practice a few
    // times less, most near pairs sitting tens of sigma from c); otherwise,
    // and without culling (no boxes), on exact (hi, lo) differences, e.g.
    // where a blown-up step has thrown NPs far out or the slots are not in
    // spatial order.  The choice is uniform per workgroup and made before
    // anything else is loaded.  The two loops are separate instances (REL),
    // so the common one keeps its own register allocation, launched on the
    // same grid: first the exact one, which leaves compact workgroups at
    // once and takes only the near group pairs of stretched ones; then the
    // relative one, which takes compact workgroups whole and the far group
    // pairs of stretched ones, adding them to what the exact one wrote.  A
    // stretched workgroup thus adds no long serial tail after the relative
    // launch.  Without culling, or in diagnostic mode, the exact instance
    // runs alone and takes everything.
    bool rel = false;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (CULL && !DIAG) {
        float3 blo = make_float3(INFINITY, INFINITY, INFINITY);
        float3 bhi = make_float3(-INFINITY, -INFINITY, -INFINITY);
        for (int g4 = 0; g4 < BLOCK / kGroup; ++g4) {
            const int gq = tx * (BLOCK / kGroup) + g4;
            if (gq >= ngroups) break;
            const Box bq = box[gq];
            blo = make_float3(fminf(blo.x, bq.lo.x), fminf(blo.y, bq.lo.y), fminf(blo.z, bq.lo.z));
            bhi = make_float3(fmaxf(bhi.x, bq.hi.x), fmaxf(bhi.y, bq.hi.y), fmaxf(bhi.z, bq.hi.z));
        }
        c = make_float4(0.5f * (blo.x + bhi.x), 0.5f * (blo.y + bhi.y), 0.5f * (blo.z + bhi.z),
                        0.f);
        const float ext = fmaxf(fmaxf(bhi.x - blo.x, bhi.y - blo.y), bhi.z - blo.z);
        rel = !LD_PAIR_REL_GUARD || ext < 2.f * kRelReach;    // false for NaN or infinite boxes
    }
    constexpr bool SPLIT = CULL && !DIAG;
    if (!REL && rel) return;                     // uniform per workgroup

    const int i = tx * BLOCK + tid;
    const bool live = i < n;
    const float4 pi = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 li = live ? lo[i] : make_float4(0.f, 0.f, 0.f, 0.f);

    // This wavefront's bounding box (culling only).
    Box bi;
    if constexpr (CULL) {
        const int gi = (tx * BLOCK + (tid & ~(kGroup - 1))) / kGroup;
        if (gi < ngroups) {
            bi = box[gi];
        } else {
            bi.lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
            bi.hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
        }
    }
    const float4 pr = make_float4((pi.x - c.x) + li.x, (pi.y - c.y) + li.y, (pi.z - c.z) + li.z,
                                  pi.w);

    const int j0 = ty * j_per_split;
    const int j1 = min(n, j0 + j_per_split);
    Acc a;
#pragma unroll 1
    for (int jt = j0; jt < j1; jt += BLOCK) {
        __syncthreads();
        const int j = jt + tid;
        {
            float4 h = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            float4 r = REL ? h : make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < j1) {
                h = pos[j];
                const float4 l = lo[j];
                r = REL ? make_float4((h.x - c.x) + l.x, (h.y - c.y) + l.y, (h.z - c.z) + l.z, h.w)
                        : l;
            }
            sp[tid] = h;
            sr[tid] = r;
        }
        __syncthreads();
#pragma unroll 1
        for (int g = 0; g < BLOCK / kGroup; ++g) {
            const int jg = jt + g * kGroup;
            bool near = true;
            if constexpr (CULL) {
                const int gj = jg / kGroup;
                near = false;
                bool coulomb = false;
                if (jg < j1 && gj < ngroups) {
                    const Box bj = box[gj];
                    if (REL && rel) {
                        near = box_dist2(bi, bj) < cull2;
                    } else {
                        // the i group's own box may be stretched across the
                        // droplet by one NP thrown out: test each lane's i
                        near = __ballot(live && point_box_dist2(pi, bj) < cull2) != 0;
                    }
                    coulomb = bi.lo.w != 0.f && bj.lo.w != 0.f;
                }
                if (!near && !__builtin_amdgcn_readfirstlane((int)coulomb)) continue;
                // a stretched workgroup's near pairs go to the exact
                // instance, its far ones to the relative instance
                if constexpr (SPLIT) {
                    if (REL ? (!rel && near) : !near) continue;
                }
            }
            if constexpr (DIAG) near = true;
            if (__builtin_amdgcn_readfirstlane((int)near)) {
                bool lj;
                if constexpr (REL)
                    lj = group_near_rel<COMP, DIAG>(sr + g * kGroup, jg, i, pr, cull2, a);
                else
                    lj = group_near<COMP, DIAG>(sp + g * kGroup, sr + g * kGroup, jg, i, pi, li,
                                                cull2, a);
                // record the pair of groups if it holds a Lennard-Jones
                // candidate, for the Lennard-Jones kernel
                if (nearbits && __ballot(lj && live) && (tid & (kGroup - 1)) == 0) {
                    const int gi = (tx * BLOCK + tid) / kGroup, gj = jg / kGroup;
                    atomicOr(&nearbits[(size_t)gi * nb_words + (gj >> 5)], 1u << (gj & 31));
                }
            } else {
                group_far<COMP>(sp + g * kGroup, pi, a);
            }
        }
    }
    if constexpr (COMP == 1) {
        a.Fx = (double)a.sx - (double)a.cx;
        a.Fy = (double)a.sy - (double)a.cy;
        a.Fz = (double)a.sz - (double)a.cz;
    }
    if (live) {
        // F_i = -q_i sum_j q_j r^-3 (x_j - x_i)
        const double qi = (double)pi.w;
        double* F = Fpart + (size_t)ty * 3 * (size_t)n;
        if (REL && !rel) {                       // after the exact instance's near part
            F[i] += -qi * a.Fx;
            F[(size_t)n + i] += -qi * a.Fy;
            F[2 * (size_t)n + i] += -qi * a.Fz;
        } else {
            F[i] = -qi * a.Fx;
            F[(size_t)n + i] = -qi * a.Fy;
            F[2 * (size_t)n + i] = -qi * a.Fz;
        }
        if constexpr (DIAG) {
            S_out[i] = a.S;
            U_out[i] = 0.0;
            U_out[(size_t)n + i] = a.Uc;
        }
    }
}

constexpr int kLjBlock = 256;
constexpr int kLjWaves = kLjBlock / kGroup;

// Lennard-Jones forces of every slot, added into partial 0 (and, with DIAG,
// into S and the LJ energy row of U).  One workgroup per 64-slot i group:
// its four wavefronts test the same 64 boxes at a time and share the j
// groups that come within the largest LJ range round-robin (the r-th near
// group goes to wavefront r mod 4); each wavefront stages its j groups in
// its own LDS slice, and the four partial sums are added in wavefront order
// at the end.  Without boxes every group is visited.
template <bool DIAG>
__global__ __launch_bounds__(kLjBlock) void k_lj(const float4* __restrict__ pos,
                                                  const float4* __restrict__ lo,
                                                  const int* __restrict__ typ,
                                                  const Box* __restrict__ box, int n,
                                                  double* __restrict__ F,
                                                  double* __restrict__ S_out,
                                                  double* __restrict__ U_out, PairTable tab,
                                                  unsigned* __restrict__ nearbits,
                                                  int nb_words) {
    __shared__ float4 sh[kLjWaves][kGroup];
    __shared__ float4 sl[kLjWaves][kGroup];
    __shared__ int st[kLjWaves][kGroup];
    __shared__ double t64[4 * kMaxTypes * kMaxTypes];
    __shared__ double red[kLjWaves][5][kGroup];
    for (int k = threadIdx.x; k < kMaxTypes * kMaxTypes; k += kLjBlock) {
        t64[k] = tab.sig2d[k];
        t64[kMaxTypes * kMaxTypes + k] = tab.e24d[k];
        t64[2 * kMaxTypes * kMaxTypes + k] = tab.e4d[k];
        t64[3 * kMaxTypes * kMaxTypes + k] = tab.rc2d[k];
    }
    __syncthreads();
    const int w = threadIdx.x / kGroup;
    const int lane = threadIdx.x % kGroup;
    const int ngroups = (n + kGroup - 1) / kGroup;
    const int gi = blockIdx.x;
    const int i = gi * kGroup + lane;
    const bool live = i < n;
    const float4 pi = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 li = live ? lo[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = live ? typ[i] : 0;
    const int T = tab.T;
    Box bi;
    if (box) bi = box[gi];
    // box test and FP32 screen (the (hi, lo) difference: relative error
    // ~1e-7 in r^2) with a margin; the cutoff itself is decided in FP64
    const float cull2 = tab.rc2max * 1.0001f;
    double L[3] = {0.0, 0.0, 0.0};
    double S = 0.0, U = 0.0;
    int rank = 0;                                // near groups seen so far (all wavefronts)
    const unsigned* row = nearbits ? nearbits + (size_t)gi * nb_words : nullptr;
    for (int c0 = 0; c0 < ngroups; c0 += kGroup) {
        const int gj = c0 + lane;
        bool nb = gj < ngroups;
        if (row)                                 // the pairs the Coulomb kernel found near
            nb = nb && ((row[gj >> 5] >> (gj & 31)) & 1u);
        else if (nb && box)
            nb = box_dist2(bi, box[gj]) < cull2;
        unsigned long long m = __ballot(nb);
        while (m) {
            const int g = c0 + __builtin_ctzll(m);
            m &= m - 1ull;
            if ((rank++ & (kLjWaves - 1)) != w) continue;
            const int j = g * kGroup + lane;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            sh[w][lane] = j < n ? pos[j] : make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            sl[w][lane] = j < n ? lo[j] : make_float4(0.f, 0.f, 0.f, 0.f);
            st[w][lane] = j < n ? typ[j] : 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 2
            for (int k = 0; k < kGroup; ++k) {
                const float4 pj = sh[w][k];
                const float4 lj = sl[w][k];
                const float dx = (pj.x - pi.x) + (lj.x - li.x);
                const float dy = (pj.y - pi.y) + (lj.y - li.y);
                const float dz = (pj.z - pi.z) + (lj.z - li.z);
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                if (r2 < cull2 && live && g * kGroup + k != i)
                    lj_pair64<DIAG>(pj, lj, pi, li, t64, ti * T + st[w][k], L, S, U);
            }
        }
    }
    red[w][0][lane] = L[0];
    red[w][1][lane] = L[1];
    red[w][2][lane] = L[2];
    if constexpr (DIAG) {
        red[w][3][lane] = S;
        red[w][4][lane] = U;
    }
    __syncthreads();
    if (row)                                     // leave the bitmap all zero
        for (int k = threadIdx.x; k < nb_words; k += kLjBlock) nearbits[(size_t)gi * nb_words + k] = 0u;
    if (w != 0 || !live) return;
    double Ls[3] = {0.0, 0.0, 0.0}, Ss = 0.0, Us = 0.0;
    for (int v = 0; v < kLjWaves; ++v) {
        for (int c = 0; c < 3; ++c) Ls[c] += red[v][c][lane];
        if constexpr (DIAG) {
            Ss += red[v][3][lane];
            Us += red[v][4][lane];
        }
    }
    // F_i += -sum_j g_ij (x_j - x_i)
    F[i] -= Ls[0];
    F[(size_t)n + i] -= Ls[1];
    F[2 * (size_t)n + i] -= Ls[2];
    if constexpr (DIAG) {
        S_out[i] += Ss;
        U_out[i] += Us;
    }
}

template <int BLOCK, int COMP, bool DIAG, bool CULL>
hipError_t launch_t(const PairLaunch& L, const PairTable& tab, hipStream_t s) {
    const int tiles = (L.n + BLOCK - 1) / BLOCK;
    const int per = (tiles + L.j_split - 1) / L.j_split;
    const dim3 grid(pair_grid(tiles, L.j_split));
    // with culling: the exact instance (stretched workgroups' near pairs)
    // first, then the relative one, which adds to it; otherwise the exact
    // instance alone
    if (!(CULL && !DIAG) || LD_PAIR_REL_GUARD)
        hipLaunchKernelGGL((k_pair<BLOCK, COMP, DIAG, CULL, false>), grid, dim3(BLOCK), 0, s,
                           L.pos, L.lo, L.box, L.n, per * BLOCK, tab.rc2max, L.Fpart, L.S, L.U,
                           L.nearbits, L.nb_words);
    if constexpr (CULL && !DIAG)
        hipLaunchKernelGGL((k_pair<BLOCK, COMP, DIAG, CULL, true>), grid, dim3(BLOCK), 0, s,
                           L.pos, L.lo, L.box, L.n, per * BLOCK, tab.rc2max, L.Fpart, L.S, L.U,
                           L.nearbits, L.nb_words);
    return hipGetLastError();
}

template <int BLOCK>
hipError_t launch_b(const PairLaunch& L, const PairTable& tab, hipStream_t s) {
    const bool diag = L.S != nullptr;
    if (diag) return launch_t<BLOCK, 0, true, false>(L, tab, s);
    if (L.comp == 0) {
        return L.cull ? launch_t<BLOCK, 0, false, true>(L, tab, s)
                      : launch_t<BLOCK, 0, false, false>(L, tab, s);
    }
    return L.cull ? launch_t<BLOCK, 1, false, true>(L, tab, s)
                  : launch_t<BLOCK, 1, false, false>(L, tab, s);
}

hipError_t launch_coulomb(const PairLaunch& L, const PairTable& tab, hipStream_t s) {
    switch (L.block) {
        case 64: return launch_b<64>(L, tab, s);
        case 128: return launch_b<128>(L, tab, s);
        case 256: return launch_b<256>(L, tab, s);
        case 512: return launch_b<512>(L, tab, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pair(const PairLaunch& L, const PairTable& tab, hipStream_t s,
                       hipEvent_t after_coulomb) {
    hipError_t e = launch_coulomb(L, tab, s);
    if (e != hipSuccess) return e;
    if (after_coulomb && (e = hipEventRecord(after_coulomb, s)) != hipSuccess) return e;
    const int ngroups = (L.n + kGroup - 1) / kGroup;
    const dim3 grid(ngroups);
    const Box* box = L.box;          // boxes are kept current by sort and update
    if (L.S)
        hipLaunchKernelGGL(k_lj<true>, grid, dim3(kLjBlock), 0, s, L.pos, L.lo, L.typ, box, L.n,
                           L.Fpart, L.S, L.U, tab, L.nearbits, L.nb_words);
    else
        hipLaunchKernelGGL(k_lj<false>, grid, dim3(kLjBlock), 0, s, L.pos, L.lo, L.typ, box,
                           L.n, L.Fpart, L.S, L.U, tab, L.nearbits, L.nb_words);
    return hipGetLastError();
}

}  // namespace ld
