// All-pairs force kernel: the O(N^2) part of each step (section 2.2, step
// (ii): Lennard-Jones and Coulomb forces, both unshifted; Coulomb here runs
// over all pairs).
//
// Layout.  One work-item owns one particle i (slot order).  A workgroup of
// BLOCK work-items streams the j range of its split through LDS one tile of
// BLOCK particles at a time; every lane reads the same LDS word per j (a
// broadcast), so the j stream costs one ds_read per wavefront per j and the
// VALU does the rest.
//
// Per pair the Coulomb-only path is 12 FP32 VALU operations plus one
// v_rsq_f32: three subtractions, r^2 as mul+fma+fma, q_j r^-3 as three
// multiplications and three fma into the block accumulators.  Lennard-Jones is
// short-ranged (lj_cut sigma_ij), so it lives in a rarely taken branch.  With
// tile culling on, a 64-particle j group whose bounding box is farther than
// the largest LJ range from the wavefront's own box skips even the range
// test.
//
// Precision.  The pair terms are FP32.  Each lane sums KB = 32 of them in an
// FP32 block accumulator and then moves the block into FP64 totals (COMP=0)
// or into a blocked Kahan pair (COMP=1, flushed to FP64 at the end).  The
// worst-case rounding of a 32-term FP32 block is 31 u sum|f| ~ 1.8e-6 of the
// conditioning scale S_i = sum_j |f_ij|.
#include "ld_pair_core.h"

namespace ld {
namespace {

using namespace pair;

template <int BLOCK, int COMP, bool DIAG, bool CULL>
__global__ __launch_bounds__(BLOCK) void k_pair(const float4* __restrict__ pos,
                                                const float4* __restrict__ lo,
                                                const int* __restrict__ typ,
                                                const Box* __restrict__ box, int n,
                                                int j_per_split, double* __restrict__ Fpart,
                                                double* __restrict__ S_out,
                                                double* __restrict__ U_out, PairTable tab) {
    __shared__ float4 sp[BLOCK];
    __shared__ int stp[BLOCK];
    __shared__ float ttab[4 * kMaxTypes * kMaxTypes];

    const int tid = threadIdx.x;
    const int T = tab.T;
    for (int k = tid; k < kMaxTypes * kMaxTypes; k += BLOCK) {
        ttab[k] = tab.sig2[k];
        ttab[kMaxTypes * kMaxTypes + k] = tab.rc2[k];
        ttab[2 * kMaxTypes * kMaxTypes + k] = tab.e24[k];
        ttab[3 * kMaxTypes * kMaxTypes + k] = tab.e4[k];
    }
    const int i = blockIdx.x * BLOCK + tid;
    const bool live = i < n;
    const float4 pi = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 li = live ? lo[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = live ? typ[i] : 0;
    const int ngroups = (n + kGroup - 1) / kGroup;

    // This wavefront's bounding box (culling only).
    Box bi;
    if constexpr (CULL) {
        const int gi = (blockIdx.x * BLOCK + (tid & ~(kGroup - 1))) / kGroup;
        if (gi < ngroups) {
            bi = box[gi];
        } else {
            bi.lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
            bi.hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
        }
    }
    // Tile culling must never drop a pair that the range test would keep:
    // a small margin covers FP32 rounding of box distances against r^2.
    const float cull2 = tab.rc2max * 1.0001f;

    const int j0 = blockIdx.y * j_per_split;
    const int j1 = min(n, j0 + j_per_split);
    Acc a;
    for (int jt = j0; jt < j1; jt += BLOCK) {
        __syncthreads();
        const int j = jt + tid;
        if (j < j1) {
            sp[tid] = pos[j];
            stp[tid] = typ[j];
        } else {
            sp[tid] = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
            stp[tid] = 0;
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
                    near = box_dist2(bi, bj) < cull2;
                    // a far pair of groups one of which is uncharged has no
                    // force at all: skip it
                    coulomb = bi.lo.w != 0.f && bj.lo.w != 0.f;
                }
                if (!near && !__builtin_amdgcn_readfirstlane((int)coulomb)) continue;
            }
            if constexpr (DIAG) near = true;
            if (__builtin_amdgcn_readfirstlane((int)near)) {
                group_near<COMP, DIAG>(sp + g * kGroup, stp + g * kGroup, ttab, T,
                                       tab.rc2max, jg, i, ti, pi, lo + jg,
                                       max(0, min(kGroup, j1 - jg)), li, a);
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
        // F_i = -q_i sum_j q_j r^-3 (x_j - x_i) - sum_j g_ij (x_j - x_i)
        const double qi = (double)pi.w;
        double* F = Fpart + (size_t)blockIdx.y * 3 * (size_t)n;
        F[i] = -qi * a.Fx - a.Lx;
        F[(size_t)n + i] = -qi * a.Fy - a.Ly;
        F[2 * (size_t)n + i] = -qi * a.Fz - a.Lz;
        if constexpr (DIAG) {
            S_out[i] = a.S;
            U_out[i] = a.Ul;
            U_out[(size_t)n + i] = a.Uc;
        }
    }
}

template <int BLOCK, int COMP, bool DIAG, bool CULL>
hipError_t launch_t(const PairLaunch& L, const PairTable& tab, hipStream_t s) {
    const int tiles = (L.n + BLOCK - 1) / BLOCK;
    const int per = (tiles + L.j_split - 1) / L.j_split;
    dim3 grid(tiles, L.j_split);
    hipLaunchKernelGGL((k_pair<BLOCK, COMP, DIAG, CULL>), grid, dim3(BLOCK), 0, s, L.pos, L.lo, L.typ,
                       L.box, L.n, per * BLOCK, L.Fpart, L.S, L.U, tab);
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

}  // namespace

hipError_t launch_pair(const PairLaunch& L, const PairTable& tab, hipStream_t s) {
    switch (L.block) {
        case 64: return launch_b<64>(L, tab, s);
        case 128: return launch_b<128>(L, tab, s);
        case 256: return launch_b<256>(L, tab, s);
        case 512: return launch_b<512>(L, tab, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ld
