// Inner loops of the all-pairs force sum, shared by the single-droplet
// kernel (ld_pair.hip) and the ensemble kernel (ld_ens.hip).
//
// Per pair the Coulomb-only path is 12 FP32 VALU operations plus one
// v_rsq_f32: three subtractions, r^2 as mul+fma+fma, q_j r^-3 as three
// multiplications and three fma into FP32 block accumulators.  Each lane sums
// KB = 32 pair terms in FP32 and then moves the block into FP64 totals
// (COMP=0) or into a blocked Kahan pair (COMP=1); LJ terms (near groups
// only) are computed and summed in FP64 by their own kernel.  The
// worst-case rounding of a 32-term FP32 block is 31 u sum|f| ~ 1.8e-6 of
// S_i = sum_j |f_ij|.
#pragma once

#include "ld_internal.h"

namespace ld {
namespace pair {

// Upper bound on the FP32 1/r of the near loops: 1/r of any two distinct
// particles is far below it (they never come within 1e-10 sigma), and
// |q_j| kInvRCap^3 stays finite, so the self pair (r = 0) adds w * 0 = 0.
// Two distinct particles at bitwise equal positions would get a zero
// Coulomb term here (their Lennard-Jones term is still infinite).
constexpr float kInvRCap = 1e10f;

constexpr int KB = 32;

struct Acc {
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;   // sum_j q_j r^-3 (x_j - x_i), FP64
    float sx = 0.f, sy = 0.f, sz = 0.f;    // Kahan sums (COMP == 1)
    float cx = 0.f, cy = 0.f, cz = 0.f;    // Kahan compensations
    double S = 0.0, Uc = 0.0;              // diagnostic mode only (Coulomb part)
};

template <int COMP>
__device__ __forceinline__ void flush(Acc& a, float bx, float by, float bz) {
    if constexpr (COMP == 0) {
        a.Fx += (double)bx;
        a.Fy += (double)by;
        a.Fz += (double)bz;
    } else {
        float y, t;
        y = bx - a.cx; t = a.sx + y; a.cx = (t - a.sx) - y; a.sx = t;
        y = by - a.cy; t = a.sy + y; a.cy = (t - a.sy) - y; a.sy = t;
        y = bz - a.cz; t = a.sz + y; a.cz = (t - a.sz) - y; a.sz = t;
    }
}

// 64 j particles with no LJ partner in range and no self pair: Coulomb only.
// UNROLL: pairs in flight per lane; full unrolling (32) suits the
// single-droplet kernel's register budget, the ensemble kernel takes fewer.
template <int COMP, int UNROLL = 32>
__device__ __forceinline__ void group_far(const float4* __restrict__ sp, const float4 pi,
                                          Acc& a) {
#pragma unroll
    for (int kb = 0; kb < kGroup; kb += KB) {
        float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll UNROLL
        for (int k = 0; k < KB; ++k) {
            const float4 pj = sp[kb + k];
            const float dx = pj.x - pi.x;
            const float dy = pj.y - pi.y;
            const float dz = pj.z - pi.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float w = (pj.w * ri) * (ri * ri);
            bx = fmaf(w, dx, bx);
            by = fmaf(w, dy, by);
            bz = fmaf(w, dz, bz);
        }
        flush<COMP>(a, bx, by, bz);
    }
}

// 64 j particles near i's group (within the largest LJ range of its box) or
// holding i itself: the Coulomb terms with the low words of the positions
// in the differences, the self pair left out.  The difference of the FP32
// high words of two nearby particles is exact, and adding the difference of
// their low words gives r_ij to FP32 rounding of r_ij itself.  Used where
// the relative positions below would lose too much (a workgroup whose box
// is stretched by NPs thrown far out).  Returns whether any j of the group
// lies within sqrt(lj2) of i (i itself counts, so the group holding i is
// always flagged; the Lennard-Jones kernels skip j = i).
template <int COMP, bool DIAG>
__device__ __forceinline__ bool group_near(const float4* __restrict__ sp,
                                           const float4* __restrict__ sl, int jbase, int i,
                                           const float4 pi, const float4 li, float lj2, Acc& a) {
    bool lj_any = false;
#pragma unroll
    for (int kb = 0; kb < kGroup; kb += KB) {
        float bx = 0.f, by = 0.f, bz = 0.f;   // Coulomb, FP32 block
#pragma unroll 4
        for (int k = 0; k < KB; ++k) {
            const float4 pj = sp[kb + k];
            const float4 lj = sl[kb + k];
            const float dx = (pj.x - pi.x) + (lj.x - li.x);
            const float dy = (pj.y - pi.y) + (lj.y - li.y);
            const float dz = (pj.z - pi.z) + (lj.z - li.z);
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            // the self pair has dx = dy = dz = 0 exactly; capping 1/r keeps
            // its weight finite, so its term is 0 without a test
            const float ri = fminf(__builtin_amdgcn_rsqf(r2), kInvRCap);
            const float w = (pj.w * ri) * (ri * ri);
            lj_any |= r2 < lj2;                 // the self pair flags the diagonal group
            if constexpr (DIAG) {
                if (jbase + kb + k != i) {
                    const float qq = pi.w * pj.w;
                    a.S += (double)(fabsf(qq) * ri * ri);
                    a.Uc += 0.5 * (double)(qq * ri);
                }
            }
            bx = fmaf(w, dx, bx);
            by = fmaf(w, dy, by);
            bz = fmaf(w, dz, bz);
        }
        flush<COMP>(a, bx, by, bz);
    }
    return lj_any;
}

// 64 j particles near i's group (within the largest LJ range of its box) or
// holding i itself: the Coulomb terms, the self pair left out, from
// positions taken relative to an origin c near both groups (the centre of
// the box of the workgroup's slots, or of the ensemble tile's box).  Each
// staged j and the lane's own i hold (hi - c) + lo rounded to FP32, so a
// difference carries the rounding of |x - c| (tens of sigma for the groups
// this loop sees) instead of |x|: near |x| = 300 sigma one ulp of a
// coordinate is 3e-5 sigma, which at contact distance would move a Coulomb
// term by ~1e-4 of itself; at |x - c| = 64 sigma it is 8e-6 sigma.  One LDS
// read and three subtractions per pair, as in the far loop.  The
// Lennard-Jones terms of these groups are added by a kernel of their own
// (k_lj), in FP64 from the exact (hi, lo) differences.  Returns whether any
// j of the group lies within sqrt(lj2) of i (i itself counts, so the group
// holding i is always flagged): the Lennard-Jones kernel visits only such
// group pairs and skips j = i.
template <int COMP, bool DIAG>
__device__ __forceinline__ bool group_near_rel(const float4* __restrict__ sr, int jbase, int i,
                                               const float4 ri4, float lj2, Acc& a) {
    bool lj_any = false;
#pragma unroll
    for (int kb = 0; kb < kGroup; kb += KB) {
        float bx = 0.f, by = 0.f, bz = 0.f;   // Coulomb, FP32 block
#pragma unroll 4
        for (int k = 0; k < KB; ++k) {
            const float4 pj = sr[kb + k];
            const float dx = pj.x - ri4.x, dy = pj.y - ri4.y, dz = pj.z - ri4.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            // the self pair has dx = dy = dz = 0 exactly; capping 1/r keeps
            // its weight finite, so its term is 0 without a test
            const float ri = fminf(__builtin_amdgcn_rsqf(r2), kInvRCap);
            const float w = (pj.w * ri) * (ri * ri);
            lj_any |= r2 < lj2;                 // the self pair flags the diagonal group
            if constexpr (DIAG) {
                if (jbase + kb + k != i) {
                    const float qq = ri4.w * pj.w;
                    a.S += (double)(fabsf(qq) * ri * ri);
                    a.Uc += 0.5 * (double)(qq * ri);
                }
            }
            bx = fmaf(w, dx, bx);
            by = fmaf(w, dy, by);
            bz = fmaf(w, dz, bz);
        }
        flush<COMP>(a, bx, by, bz);
    }
    return lj_any;
}

// One Lennard-Jones pair (section 2.1: truncated at lj_cut sigma_ij, not
// shifted) in FP64 from the exact difference of the (hi, lo) positions, if
// it is within the cutoff.  t64: sigma_ij^2, 24 eps_ij, 4 eps_ij and
// (lj_cut sigma_ij)^2, each kMaxTypes^2 long.  Near the minimum the force is
// a small difference of two large terms; FP32 operands would leave an error
// of ~1e-6 of 24 eps_ij / r there.  Accumulates sum_j g_ij (x_j - x_i) and,
// with DIAG, |f_ij| and half the pair energy.
template <bool DIAG>
__device__ __forceinline__ void lj_pair64(const float4 pj, const float4 lj, const float4 pi,
                                          const float4 li, const double* __restrict__ t64,
                                          int pidx, double L[3], double& S, double& U) {
    const double ex = ((double)pj.x - (double)pi.x) + ((double)lj.x - (double)li.x);
    const double ey = ((double)pj.y - (double)pi.y) + ((double)lj.y - (double)li.y);
    const double ez = ((double)pj.z - (double)pi.z) + ((double)lj.z - (double)li.z);
    const double q2 = ex * ex + ey * ey + ez * ez;
    if (!(q2 < t64[3 * kMaxTypes * kMaxTypes + pidx])) return;
    const double ir2 = 1.0 / q2;
    const double s2 = t64[pidx] * ir2;                         // sigma_ij^2 / r^2
    const double s6 = s2 * s2 * s2;
    const double g = t64[kMaxTypes * kMaxTypes + pidx] * s6 * (2.0 * s6 - 1.0) * ir2;
    L[0] += g * ex;
    L[1] += g * ey;
    L[2] += g * ez;
    if constexpr (DIAG) {
        S += fabs(g) * sqrt(q2);
        U += 0.5 * (t64[2 * kMaxTypes * kMaxTypes + pidx] * s6 * (s6 - 1.0));
    }
}

__device__ __forceinline__ float box_dist2(const Box& a, const Box& b) {
    const float gx = fmaxf(0.f, fmaxf(b.lo.x - a.hi.x, a.lo.x - b.hi.x));
    const float gy = fmaxf(0.f, fmaxf(b.lo.y - a.hi.y, a.lo.y - b.hi.y));
    const float gz = fmaxf(0.f, fmaxf(b.lo.z - a.hi.z, a.lo.z - b.hi.z));
    return gx * gx + gy * gy + gz * gz;
}

// Squared distance from point p to box b (0 inside; NaN coordinates give 0).
__device__ __forceinline__ float point_box_dist2(const float4& p, const Box& b) {
    const float gx = fmaxf(0.f, fmaxf(b.lo.x - p.x, p.x - b.hi.x));
    const float gy = fmaxf(0.f, fmaxf(b.lo.y - p.y, p.y - b.hi.y));
    const float gz = fmaxf(0.f, fmaxf(b.lo.z - p.z, p.z - b.hi.z));
    return gx * gx + gy * gy + gz * gz;
}

}  // namespace pair
}  // namespace ld
