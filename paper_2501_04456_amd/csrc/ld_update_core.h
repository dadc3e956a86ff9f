// Per-particle pieces of the update (section 2.2 steps (iii)-(vi)) shared by
// the single-droplet and ensemble update kernels: the Philox noise stream,
// the external forces and the group bounding boxes.
#pragma once

#include "ld_internal.h"

namespace ld {
namespace upd {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ((u >> 9) + 1/2) 2^-23: exact in FP32 and FP64.
__device__ __forceinline__ double u23(uint32_t u) {
    return ((double)(u >> 9) + 0.5) * (1.0 / 8388608.0);
}

// Three standard normals for particle id at step n (Box-Muller in FP64: the
// logarithm, square root and sine/cosine in FP32 would carry relative errors
// of ~1e-7, which a stiff Lennard-Jones contact turns into a visible drift of
// the trajectory; in FP64 they cost well under a microsecond per step).
__device__ __forceinline__ void gauss3(uint32_t id, unsigned long long n, unsigned long long seed,
                                       double xi[3]) {
    uint32_t c0 = id, c1 = (uint32_t)n, c2 = (uint32_t)(n >> 32), c3 = 0u;
    philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double a = sqrt(-2.0 * log(u23(c0)));
    const double b = sqrt(-2.0 * log(u23(c2)));
    double s1, k1, s3, k3;
    sincospi(2.0 * u23(c1), &s1, &k1);
    sincospi(2.0 * u23(c3), &s3, &k3);
    xi[0] = a * k1;
    xi[1] = a * s1;
    xi[2] = b * k3;
}

// External force at x for type t and droplet radius R (FP64): the surface
// spring (one-sided, equilibrium wall_offset inside R; band mode limits it to
// within sigma/2 of R), gravity and the centrifugal force.
__device__ __forceinline__ void ext_force(const double x[3], int t, double R,
                                          const ExtParams& P, double F[3]) {
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double Rw = R - P.wall_offset[t];
    bool on = r > Rw;
    if (P.wall_band) {
        const double h = P.half_sigma[t];
        on = on && (r > R - h) && (r < R + h);
    }
    const double m = (on && r > 0.0) ? -P.k_wall[t] * (r - Rw) / r : 0.0;
    const double c = P.mass[t] * P.omega2;
    F[0] = m * x[0] + P.mass[t] * P.gravity[0] + c * x[0];
    F[1] = m * x[1] + P.mass[t] * P.gravity[1] + c * x[1];
    F[2] = m * x[2] + P.mass[t] * P.gravity[2] + (P.rotation == 0 ? c * x[2] : 0.0);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Bounding box of each 64-slot group (one wavefront per group); lo.w = 1 if
// the group holds a charged particle, else 0.
__device__ __forceinline__ void write_box(const float4 h, bool live, int s, Box* box) {
    const float lx = wave_min(live ? h.x : INFINITY), hx = wave_max(live ? h.x : -INFINITY);
    const float ly = wave_min(live ? h.y : INFINITY), hy = wave_max(live ? h.y : -INFINITY);
    const float lz = wave_min(live ? h.z : INFINITY), hz = wave_max(live ? h.z : -INFINITY);
    const bool charged = __any(live && h.w != 0.f);
    if ((threadIdx.x & (kGroup - 1)) == 0 && lx <= hx) {
        Box b;
        b.lo = make_float4(lx, ly, lz, charged ? 1.f : 0.f);
        b.hi = make_float4(hx, hy, hz, 0.f);
        box[s / kGroup] = b;
    }
}

// One overdamped Euler-Maruyama step of one particle held as an FP32 pair
// (h, l) whose sum is the FP64 position:
//   x <- x + mu dt (F_pair + F_ext(R)) + sqrt(2 kT mu dt) xi.
// Returns false if a move component is non-finite or exceeds jump_max.
__device__ __forceinline__ bool advance(float4& h, float4& l, const double F[3], int ty,
                                        double R, double dt, const ExtParams& P, uint32_t id,
                                        unsigned long long step, unsigned long long seed) {
    const double x[3] = {(double)h.x + (double)l.x, (double)h.y + (double)l.y,
                         (double)h.z + (double)l.z};
    double Fe[3];
    ext_force(x, ty, R, P, Fe);
    const double mu = P.mu[ty];
    double xi[3] = {0.0, 0.0, 0.0};
    double amp = 0.0;
    if (P.noise != 0 && P.kT > 0.0) {
        gauss3(id, step, seed, xi);
        amp = sqrt(2.0 * P.kT * mu * dt);
        if (P.noise == 2) {
            const double m = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
            const double f = 1.7320508075688772 / m;
            xi[0] *= f; xi[1] *= f; xi[2] *= f;
        }
    }
    bool ok = true;
    double xn[3];
    for (int c = 0; c < 3; ++c) {
        const double d = mu * dt * (F[c] + Fe[c]) + amp * xi[c];
        if (!isfinite(d) || (P.jump_max > 0.0 && fabs(d) > P.jump_max)) ok = false;
        xn[c] = x[c] + d;
    }
    h.x = (float)xn[0];
    h.y = (float)xn[1];
    h.z = (float)xn[2];
    l = make_float4((float)(xn[0] - (double)h.x), (float)(xn[1] - (double)h.y),
                    (float)(xn[2] - (double)h.z), 0.f);
    return ok;
}

}  // namespace upd
}  // namespace ld
