// O(N) kernels of a step: external forces, Brownian noise and the overdamped
// Langevin update (section 2.2, steps (iii)-(vi)), plus gathers and
// deterministic reductions used by the force and diagnostic calls.
#include "ld_update_core.h"

namespace ld {
namespace {

using namespace upd;

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_update(StepLaunch L, ExtParams P) {
    const long long step = L.st->step;
    const double t = L.st->t;
    const double tn = t + L.dt;
    const double R = radius_at(P.R, tn);   // the new radius precedes the surface forces
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const bool live = s < L.n;
    float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live) {
        h = L.pos[s];
        const float4 l = L.lo[s];
        const int ty = L.typ[s];
        double F[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < L.j_split; ++k) {
            const double* Fp = L.Fpart + (size_t)k * 3 * (size_t)L.n;
            F[0] += Fp[s];
            F[1] += Fp[(size_t)L.n + s];
            F[2] += Fp[2 * (size_t)L.n + s];
        }
        float4 nl = l;
        if (!advance(h, nl, F, ty, R, L.dt, P, (uint32_t)L.oid[s], (unsigned long long)step,
                     L.seed))
            atomicMin(&L.st->bad_step, (unsigned long long)step);
        L.pos[s] = h;
        L.lo[s] = nl;
    }
    if (L.box) write_box(h, live, s, L.box);
}

// Step counter and time advance after the update (a launch of its own: a
// per-workgroup completion count would serialise one device-scope atomic
// and fence per workgroup).  t_{n+1} = t_n + dt as the update computed it.
__global__ void k_advance(DevState* st, double dt) {
    st->t = st->t + dt;
    st->step = st->step + 1;
}

__global__ __launch_bounds__(kBlock) void k_boxes(const float4* __restrict__ pos, int n,
                                                  Box* box) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const bool live = s < n;
    const float4 h = live ? pos[s] : make_float4(0.f, 0.f, 0.f, 0.f);
    write_box(h, live, s, box);
}

__global__ __launch_bounds__(kBlock) void k_gather(
    const float4* __restrict__ pos, const float4* __restrict__ lo, const int* __restrict__ typ,
    const int* __restrict__ oid, const double* __restrict__ Fpart, int j_split,
    const double* __restrict__ S_slot, int n, const DevState* st, ExtParams P, double* F_pair,
    double* F_ext, double* S) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int o = oid[s];
    if (F_pair) {
        double F[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < j_split; ++k) {
            const double* Fp = Fpart + (size_t)k * 3 * (size_t)n;
            F[0] += Fp[s];
            F[1] += Fp[(size_t)n + s];
            F[2] += Fp[2 * (size_t)n + s];
        }
        F_pair[3 * (size_t)o] = F[0];
        F_pair[3 * (size_t)o + 1] = F[1];
        F_pair[3 * (size_t)o + 2] = F[2];
    }
    if (F_ext) {
        const float4 h = pos[s], l = lo[s];
        const double x[3] = {(double)h.x + (double)l.x, (double)h.y + (double)l.y,
                             (double)h.z + (double)l.z};
        double Fe[3];
        ext_force(x, typ[s], radius_at(P.R, st->t), P, Fe);
        F_ext[3 * (size_t)o] = Fe[0];
        F_ext[3 * (size_t)o + 1] = Fe[1];
        F_ext[3 * (size_t)o + 2] = Fe[2];
    }
    if (S) S[o] = S_slot[s];
}

// One workgroup per row; each lane reduces a fixed strided subset in order,
// then a fixed tree: the result depends only on n.  OP: 0 sum, 1 max, 2 min.
template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
    if constexpr (OP == 0) return a + b;
    else if constexpr (OP == 1) return fmax(a, b);
    else return fmin(a, b);
}

template <int OP>
__global__ __launch_bounds__(1024) void k_rowreduce(const double* __restrict__ in, int n,
                                                    double* out) {
    __shared__ double red[1024];
    const double* row = in + (size_t)blockIdx.x * (size_t)n;
    double acc = OP == 0 ? 0.0 : (OP == 1 ? -INFINITY : INFINITY);
    for (int k = threadIdx.x; k < n; k += 1024) acc = red_op<OP>(acc, row[k]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red_op<OP>(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Per-slot diagnostic terms: rows 0 U_wall, 1 U_grav, 2 U_cf, 3-5 F_pair,
// 6 |F_pair|, 7 |x|.
__global__ __launch_bounds__(kBlock) void k_diag_terms(
    const float4* __restrict__ pos, const float4* __restrict__ lo, const int* __restrict__ typ,
    const double* __restrict__ Fpart, int j_split, int n, const DevState* st, ExtParams P,
    double* work) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    const int t = typ[s];
    const double x[3] = {(double)h.x + (double)l.x, (double)h.y + (double)l.y,
                         (double)h.z + (double)l.z};
    const double R = radius_at(P.R, st->t);
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double Rw = R - P.wall_offset[t];
    bool on = r > Rw;
    if (P.wall_band) on = on && (r > R - P.half_sigma[t]) && (r < R + P.half_sigma[t]);
    const size_t N = (size_t)n;
    work[s] = on ? 0.5 * P.k_wall[t] * (r - Rw) * (r - Rw) : 0.0;
    work[N + s] = -P.mass[t] * (P.gravity[0] * x[0] + P.gravity[1] * x[1] + P.gravity[2] * x[2]);
    const double rho2 = x[0] * x[0] + x[1] * x[1] + (P.rotation == 0 ? x[2] * x[2] : 0.0);
    work[2 * N + s] = -0.5 * P.mass[t] * P.omega2 * rho2;
    double F[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < j_split; ++k) {
        const double* Fp = Fpart + (size_t)k * 3 * N;
        F[0] += Fp[s];
        F[1] += Fp[N + s];
        F[2] += Fp[2 * N + s];
    }
    work[3 * N + s] = F[0];
    work[4 * N + s] = F[1];
    work[5 * N + s] = F[2];
    work[6 * N + s] = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    work[7 * N + s] = r;
}

__global__ void k_diag_finish(const double* sums, const double* maxes, const double* U,
                              double* out) {
    out[0] = U[0];
    out[1] = U[1];
    out[2] = sums[0];
    out[3] = sums[1];
    out[4] = sums[2];
    out[5] = sums[3];
    out[6] = sums[4];
    out[7] = sums[5];
    out[8] = maxes[0];
    out[9] = maxes[1];
}

// MSD reference: the FP64 position hi + lo of every NP, in original order
// ([3][n]).
__global__ __launch_bounds__(kBlock) void k_msd_ref(const float4* __restrict__ pos,
                                                   const float4* __restrict__ lo,
                                                   const int* __restrict__ oid, int n,
                                                   double* __restrict__ ref) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    const size_t o = (size_t)oid[s], N = (size_t)n;
    ref[o] = (double)h.x + (double)l.x;
    ref[N + o] = (double)h.y + (double)l.y;
    ref[2 * N + o] = (double)h.z + (double)l.z;
}

// Squared displacement of every slot from its reference position.
__global__ __launch_bounds__(kBlock) void k_msd_terms(const float4* __restrict__ pos,
                                                     const float4* __restrict__ lo,
                                                     const int* __restrict__ oid, int n,
                                                     const double* __restrict__ ref,
                                                     double* __restrict__ work) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    const size_t o = (size_t)oid[s], N = (size_t)n;
    const double dx = ((double)h.x + (double)l.x) - ref[o];
    const double dy = ((double)h.y + (double)l.y) - ref[N + o];
    const double dz = ((double)h.z + (double)l.z) - ref[2 * N + o];
    work[s] = dx * dx + dy * dy + dz * dz;
}

__global__ void k_mean_finish(double* v, int n) { v[0] = v[0] / (double)n; }

}  // namespace

hipError_t launch_msd_ref(const float4* pos, const float4* lo, const int* oid, int n,
                          double* ref, hipStream_t s) {
    hipLaunchKernelGGL(k_msd_ref, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, lo,
                       oid, n, ref);
    return hipGetLastError();
}

hipError_t launch_msd(const float4* pos, const float4* lo, const int* oid, int n,
                      const double* ref, double* work, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_msd_terms, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, lo,
                       oid, n, ref, work);
    hipLaunchKernelGGL(k_rowreduce<0>, dim3(1), dim3(1024), 0, s, work, n, out);
    hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(1), 0, s, out, n);
    return hipGetLastError();
}

hipError_t launch_update(const StepLaunch& L, const ExtParams& P, hipStream_t s) {
    const int blocks = (L.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_update, dim3(blocks), dim3(kBlock), 0, s, L, P);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, L.st, L.dt);
    return hipGetLastError();
}

hipError_t launch_advance(DevState* st, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, st, dt);
    return hipGetLastError();
}

hipError_t launch_boxes(const float4* pos, int n, Box* box, hipStream_t s) {
    const int blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_boxes, dim3(blocks), dim3(kBlock), 0, s, pos, n, box);
    return hipGetLastError();
}

hipError_t launch_gather(const float4* pos, const float4* lo, const int* typ, const int* oid,
                         const double* Fpart, int j_split, const double* S_slot, int n,
                         const DevState* st, const ExtParams& P, double* F_pair,
                         double* F_ext, double* S, hipStream_t s) {
    const int blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kBlock), 0, s, pos, lo, typ, oid, Fpart,
                       j_split, S_slot, n, st, P, F_pair, F_ext, S);
    return hipGetLastError();
}

hipError_t launch_rowsum(const double* in, int rows, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_rowreduce<0>, dim3(rows), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_rowmin(const double* in, int rows, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_rowreduce<2>, dim3(rows), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_rowmax(const double* in, int rows, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_rowreduce<1>, dim3(rows), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_diag(const float4* pos, const float4* lo, const int* typ,
                       const double* Fpart, int j_split, const double* U_slot, int n,
                       const DevState* st, const ExtParams& P, double* work, double* out,
                       hipStream_t s) {
    const int blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_diag_terms, dim3(blocks), dim3(kBlock), 0, s, pos, lo, typ, Fpart,
                       j_split, n, st, P, work);
    double* sums = work + 8 * (size_t)n;
    double* maxes = sums + 8;
    double* U = maxes + 8;
    hipLaunchKernelGGL(k_rowreduce<0>, dim3(6), dim3(1024), 0, s, work, n, sums);
    hipLaunchKernelGGL(k_rowreduce<1>, dim3(2), dim3(1024), 0, s, work + 6 * (size_t)n, n,
                       maxes);
    hipLaunchKernelGGL(k_rowreduce<0>, dim3(2), dim3(1024), 0, s, U_slot, n, U);
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(1), 0, s, sums, maxes, U, out);
    return hipGetLastError();
}

}  // namespace ld
