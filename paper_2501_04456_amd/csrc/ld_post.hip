// Post-processing on the device (section 3): the pair-distance histogram
// behind the RDF, Eq. (6), the centre-distance histogram behind the radial
// concentration, Eq. (8), moments for the radius of gyration, Eqs. (3)-(4),
// and occupied-box counts for the box-counting dimension.
//
// Distances use the full FP64 positions hi + lo.  Contraction into fma is
// switched off here so each distance rounds exactly as written, which makes
// the integer bin of every pair reproducible.
#include "ld_internal.h"

namespace ld {
namespace {

constexpr int kRdfBlock = 256;
constexpr int kMaxBins = 4096;

__device__ __forceinline__ void full_pos(const float4* pos, const float4* lo, int s,
                                         double x[3]) {
    const float4 h = pos[s], l = lo[s];
    x[0] = (double)h.x + (double)l.x;
    x[1] = (double)h.y + (double)l.y;
    x[2] = (double)h.z + (double)l.z;
}

__global__ __launch_bounds__(kRdfBlock) void k_rdf(const float4* __restrict__ pos,
                                                   const float4* __restrict__ lo, int n,
                                                   double r_max, int n_bins, double dr,
                                                   unsigned long long* counts) {
#pragma clang fp contract(off)
    __shared__ unsigned int hist[kMaxBins];
    __shared__ double sx[kRdfBlock], sy[kRdfBlock], sz[kRdfBlock];
    for (int b = threadIdx.x; b < n_bins; b += kRdfBlock) hist[b] = 0u;
    const int i = blockIdx.x * kRdfBlock + threadIdx.x;
    double xi[3] = {0.0, 0.0, 0.0};
    if (i < n) full_pos(pos, lo, i, xi);
    for (int jt = blockIdx.x * kRdfBlock; jt < n; jt += kRdfBlock) {
        __syncthreads();
        const int j = jt + threadIdx.x;
        if (j < n) {
            double xj[3];
            full_pos(pos, lo, j, xj);
            sx[threadIdx.x] = xj[0];
            sy[threadIdx.x] = xj[1];
            sz[threadIdx.x] = xj[2];
        }
        __syncthreads();
        if (i < n) {
            const int m = min(kRdfBlock, n - jt);
            for (int k = 0; k < m; ++k) {
                if (jt + k <= i) continue;
                const double dx = xi[0] - sx[k];
                const double dy = xi[1] - sy[k];
                const double dz = xi[2] - sz[k];
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r < r_max) {
                    const int b = (int)floor(r / dr);
                    if (b >= 0 && b < n_bins) atomicAdd(&hist[b], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += kRdfBlock)
        if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

// Distances from the centre into bins; typ != null keeps type `want` only.
__global__ __launch_bounds__(256) void k_centre_hist(const float4* __restrict__ pos,
                                                     const float4* __restrict__ lo, int n,
                                                     double r_max, int n_bins, double dr,
                                                     const double* __restrict__ centre,
                                                     unsigned long long* counts,
                                                     const int* __restrict__ typ, int want) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    if (typ && typ[s] != want) return;
    double x[3];
    full_pos(pos, lo, s, x);
    const double dx = x[0] - centre[0], dy = x[1] - centre[1], dz = x[2] - centre[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r < r_max) {
        const int b = (int)floor(r / dr);
        if (b >= 0 && b < n_bins) atomicAdd(&counts[b], 1ull);
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, int m) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < m) p[k] = 0ull;
}

// rows: 0..2 positions, 3..5 filled later by k_dev2
__global__ __launch_bounds__(256) void k_pos_rows(const float4* __restrict__ pos,
                                                  const float4* __restrict__ lo, int n,
                                                  double* work) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    double x[3];
    full_pos(pos, lo, s, x);
    work[s] = x[0];
    work[(size_t)n + s] = x[1];
    work[2 * (size_t)n + s] = x[2];
}

__global__ __launch_bounds__(256) void k_dev2(const float4* __restrict__ pos,
                                              const float4* __restrict__ lo, int n,
                                              const double* __restrict__ sums, double* work) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    double x[3];
    full_pos(pos, lo, s, x);
    const double c0 = sums[0] / n, c1 = sums[1] / n, c2 = sums[2] / n;
    const double dx = c0 - x[0], dy = c1 - x[1], dz = c2 - x[2];
    work[s] = dx * dx + dy * dy + dz * dz;
}

__global__ void k_moments_finish(const double* sums, const double* s2, int n, double* out4) {
    out4[0] = sums[0] / n;
    out4[1] = sums[1] / n;
    out4[2] = sums[2] / n;
    out4[3] = sqrt(s2[0] / n);
}

__global__ __launch_bounds__(256) void k_box_keys(const float4* __restrict__ pos,
                                                  const float4* __restrict__ lo, int n,
                                                  int n_pow2, const double* __restrict__ lo3,
                                                  double eps, unsigned long long* keys) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_pow2) return;
    if (s >= n) {
        keys[s] = ~0ull;
        return;
    }
    double x[3];
    full_pos(pos, lo, s, x);
    const unsigned long long ix = (unsigned long long)floor((x[0] - lo3[0]) / eps);
    const unsigned long long iy = (unsigned long long)floor((x[1] - lo3[1]) / eps);
    const unsigned long long iz = (unsigned long long)floor((x[2] - lo3[2]) / eps);
    keys[s] = (ix << 42) | (iy << 21) | iz;
}

// Compact box keys: (box index << 32) | slot, box index = (ix ny + iy) nz + iz
// with ix, iy, iz formed exactly as in k_box_keys; the caller guarantees
// nx ny nz <= 2^32.
__global__ __launch_bounds__(256) void k_box_keys32(const float4* __restrict__ pos,
                                                    const float4* __restrict__ lo, int n,
                                                    const double* __restrict__ lo3, double eps,
                                                    unsigned long long ny, unsigned long long nz,
                                                    unsigned long long* keys) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    double x[3];
    full_pos(pos, lo, s, x);
    const unsigned long long ix = (unsigned long long)floor((x[0] - lo3[0]) / eps);
    const unsigned long long iy = (unsigned long long)floor((x[1] - lo3[1]) / eps);
    const unsigned long long iz = (unsigned long long)floor((x[2] - lo3[2]) / eps);
    keys[s] = (((ix * ny + iy) * nz + iz) << 32) | (unsigned long long)(unsigned)s;
}

// Distinct high words of keys sorted by them.
__global__ __launch_bounds__(256) void k_count_distinct_high(const unsigned long long* keys, int n,
                                                             unsigned long long* count) {
    __shared__ unsigned int red[256];
    unsigned int c = 0;
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
        c += (s == 0 || (keys[s] >> 32) != (keys[s - 1] >> 32)) ? 1u : 0u;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)red[0]);
}

__global__ __launch_bounds__(256) void k_count_distinct(const unsigned long long* keys, int n,
                                                        unsigned long long* count) {
    __shared__ unsigned int red[256];
    unsigned int c = 0;
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
        c += (s == 0 || keys[s] != keys[s - 1]) ? 1u : 0u;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)red[0]);
}

__global__ __launch_bounds__(256) void k_set_charge(float4* pos, const int* __restrict__ oid,
                                                   const float* __restrict__ qhat, int n) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) pos[s].w = qhat[oid[s]];
}

}  // namespace

hipError_t launch_rdf(const float4* pos, const float4* lo, int n, double r_max, int n_bins,
                      const double* centre, unsigned long long* counts,
                      unsigned long long* ccounts, hipStream_t s) {
    if (n_bins < 1 || n_bins > kMaxBins) return hipErrorInvalidValue;
    const double dr = r_max / n_bins;
    hipLaunchKernelGGL(k_zero_u64, dim3((n_bins + 255) / 256), dim3(256), 0, s, counts, n_bins);
    hipLaunchKernelGGL(k_zero_u64, dim3((n_bins + 255) / 256), dim3(256), 0, s, ccounts, n_bins);
    hipLaunchKernelGGL(k_rdf, dim3((n + kRdfBlock - 1) / kRdfBlock), dim3(kRdfBlock), 0, s, pos,
                       lo, n, r_max, n_bins, dr, counts);
    hipLaunchKernelGGL(k_centre_hist, dim3((n + 255) / 256), dim3(256), 0, s, pos, lo, n, r_max,
                       n_bins, dr, centre, ccounts, nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_centre_hist(const float4* pos, const float4* lo, const int* typ, int want, int n,
                              double r_max, int n_bins, const double* centre,
                              unsigned long long* ccounts, hipStream_t s) {
    if (n_bins < 1 || n_bins > kMaxBins) return hipErrorInvalidValue;
    const double dr = r_max / n_bins;
    hipLaunchKernelGGL(k_zero_u64, dim3((n_bins + 255) / 256), dim3(256), 0, s, ccounts, n_bins);
    hipLaunchKernelGGL(k_centre_hist, dim3((n + 255) / 256), dim3(256), 0, s, pos, lo, n, r_max,
                       n_bins, dr, centre, ccounts, typ, want);
    return hipGetLastError();
}

hipError_t launch_pos_rows(const float4* pos, const float4* lo, int n, double* work,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_pos_rows, dim3((n + 255) / 256), dim3(256), 0, s, pos, lo, n, work);
    return hipGetLastError();
}

hipError_t launch_set_charge(float4* pos, const int* oid, const float* qhat, int n,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_set_charge, dim3((n + 255) / 256), dim3(256), 0, s, pos, oid, qhat, n);
    return hipGetLastError();
}

hipError_t launch_moments(const float4* pos, const float4* lo, int n, double* work,
                          double* out4, hipStream_t s) {
    const dim3 g((n + 255) / 256);
    double* sums = work + 3 * (size_t)n;
    double* s2 = sums + 4;
    hipLaunchKernelGGL(k_pos_rows, g, dim3(256), 0, s, pos, lo, n, work);
    hipError_t e = launch_rowsum(work, 3, n, sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dev2, g, dim3(256), 0, s, pos, lo, n, sums, work);
    e = launch_rowsum(work, 1, n, s2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_finish, dim3(1), dim3(1), 0, s, sums, s2, n, out4);
    return hipGetLastError();
}

hipError_t launch_boxcount_radix(const float4* pos, const float4* lo, int n, const double* lo3,
                                 double eps, unsigned long long ny, unsigned long long nz,
                                 int bits, unsigned long long* keys, unsigned long long* tmp,
                                 unsigned* hist, unsigned long long* count, hipStream_t s) {
    hipLaunchKernelGGL(k_box_keys32, dim3((n + 255) / 256), dim3(256), 0, s, pos, lo, n, lo3, eps,
                       ny, nz, keys);
    unsigned long long* sorted = nullptr;
    hipError_t e = launch_radix_by_high(keys, tmp, n, bits, hist, s, false, &sorted);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, count, 1);
    hipLaunchKernelGGL(k_count_distinct_high, dim3(64), dim3(256), 0, s, sorted, n, count);
    return hipGetLastError();
}

hipError_t launch_boxcount(const float4* pos, const float4* lo, int n, const double* lo3,
                           double eps, unsigned long long* keys, int n_pow2,
                           unsigned long long* count, hipStream_t s) {
    hipLaunchKernelGGL(k_box_keys, dim3((n_pow2 + 255) / 256), dim3(256), 0, s, pos, lo, n,
                       n_pow2, lo3, eps, keys);
    hipError_t e = launch_bitonic(keys, n_pow2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, count, 1);
    hipLaunchKernelGGL(k_count_distinct, dim3(64), dim3(256), 0, s, keys, n, count);
    return hipGetLastError();
}

}  // namespace ld
