// Spatial ordering of the particle slots along a Hilbert curve, so
// that every 64-slot group is spatially compact and the pair kernel can cull
// Lennard-Jones range tests per group pair.  The ordering is a permutation
// of slots only: each slot carries its original index, which keys the
// Brownian noise and orders every output.
//
// Sorting is a 64-bit bitonic network: 2048-key chunks are sorted and merged
// inside LDS, longer strides run as one global compare-exchange pass each.
#include "ld_internal.h"

namespace ld {
namespace {

constexpr int kLocal = 2048;      // keys per LDS chunk (1024 work-items, 2 keys each)

__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* keys, int k_fixed) {
    __shared__ unsigned long long sk[kLocal];
    const int base = blockIdx.x * kLocal;
    const int t = threadIdx.x;
    sk[t] = keys[base + t];
    sk[t + 1024] = keys[base + t + 1024];
    __syncthreads();
    // k_fixed == 0: sort the chunk completely (all stages k <= kLocal);
    // otherwise finish stage k_fixed for strides j < kLocal.
    const int k_lo = k_fixed ? k_fixed : 2;
    const int k_hi = k_fixed ? k_fixed : kLocal;
    for (int k = k_lo; k <= k_hi; k <<= 1) {
        for (int j = (k_fixed ? kLocal / 2 : k / 2); j > 0; j >>= 1) {
            const int i = (t / j) * 2 * j + (t % j);
            const int l = i + j;
            const bool asc = (((base + i) & k) == 0);
            const unsigned long long a = sk[i], b = sk[l];
            if ((a > b) == asc) {
                sk[i] = b;
                sk[l] = a;
            }
            __syncthreads();
        }
    }
    keys[base + t] = sk[t];
    keys[base + t + 1024] = sk[t + 1024];
}

__global__ __launch_bounds__(256) void k_bitonic_global(unsigned long long* keys, int npairs,
                                                        int k, int j) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= npairs) return;
    const int i = (t / j) * 2 * j + (t % j);
    const int l = i + j;
    const bool asc = ((i & k) == 0);
    const unsigned long long a = keys[i], b = keys[l];
    if ((a > b) == asc) {
        keys[i] = b;
        keys[l] = a;
    }
}

// Per-block min / max of the hi positions.
__global__ __launch_bounds__(256) void k_bounds_part(const float4* __restrict__ pos, int n,
                                                     float* part) {
    __shared__ float red[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
        const float4 h = pos[s];
        v[0] = fminf(v[0], h.x); v[1] = fminf(v[1], h.y); v[2] = fminf(v[2], h.z);
        v[3] = fmaxf(v[3], h.x); v[4] = fmaxf(v[4], h.y); v[5] = fmaxf(v[5], h.z);
    }
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 3; ++c)
                red[c][threadIdx.x] = fminf(red[c][threadIdx.x], red[c][threadIdx.x + w]);
            for (int c = 3; c < 6; ++c)
                red[c][threadIdx.x] = fmaxf(red[c][threadIdx.x], red[c][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}


__global__ __launch_bounds__(256) void k_curve_keys(const float4* __restrict__ pos, int n,
                                                    int n_pow2, const float* __restrict__ part,
                                                    int nparts, unsigned long long* keys) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_pow2) return;
    if (s >= n) {
        keys[s] = ~0ull;
        return;
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nparts; ++b)
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], part[b * 6 + c]);
            hi[c] = fmaxf(hi[c], part[b * 6 + 3 + c]);
        }
    const float ext = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), fmaxf(hi[2] - lo[2], 1e-30f));
    const float scale = 1023.0f / ext;
    const float4 h = pos[s];
    const unsigned qx = (unsigned)fminf(1023.f, fmaxf(0.f, (h.x - lo[0]) * scale));
    const unsigned qy = (unsigned)fminf(1023.f, fmaxf(0.f, (h.y - lo[1]) * scale));
    const unsigned qz = (unsigned)fminf(1023.f, fmaxf(0.f, (h.z - lo[2]) * scale));
    const unsigned code = hilbert_index<10>(qx, qy, qz);
    // Uncharged particles go after all charged ones (bit 62), so 64-slot
    // groups are charge-homogeneous and the pair kernel can skip far group
    // pairs whose Coulomb term is identically zero.
    const unsigned long long neutral = (h.w == 0.f) ? 1ull : 0ull;
    keys[s] = (neutral << 62) | ((unsigned long long)code << 32) | (unsigned)s;
}

__global__ __launch_bounds__(256) void k_permute4(const unsigned long long* __restrict__ keys,
                                                  int n, const float4* __restrict__ a,
                                                  float4* __restrict__ b) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) b[s] = a[(int)(unsigned)keys[s]];
}

__global__ __launch_bounds__(256) void k_permute1(const unsigned long long* __restrict__ keys,
                                                  int n, const int* __restrict__ a,
                                                  int* __restrict__ b) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) b[s] = a[(int)(unsigned)keys[s]];
}

}  // namespace

hipError_t launch_bitonic(unsigned long long* keys, int n_pow2, hipStream_t s) {
    if (n_pow2 < kLocal || (n_pow2 & (n_pow2 - 1))) return hipErrorInvalidValue;
    const int chunks = n_pow2 / kLocal;
    hipLaunchKernelGGL(k_bitonic_local, dim3(chunks), dim3(1024), 0, s, keys, 0);
    const int npairs = n_pow2 / 2;
    for (int k = 2 * kLocal; k <= n_pow2; k <<= 1) {
        for (int j = k / 2; j >= kLocal; j >>= 1) {
            hipLaunchKernelGGL(k_bitonic_global, dim3((npairs + 255) / 256), dim3(256), 0, s,
                               keys, npairs, k, j);
        }
        hipLaunchKernelGGL(k_bitonic_local, dim3(chunks), dim3(1024), 0, s, keys, k);
    }
    return hipGetLastError();
}

hipError_t launch_sort(float4* pos, float4* lo, int* typ, int* oid, int n, const SortBuffers& B,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_bounds_part, dim3(B.bounds_parts), dim3(256), 0, s, pos, n,
                       B.bounds_part);
    hipLaunchKernelGGL(k_curve_keys, dim3((B.n_pow2 + 255) / 256), dim3(256), 0, s, pos, n, B.n_pow2,
                       B.bounds_part, B.bounds_parts, B.keys);
    return launch_sort_by_keys(pos, lo, typ, oid, n, B, s);
}

hipError_t launch_sort_by_keys(float4* pos, float4* lo, int* typ, int* oid, int n,
                               const SortBuffers& B, hipStream_t s) {
    hipError_t e = launch_bitonic(B.keys, B.n_pow2, s);
    if (e != hipSuccess) return e;
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(k_permute4, g, dim3(256), 0, s, B.keys, n, pos, B.tmp4);
    e = hipMemcpyAsync(pos, B.tmp4, sizeof(float4) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_permute4, g, dim3(256), 0, s, B.keys, n, lo, B.tmp4);
    e = hipMemcpyAsync(lo, B.tmp4, sizeof(float4) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_permute1, g, dim3(256), 0, s, B.keys, n, typ, B.tmp_i);
    e = hipMemcpyAsync(typ, B.tmp_i, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_permute1, g, dim3(256), 0, s, B.keys, n, oid, B.tmp_i);
    e = hipMemcpyAsync(oid, B.tmp_i, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace ld
