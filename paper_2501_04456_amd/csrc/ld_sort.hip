// Spatial ordering of the particle slots along a Hilbert curve, so
// that every 64-slot group is spatially compact and the pair kernel can cull
// Lennard-Jones range tests per group pair.  The ordering is a permutation
// of slots only: each slot carries its original index, which keys the
// Brownian noise and orders every output.
//
// Sorting is a 64-bit bitonic network: 2048-key chunks are sorted and merged
// inside LDS, longer strides run as one global compare-exchange pass each.
// Keys whose sort word is a small integer (a cell index) take a stable LSD
// radix sort instead: 8-bit digits, per-workgroup digit counts, a scan of
// each digit's counts over the tiles (one wavefront per digit), and a
// scatter that adds the digits' own prefix and ranks equal digits in slot
// order.
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


// The curve runs over the particles' bounding box clipped to [-clip, clip]
// per axis (particles outside take the edge cells), so a few stray
// particles far outside the droplet cannot coarsen the order of the rest.
__global__ __launch_bounds__(256) void k_curve_keys(const float4* __restrict__ pos, int n,
                                                    int n_pow2, const float* __restrict__ part,
                                                    int nparts, float clip,
                                                    unsigned long long* keys) {
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
    for (int c = 0; c < 3; ++c) {
        lo[c] = fminf(fmaxf(lo[c], -clip), clip);
        hi[c] = fmaxf(fminf(hi[c], clip), -clip);
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

__global__ __launch_bounds__(256) void k_permute_all(
    const unsigned long long* __restrict__ keys, int n, const float4* __restrict__ pos,
    const float4* __restrict__ lo, const int* __restrict__ typ, const int* __restrict__ oid,
    float4* __restrict__ pos2, float4* __restrict__ lo2, int* __restrict__ typ2,
    int* __restrict__ oid2) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int src = (int)(unsigned)keys[s];
    pos2[s] = pos[src];
    lo2[s] = lo[src];
    typ2[s] = typ[src];
    oid2[s] = oid[src];
}

__global__ __launch_bounds__(256) void k_permute1(const unsigned long long* __restrict__ keys,
                                                  int n, const int* __restrict__ a,
                                                  int* __restrict__ b) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) b[s] = a[(int)(unsigned)keys[s]];
}

// ---- radix sort of keys by their high word ---------------------------------

constexpr int kRT = kRadixThreads;         // threads of the histogram and scatter kernels
constexpr int kRRounds = kRadixRounds;     // 256-key rounds per tile
constexpr int kRTile = kRadixTile;         // keys per workgroup tile

// Digit counts of one tile: hist[digit * nwg + tile].
__global__ __launch_bounds__(kRT) void k_radix_hist(const unsigned long long* __restrict__ in,
                                                    int n, int shift, unsigned* hist, int nwg) {
    __shared__ unsigned h[256];
    const int t = threadIdx.x;
    h[t] = 0u;
    // every round's key in flight at once
    unsigned d[kRRounds];
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
        const int e = blockIdx.x * kRTile + r * kRT + t;
        d[r] = e < n ? (unsigned)(in[e] >> (32 + shift)) & 255u : 256u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRRounds; ++r)
        if (d[r] < 256u) atomicAdd(&h[d[r]], 1u);
    __syncthreads();
    hist[(size_t)t * nwg + blockIdx.x] = h[t];
}

// Per-digit exclusive scan of the tile counts, one wavefront per digit:
// hist[d * nwg + b] becomes the count of digit d in tiles before b, and
// hist[256 * nwg + d] the digit's total.  The digits' own prefix is taken
// by each scatter workgroup, so no single-workgroup pass over all counters
// remains.
__global__ __launch_bounds__(256) void k_radix_rows(unsigned* hist, int nwg) {
    const int d = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    unsigned* row = hist + (size_t)d * nwg;
    unsigned carry = 0u;
    for (int b0 = 0; b0 < nwg; b0 += 64) {
        const int b = b0 + lane;
        const unsigned v = b < nwg ? row[b] : 0u;
        unsigned x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (b < nwg) row[b] = carry + x - v;
        carry += __shfl(x, 63);
    }
    if (lane == 0) hist[256 * (size_t)nwg + d] = carry;
}

// Stable scatter of one tile by digit: a key's destination is its digit's
// offset (scanned counts of all earlier tiles and digits) plus the number
// of equal digits before it in the tile -- earlier rounds, earlier
// wavefronts of its round, earlier lanes of its wavefront (matched with
// eight ballots).
__global__ __launch_bounds__(kRT) void k_radix_scatter(const unsigned long long* __restrict__ in,
                                                       unsigned long long* __restrict__ out,
                                                       int n, int shift,
                                                       const unsigned* __restrict__ hist,
                                                       int nwg) {
    __shared__ unsigned base[256];
    __shared__ unsigned wcnt[kRT / 64][256];
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    // digit offset = the totals of all smaller digits (an exclusive scan of
    // the 256 totals) + this digit's count in earlier tiles
    {
        const unsigned tot = hist[256 * (size_t)nwg + t];
        unsigned x = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned y = __shfl_up(x, o);
            if (l >= o) x += y;
        }
        if (l == 63) wcnt[0][w] = x;
        __syncthreads();
        unsigned before = 0u;
        for (int k = 0; k < w; ++k) before += wcnt[0][k];
        base[t] = before + x - tot + hist[(size_t)t * nwg + blockIdx.x];
        __syncthreads();                               // wcnt is cleared below
    }
    const unsigned long long below = (1ull << l) - 1ull;
    // every round's key in flight at once (the rounds below wait on barriers)
    unsigned long long kr[kRRounds];
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
        const int e = blockIdx.x * kRTile + r * kRT + t;
        kr[r] = e < n ? in[e] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
        const int e = blockIdx.x * kRTile + r * kRT + t;
        const bool valid = e < n;
        const unsigned long long key = kr[r];
        const unsigned d = (unsigned)(key >> (32 + shift)) & 255u;
#pragma unroll
        for (int k = 0; k < kRT / 64; ++k) wcnt[k][t] = 0u;
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(valid && bit);
            same &= bit ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(same & below);
        __syncthreads();                               // wcnt cleared, base current
        if (valid && rank == 0u) wcnt[w][d] = (unsigned)__popcll(same);
        __syncthreads();
        if (valid) {
            unsigned pos = base[d] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            out[pos] = key;
        }
        __syncthreads();
        unsigned add = 0u;
#pragma unroll
        for (int k = 0; k < kRT / 64; ++k) add += wcnt[k][t];
        base[t] += add;
    }
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
                       hipStream_t s, float clip) {
    hipLaunchKernelGGL(k_bounds_part, dim3(B.bounds_parts), dim3(256), 0, s, pos, n,
                       B.bounds_part);
    hipLaunchKernelGGL(k_curve_keys, dim3((B.n_pow2 + 255) / 256), dim3(256), 0, s, pos, n, B.n_pow2,
                       B.bounds_part, B.bounds_parts, clip, B.keys);
    return launch_sort_by_keys(pos, lo, typ, oid, n, B, s);
}

hipError_t permute_slots(float4* pos, float4* lo, int* typ, int* oid, int n,
                         const SortBuffers& B, hipStream_t s) {
    hipError_t e;
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

hipError_t launch_sort_by_keys(float4* pos, float4* lo, int* typ, int* oid, int n,
                               const SortBuffers& B, hipStream_t s) {
    const hipError_t e = launch_bitonic(B.keys, B.n_pow2, s);
    if (e != hipSuccess) return e;
    return permute_slots(pos, lo, typ, oid, n, B, s);
}

int radix_tiles(int n) { return (n + kRTile - 1) / kRTile; }

hipError_t launch_radix_by_high(unsigned long long* keys, unsigned long long* tmp, int n, int bits,
                                unsigned* hist, hipStream_t s, bool first_counted,
                                unsigned long long** sorted) {
    if (sorted) *sorted = keys;
    if (n <= 0) return hipSuccess;
    const int nwg = radix_tiles(n);
    unsigned long long* src = keys;
    unsigned long long* dst = tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        if (shift > 0 || !first_counted)
            hipLaunchKernelGGL(k_radix_hist, dim3(nwg), dim3(kRT), 0, s, src, n, shift, hist, nwg);
        hipLaunchKernelGGL(k_radix_rows, dim3(64), dim3(256), 0, s, hist, nwg);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nwg), dim3(kRT), 0, s, src, dst, n, shift, hist,
                           nwg);
        unsigned long long* x = src;
        src = dst;
        dst = x;
    }
    if (sorted) {
        *sorted = src;                 // no copy: the caller reads the sorted keys there
    } else if (src != keys) {
        const hipError_t e = hipMemcpyAsync(keys, src, sizeof(unsigned long long) * n,
                                            hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t permute_slots_into(const unsigned long long* keys, int n, const float4* pos,
                              const float4* lo, const int* typ, const int* oid, float4* pos2,
                              float4* lo2, int* typ2, int* oid2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_all, dim3((n + 255) / 256), dim3(256), 0, s, keys, n, pos, lo,
                       typ, oid, pos2, lo2, typ2, oid2);
    return hipGetLastError();
}

}  // namespace ld
