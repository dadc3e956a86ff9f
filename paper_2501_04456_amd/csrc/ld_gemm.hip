// Dense matrix products of the learned far field on the matrix cores:
// C = op(A) op(B) (+ bias) (-> SiLU) with BF16 operands and FP32
// accumulation (v_mfma_f32_16x16x32_bf16), plus the elementwise pieces of
// training (SiLU derivative, bias gradients, mean-squared loss, Adam).
//
// Tiling: a workgroup of 4 wavefronts owns a 64 x 64 tile of C; each
// wavefront owns 16 rows x 64 columns (four 16 x 16 MFMA tiles).  K advances
// 32 at a time through LDS: the A tile is staged row-major [64][32], the B
// tile column-major [64][32], so every MFMA operand (8 consecutive K values of
// one row / column) is one 16-byte LDS read.  Operands are rounded from FP32
// to BF16 (nearest even) as they are staged; transposed operands are read
// with the transpose folded into the global index.
//
// MFMA 16x16x32 operand layout (wave64): lane l supplies A[l % 16][8 (l/16)
// + 0..7] and B[8 (l/16) + 0..7][l % 16]; it receives C[4 (l/16) + 0..3][l % 16].
#include <algorithm>

#include "ld_internal.h"
#include "ld_gemm.h"

namespace ld {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, PAD = 8;

__device__ __forceinline__ __bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

// SiLU as in the fused kernel: hardware exponential and reciprocal.
__device__ __forceinline__ float silu(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// part == nullptr: the whole K range and the epilogue (bias, pre-activation,
// SiLU, accumulate).  Otherwise piece blockIdx.z of the K range, [kb, ke),
// raw sums into part[blockIdx.z][M][N].
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g, int kpiece, float* part) {
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[BN][BK + PAD];
    const int M = g.M_dev ? min(g.M, *g.M_dev) : g.M;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= M) return;
    const int kb = part ? (int)blockIdx.z * kpiece : 0;
    const int ke = part ? min(g.K, kb + kpiece) : g.K;
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    f32x4 acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < (BM * BK) / 256; ++r) {
            const int e = t + 256 * r;
            int row, kk;
            if (g.transA) { row = e % BM; kk = e / BM; }
            else { row = e / BK; kk = e % BK; }
            const int gr = m0 + row, gk = k0 + kk;
            float v = 0.f;
            if (gr < M && gk < ke)
                v = g.transA ? g.A[(size_t)gk * g.lda + gr] : g.A[(size_t)gr * g.lda + gk];
            As[row][kk] = to_bf16(v);
        }
#pragma unroll
        for (int r = 0; r < (BN * BK) / 256; ++r) {
            const int e = t + 256 * r;
            int col, kk;
            if (g.transB) { kk = e % BK; col = e / BK; }
            else { col = e % BN; kk = e / BN; }
            const int gc = n0 + col, gk = k0 + kk;
            float v = 0.f;
            if (gc < g.N && gk < ke)
                v = g.transB ? g.B[(size_t)gc * g.ldb + gk] : g.B[(size_t)gk * g.ldb + gc];
            Bt[col][kk] = to_bf16(v);
        }
        __syncthreads();
        const int kk = 8 * (l / 16);
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[w * 16 + l % 16][kk]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bt[j * 16 + l % 16][kk]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
    }
    if (part) {
        float* P = part + (size_t)blockIdx.z * (size_t)g.M * g.N;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + j * 16 + l % 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + w * 16 + 4 * (l / 16) + r;
                if (row < M && col < g.N) P[(size_t)row * g.N + col] = acc[j][r];
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + j * 16 + l % 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + w * 16 + 4 * (l / 16) + r;
            if (row >= M || col >= g.N) continue;
            float v = acc[j][r];
            if (g.bias) v += g.bias[col];
            if (g.Z) g.Z[(size_t)row * g.ldz + col] = v;
            if (g.act == 1) v = silu(v);
            float* c = g.C + (size_t)row * g.ldc + col;
            *c = g.accumulate ? *c + v : v;
        }
    }
}

// Split-K epilogue: the pieces summed in order, then as k_gemm's epilogue.
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int pieces,
                                                     const float* __restrict__ part) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t mn = (size_t)g.M * g.N;
    if (e >= mn) return;
    const int row = (int)(e / g.N), col = (int)(e % g.N);
    float v = 0.f;
    for (int z = 0; z < pieces; ++z) v += part[(size_t)z * mn + e];
    if (g.bias) v += g.bias[col];
    if (g.Z) g.Z[(size_t)row * g.ldz + col] = v;
    if (g.act == 1) v = silu(v);
    float* c = g.C + (size_t)row * g.ldc + col;
    *c = g.accumulate ? *c + v : v;
}

// dZ = dA * silu'(Z), elementwise over rows x cols (row strides ld).
__global__ __launch_bounds__(256) void k_silu_bwd(const float* __restrict__ Z, float* dA, int rows,
                                                  int cols, const int* rows_dev) {
    const int R = rows_dev ? min(rows, *rows_dev) : rows;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)R * cols) return;
    const float z = Z[e];
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    dA[e] *= s * (1.0f + z * (1.0f - s));
}

// db[c] = sum_r dZ[r][c] (one workgroup per column, fixed order).
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ dZ, int rows, int cols,
                                                float* db) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) acc += dZ[(size_t)r * cols + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

// Mean-squared loss over rows x out (only the first `out` of `ld` columns)
// and its gradient dY = 2 (y - t) / (rows out); per-workgroup partial sums.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, int ld,
                                             const float* __restrict__ T, int rows, int out,
                                             float* dY, double* part) {
    __shared__ double red[256];
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    double sq = 0.0;
    if (e < (size_t)rows * ld) {
        const size_t r = e / ld;
        const int c = (int)(e % ld);
        float d = 0.f;
        if (c < out) {
            const float diff = Y[e] - T[r * out + c];
            sq = (double)diff * diff;
            d = 2.0f * diff / (float)(rows * out);
        }
        dY[e] = d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] / ((double)rows * out);
}

__global__ __launch_bounds__(256) void k_adam(float* w, const float* __restrict__ g, float* m,
                                              float* v, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN);
    const int tiles = (int)(grid.x * grid.y);
    // split K when C has too few tiles to fill the chip and K is long: pieces
    // of at least 4 BK steps, about 1024 workgroups in all
    int pieces = 1;
    if (g.work && !g.M_dev && tiles < 256 && g.K >= 8 * BK) {
        pieces = std::min(std::max(1, 1024 / tiles), g.K / (4 * BK));
        const size_t mn = (size_t)g.M * g.N;
        pieces = (int)std::min<size_t>((size_t)pieces, g.work_floats / std::max<size_t>(mn, 1));
    }
    if (pieces <= 1) {
        hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g, 0, (float*)nullptr);
        return hipGetLastError();
    }
    const int kpiece = ((g.K + pieces - 1) / pieces + BK - 1) / BK * BK;
    pieces = (g.K + kpiece - 1) / kpiece;
    grid.z = pieces;
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g, kpiece, g.work);
    const size_t mn = (size_t)g.M * g.N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g,
                       pieces, (const float*)g.work);
    return hipGetLastError();
}

hipError_t launch_silu_bwd(const float* Z, float* dA, int rows, int cols, const int* rows_dev,
                           hipStream_t s) {
    const size_t n = (size_t)rows * cols;
    hipLaunchKernelGGL(k_silu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, dA,
                       rows, cols, rows_dev);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, int rows, int cols, float* db, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, s, dZ, rows, cols, db);
    return hipGetLastError();
}

hipError_t launch_mse(const float* Y, int ld, const float* T, int rows, int out, float* dY,
                      double* part, int* nparts, hipStream_t s) {
    const size_t n = (size_t)rows * ld;
    const int blocks = (int)((n + 255) / 256);
    *nparts = blocks;
    hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, s, Y, ld, T, rows, out, dY, part);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, int step,
                       hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace ld
