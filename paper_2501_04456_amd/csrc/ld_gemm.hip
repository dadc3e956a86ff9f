// Dense matrix products of the learned far field on the matrix cores:
// C = op(A) op(B) (+ bias) (-> SiLU, or times SiLU' of a stored
// pre-activation) with BF16 operands and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), optionally with the column sums of B (the bias
// gradients of training), plus the mean-squared loss and Adam.
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
//
// k_gemm_v is the same tiling for operands whose rows are 16-byte aligned
// (every product of the far-field network): K advances 64 at a time, each
// work-item fetches its share of an A and a B tile as four 16-byte loads
// each, two stages ahead of the matrix cores (a ring of two register sets),
// and the tiles are written to LDS as BF16, transposed on the way where K is
// the operand's strided index.  k_gemm is the general
// fallback (any alignment).
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

// The product's epilogue: bias, then act 1 (store the pre-activation in Z if
// given, apply SiLU) or act 2 (multiply by SiLU'(z) for the stored
// pre-activation z = Z[row][col], the backward pass through the activation).
__device__ __forceinline__ float epilogue(const GemmArgs& g, int row, int col, float v) {
    if (g.bias) v += g.bias[col];
    if (g.act == 2) {
        const float z = g.Z[(size_t)row * g.ldz + col];
        const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
        return v * (sg * (1.0f + z * (1.0f - sg)));
    }
    if (g.Z) g.Z[(size_t)row * g.ldz + col] = v;
    return g.act == 1 ? silu(v) : v;
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
            const float v = epilogue(g, row, col, acc[j][r]);
            float* c = g.C + (size_t)row * g.ldc + col;
            *c = g.accumulate ? *c + v : v;
        }
    }
}

constexpr int VK = 64;                 // K per stage of k_gemm_v

// Pack two floats as adjacent BF16 values (the first at the lower address).
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    return (uint32_t)__builtin_bit_cast(unsigned short, to_bf16(lo)) |
           ((uint32_t)__builtin_bit_cast(unsigned short, to_bf16(hi)) << 16);
}

// One operand tile, 64 rows (rows of A or columns of B) x VK values of k,
// fetched into registers and stored to LDS as S[row][k] in BF16.  KC: k is
// the contiguous index in memory (element (r, k) at P[r ld + k]); otherwise
// rows are (element (r, k) at P[k ld + r]).  Elements outside [0, rlim) x
// [0, klim) read as zero.
template <bool KC>
struct Tile {
    float4 v[4];

    __device__ __forceinline__ void load(const float* __restrict__ P, int ld, int r0, int rlim,
                                         int k0, int klim, int t) {
        if constexpr (KC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = t + 256 * q;
                const int r = r0 + idx / 16, k = k0 + (idx % 16) * 4;
                const float* src = P + (size_t)r * ld + k;
                if (r < rlim && k + 3 < klim) {
                    v[q] = *reinterpret_cast<const float4*>(src);
                } else {
                    const bool rr = r < rlim;
                    v[q].x = rr && k < klim ? src[0] : 0.f;
                    v[q].y = rr && k + 1 < klim ? src[1] : 0.f;
                    v[q].z = rr && k + 2 < klim ? src[2] : 0.f;
                    v[q].w = rr && k + 3 < klim ? src[3] : 0.f;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int idx = t + 256 * q;
                const int r = r0 + (idx % 16) * 4;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = k0 + 2 * (idx / 16) + h;
                    const float* src = P + (size_t)k * ld + r;
                    float4& d = v[2 * q + h];
                    if (k < klim && r + 3 < rlim) {
                        d = *reinterpret_cast<const float4*>(src);
                    } else {
                        const bool kk = k < klim;
                        d.x = kk && r < rlim ? src[0] : 0.f;
                        d.y = kk && r + 1 < rlim ? src[1] : 0.f;
                        d.z = kk && r + 2 < rlim ? src[2] : 0.f;
                        d.w = kk && r + 3 < rlim ? src[3] : 0.f;
                    }
                }
            }
        }
    }

    __device__ __forceinline__ void store(__bf16 (*S)[VK + PAD], int t) const {
        if constexpr (KC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = t + 256 * q;
                uint2 w;
                w.x = pack2(v[q].x, v[q].y);
                w.y = pack2(v[q].z, v[q].w);
                *reinterpret_cast<uint2*>(&S[idx / 16][(idx % 16) * 4]) = w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int idx = t + 256 * q;
                const int r = (idx % 16) * 4, k = 2 * (idx / 16);
                const float4 a = v[2 * q], b = v[2 * q + 1];
                *reinterpret_cast<uint32_t*>(&S[r][k]) = pack2(a.x, b.x);
                *reinterpret_cast<uint32_t*>(&S[r + 1][k]) = pack2(a.y, b.y);
                *reinterpret_cast<uint32_t*>(&S[r + 2][k]) = pack2(a.z, b.z);
                *reinterpret_cast<uint32_t*>(&S[r + 3][k]) = pack2(a.w, b.w);
            }
        }
    }
};

// As k_gemm (same arguments, epilogue and split-K pieces), for 16-byte
// aligned operands with leading dimensions divisible by 4.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_v(GemmArgs g, int kpiece, float* part) {
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][VK + PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[BN][VK + PAD];
    const int M = g.M_dev ? min(g.M, *g.M_dev) : g.M;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= M) return;
    const int kb = part ? (int)blockIdx.z * kpiece : 0;
    const int ke = part ? min(g.K, kb + kpiece) : g.K;
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    f32x4 acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // two tiles in flight: while the matrix cores work on stage k, the loads
    // of stages k + 1 and k + 2 are outstanding (a ring of two register sets)
    Tile<!TA> ta[2];       // A is k-contiguous unless transposed
    Tile<TB> tb[2];        // B (K x N) is k-contiguous only when transposed
    ta[0].load(g.A, g.lda, m0, M, kb, ke, t);
    tb[0].load(g.B, g.ldb, n0, g.N, kb, ke, t);
    if (kb + VK < ke) {
        ta[1].load(g.A, g.lda, m0, M, kb + VK, ke, t);
        tb[1].load(g.B, g.ldb, n0, g.N, kb + VK, ke, t);
    }
    // column sums of B (FP32, before rounding): the first row of tiles only;
    // this work-item's values all lie in columns n0 + 4 (t % 16) + 0..3
    const bool csum = !TB && g.colsum_B && blockIdx.x == 0;
    float4 cs = make_float4(0.f, 0.f, 0.f, 0.f);
    const int kk = 8 * (l / 16);
    for (int k0 = kb; k0 < ke; k0 += 2 * VK) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ks0 = k0 + r * VK;
            if (ks0 >= ke) break;
            __syncthreads();
            ta[r].store(As, t);
            tb[r].store(Bt, t);
            if (csum) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    cs.x += tb[r].v[q].x;
                    cs.y += tb[r].v[q].y;
                    cs.z += tb[r].v[q].z;
                    cs.w += tb[r].v[q].w;
                }
            }
            __syncthreads();
            if (ks0 + 2 * VK < ke) {         // refill this set two stages ahead
                ta[r].load(g.A, g.lda, m0, M, ks0 + 2 * VK, ke, t);
                tb[r].load(g.B, g.ldb, n0, g.N, ks0 + 2 * VK, ke, t);
            }
#pragma unroll
            for (int ks = 0; ks < VK; ks += 32) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[w * 16 + l % 16][ks + kk]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bf16x8 b =
                        *reinterpret_cast<const bf16x8*>(&Bt[j * 16 + l % 16][ks + kk]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
                }
            }
        }
    }
    if (csum) {
        // the 16 work-items of each column quad, added in a fixed order; the
        // result goes after the pieces' products (split K) or to colsum_B
        float* red = reinterpret_cast<float*>(&As[0][0]);     // 16 x 64 floats
        __syncthreads();
        *reinterpret_cast<float4*>(&red[(t / 16) * 64 + (t % 16) * 4]) = cs;
        __syncthreads();
        if (t < 64 && n0 + t < g.N) {
            float v = 0.f;
            for (int r = 0; r < 16; ++r) v += red[r * 64 + t];
            if (part)
                part[(size_t)gridDim.z * g.M * g.N + (size_t)blockIdx.z * g.N + n0 + t] = v;
            else
                g.colsum_B[n0 + t] = v;
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
            const float v = epilogue(g, row, col, acc[j][r]);
            float* c = g.C + (size_t)row * g.ldc + col;
            *c = g.accumulate ? *c + v : v;
        }
    }
}

// A 32-row A tile, k contiguous (A untransposed): two 16-byte loads per
// work-item per 64-deep stage.
struct TileA32 {
    float4 v[2];

    __device__ __forceinline__ void load(const float* __restrict__ P, int ld, int r0, int rlim,
                                         int k0, int klim, int t) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = t + 256 * q;
            const int r = r0 + idx / 16, k = k0 + (idx % 16) * 4;
            const float* src = P + (size_t)r * ld + k;
            if (r < rlim && k + 3 < klim) {
                v[q] = *reinterpret_cast<const float4*>(src);
            } else {
                const bool rr = r < rlim;
                v[q].x = rr && k < klim ? src[0] : 0.f;
                v[q].y = rr && k + 1 < klim ? src[1] : 0.f;
                v[q].z = rr && k + 2 < klim ? src[2] : 0.f;
                v[q].w = rr && k + 3 < klim ? src[3] : 0.f;
            }
        }
    }

    __device__ __forceinline__ void store(__bf16 (*S)[VK + PAD], int t) const {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = t + 256 * q;
            uint2 w;
            w.x = pack2(v[q].x, v[q].y);
            w.y = pack2(v[q].z, v[q].w);
            *reinterpret_cast<uint2*>(&S[idx / 16][(idx % 16) * 4]) = w;
        }
    }
};

// As k_gemm_v (untransposed A, no split K), with 32 x 64 output tiles: twice
// the workgroups of the 64 x 64 tiling for the tall products (M = batch),
// which otherwise run one wavefront per SIMD.  Wavefront w owns rows
// 16 (w % 2) .. + 15 and columns 32 (w / 2) .. + 31 (two MFMA tiles).
template <bool TB>
__global__ __launch_bounds__(256) void k_gemm_v32(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[32][VK + PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[BN][VK + PAD];
    const int M = g.M_dev ? min(g.M, *g.M_dev) : g.M;
    const int m0 = blockIdx.x * 32, n0 = blockIdx.y * BN;
    if (m0 >= M) return;
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    const int wr = (w & 1) * 16, wc = (w >> 1) * 32;
    f32x4 acc[2];
    for (int j = 0; j < 2; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    TileA32 ta[2];
    Tile<TB> tb[2];
    ta[0].load(g.A, g.lda, m0, M, 0, g.K, t);
    tb[0].load(g.B, g.ldb, n0, g.N, 0, g.K, t);
    if (VK < g.K) {
        ta[1].load(g.A, g.lda, m0, M, VK, g.K, t);
        tb[1].load(g.B, g.ldb, n0, g.N, VK, g.K, t);
    }
    const int kk = 8 * (l / 16);
    for (int k0 = 0; k0 < g.K; k0 += 2 * VK) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ks0 = k0 + r * VK;
            if (ks0 >= g.K) break;
            __syncthreads();
            ta[r].store(As, t);
            tb[r].store(Bt, t);
            __syncthreads();
            if (ks0 + 2 * VK < g.K) {
                ta[r].load(g.A, g.lda, m0, M, ks0 + 2 * VK, g.K, t);
                tb[r].load(g.B, g.ldb, n0, g.N, ks0 + 2 * VK, g.K, t);
            }
#pragma unroll
            for (int ks = 0; ks < VK; ks += 32) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wr + l % 16][ks + kk]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 b =
                        *reinterpret_cast<const bf16x8*>(&Bt[wc + j * 16 + l % 16][ks + kk]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = n0 + wc + j * 16 + l % 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + wr + 4 * (l / 16) + r;
            if (row >= M || col >= g.N) continue;
            const float v = epilogue(g, row, col, acc[j][r]);
            float* c = g.C + (size_t)row * g.ldc + col;
            *c = g.accumulate ? *c + v : v;
        }
    }
}

// Split-K epilogue.  A workgroup owns 32 outputs; its eight groups of 32
// work-items each add one eighth of the pieces (all of their loads in flight
// at once), and the eight group sums are added in group order: a fixed
// summation order, whatever the timing.  Outputs mn .. mn + N - 1 are the
// column sums of B (the pieces' column sums follow their products in part).
constexpr int kRedOut = 32, kRedGroups = 8;

__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int pieces,
                                                     const float* __restrict__ part) {
    __shared__ float red[kRedGroups][kRedOut];
    const int el = threadIdx.x % kRedOut, grp = threadIdx.x / kRedOut;
    const size_t e = (size_t)blockIdx.x * kRedOut + el;
    const size_t mn = (size_t)g.M * g.N;
    const size_t outs = mn + (g.colsum_B ? (size_t)g.N : 0);
    const bool live = e < outs;
    // piece z of output e sits at src[z * stride]
    const float* src = e < mn ? part + e : part + (size_t)pieces * mn + (e - mn);
    const size_t stride = e < mn ? mn : (size_t)g.N;
    const int per = (pieces + kRedGroups - 1) / kRedGroups;
    const int z0 = grp * per, z1 = min(pieces, z0 + per);
    float v = 0.f;
    if (live) {
        int z = z0;
        for (; z + 8 <= z1; z += 8) {
            float p[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) p[u] = src[(size_t)(z + u) * stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) v += p[u];
        }
        for (; z < z1; ++z) v += src[(size_t)z * stride];
    }
    red[grp][el] = v;
    __syncthreads();
    if (grp != 0 || !live) return;
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kRedGroups; ++q) t += red[q][el];
    if (e >= mn) {
        g.colsum_B[e - mn] = t;
        return;
    }
    const int row = (int)(e / g.N), col = (int)(e % g.N);
    t = epilogue(g, row, col, t);
    float* c = g.C + (size_t)row * g.ldc + col;
    *c = g.accumulate ? *c + t : t;
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

namespace {
bool aligned16(const float* p, int ld) {
    return ((uintptr_t)p & 15u) == 0 && ld % 4 == 0;
}

bool vector_path(const GemmArgs& g) { return aligned16(g.A, g.lda) && aligned16(g.B, g.ldb); }

void launch_tile_kernel(const GemmArgs& g, dim3 grid, int kpiece, float* part, hipStream_t s) {
    if (!vector_path(g)) {
        hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g, kpiece, part);
        return;
    }
    if (g.transA) {
        if (g.transB) hipLaunchKernelGGL((k_gemm_v<true, true>), grid, dim3(256), 0, s, g, kpiece, part);
        else hipLaunchKernelGGL((k_gemm_v<true, false>), grid, dim3(256), 0, s, g, kpiece, part);
    } else {
        if (g.transB) hipLaunchKernelGGL((k_gemm_v<false, true>), grid, dim3(256), 0, s, g, kpiece, part);
        else hipLaunchKernelGGL((k_gemm_v<false, false>), grid, dim3(256), 0, s, g, kpiece, part);
    }
}
}  // namespace

hipError_t launch_gemm(const GemmArgs& g0, hipStream_t s) {
    GemmArgs g = g0;
    // column sums of B inside the tile kernel only on its vector path with B
    // untransposed; otherwise by the column-sum kernel afterwards
    const bool side_colsum = g.colsum_B && (g.transB || !vector_path(g));
    if (side_colsum) g.colsum_B = nullptr;
    dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN);
    const int tiles = (int)(grid.x * grid.y);
    const size_t mn = (size_t)g.M * g.N;
    const size_t per_piece = mn + (g.colsum_B ? (size_t)g.N : 0);
    // split K when C has too few tiles to fill the chip and K is long: pieces
    // of at least two 64-deep stages, about 512 workgroups in all
    int pieces = 1;
    if (g.work && !g.M_dev && tiles < 256 && g.K >= 4 * VK) {
        pieces = std::min(std::max(1, 512 / tiles), g.K / (2 * VK));
        pieces = (int)std::min<size_t>((size_t)pieces, g.work_floats / std::max<size_t>(per_piece, 1));
    }
    if (pieces <= 1) {
        if (!g.transA && !g.colsum_B && tiles <= 256 && vector_path(g)) {
            // tall products: 32-row tiles, twice the workgroups
            const dim3 g32((g.M + 31) / 32, (g.N + BN - 1) / BN);
            if (g.transB) hipLaunchKernelGGL(k_gemm_v32<true>, g32, dim3(256), 0, s, g);
            else hipLaunchKernelGGL(k_gemm_v32<false>, g32, dim3(256), 0, s, g);
        } else {
            launch_tile_kernel(g, grid, 0, nullptr, s);
        }
    } else {
        const int kpiece = ((g.K + pieces - 1) / pieces + VK - 1) / VK * VK;
        pieces = (g.K + kpiece - 1) / kpiece;
        grid.z = pieces;
        launch_tile_kernel(g, grid, kpiece, g.work, s);
        const size_t outs = mn + (g.colsum_B ? (size_t)g.N : 0);
        hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((outs + kRedOut - 1) / kRedOut)),
                           dim3(kRedOut * kRedGroups), 0, s, g, pieces, (const float*)g.work);
    }
    if (side_colsum) {
        if (g.transB || g.ldb != g.N)    // the column-sum kernel reads packed rows
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_colsum, dim3(g.N), dim3(256), 0, s, g.B, g.K, g.N, g0.colsum_B);
    }
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
