// Launchers of the BF16-MFMA matrix products and training helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace ld {

// C[M x N] (= or +=) act(op(A)[M x K] op(B)[K x N] + bias).  op(A) = A
// (row-major, leading dimension lda) or its transpose (A stored K x M);
// likewise B.  Z (optional) receives the pre-activation values.  If M_dev is
// set, rows at or beyond *M_dev are skipped (a device-side row count).
struct GemmArgs {
    const float* A;
    int lda;
    int transA;
    const float* B;
    int ldb;
    int transB;
    float* C;
    int ldc;
    const float* bias;
    float* Z;
    int ldz;
    int M, N, K;
    int act;          // 0 none, 1 SiLU (Z stores the pre-activation), 2 times SiLU'(Z)
    int accumulate;   // 1: C += result
    const int* M_dev;
    // Optional FP32 workspace for split-K: when C has few 64 x 64 tiles and
    // K is long (the weight gradients, K = batch), K is cut into pieces
    // computed by separate workgroups into work[piece][M][N] and summed in
    // piece order by a second kernel.  Unused when NULL or too small.
    float* work;
    size_t work_floats;
    // Optional: the column sums of B (sum over k of B[k][n], FP32, N values;
    // the bias gradient when B is the pre-activation gradient).  B must not
    // be transposed.
    float* colsum_B;
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_mse(const float* Y, int ld, const float* T, int rows, int out, float* dY,
                      double* part, int* nparts, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, int step,
                       hipStream_t s);

}  // namespace ld
