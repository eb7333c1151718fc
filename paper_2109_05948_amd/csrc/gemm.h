// The library's BF16 x BF16 -> FP32 MFMA product (gemm.hip), used by the
// colour-invariant network (invnet.hip) and by the C-ABI entry
// dlm_gemm_bf16.
#pragma once

#include "dlm_common.h"

namespace dlm {

// BF16 x BF16 -> FP32 MFMA product on stream s (gemm.hip):
// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sa + k] if a_kcontig else
// A[k sa + m], B(k, n) = B[n sb + k] if b_kcontig else B[k sb + n];
// tile / splits 0 pick the workgroup tile and the K split from the shape; a
// split writes its partials to ws (splits M N floats).
struct GemmPlan {
  int tile, splits;
};
// Evaluation-mode layer epilogue of the colour-invariant network (Section
// 2.3, normalisation from the running estimates): instead of C, write
//   x[m][n] = BF16(LReLU_slope((C[m][n] + u[m / k][n] + beta[n] - mean[n])
//                               * gamma[n] / sqrt(var[n] + eps) + mu[n]))
// (computed as C sc + off, sc = gamma / sqrt(var + eps) per column)
// (x and u with pitch N); needs both operands K-contiguous, no K split and
// k >= 32 (a 32-row group of C then spans at most two colourings).
struct GemmEval {
  const float *u, *beta, *mean, *var, *gamma, *mu;
  int k;
  float slope, eps;
  uint16_t* x;
};
GemmPlan gemm_plan(int M, int N, int K, int vec, int64_t ws_bytes, int tile, int splits);
int gemm_bf16(bool a_kcontig, const uint16_t* A, int64_t sa, bool b_kcontig, const uint16_t* B, int64_t sb, float* C,
              int64_t ldc, int M, int N, int K, int tile, int splits, void* ws, int64_t ws_bytes, hipStream_t s,
              const GemmEval* eval = nullptr);
// workspace a product of this shape can use (its split partials), in bytes
int64_t gemm_workspace_bytes(int M, int N, int K);

}  // namespace dlm
