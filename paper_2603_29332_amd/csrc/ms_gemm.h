// ms_gemm.h -- bfloat16 matrix-core GEMM with fused epilogues (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace ms {

typedef __hip_bfloat16 bf16;

// C[M][N] = A B^T with A [M][K] (row stride lda) and B [N][K] (row stride
// ldb): C(m, n) = sum_k A[m * lda + k] B[n * ldb + k]. bfloat16 operands,
// float32 accumulation. Epilogue, per element (m, n):
//   v = acc * alpha + (bias ? bias[n] : 0) + (addc ? addc[m * ldc + n] : 0)
//   if dact: v *= SiLU'(dact[m * ldc + n])           (backward through SiLU)
//   if z_out: z_out[m * ldc + n] = v                  (pre-activation, f32)
//   if act == 1: v = SiLU(v);  if act == 2: v = sigmoid(v)
//   if scale: v = v * scale[n] + shift[n]             (de-standardisation)
//   if c_f32: c_f32[m * ldc + n] = v ;  if c_bf16: c_bf16[m * ldc + n] = bf16(v)
//   if c2 and n >= split: c2[m * ldc2 + n - split] = v instead of c_f32 (the
//   columns from `split` on go to a second matrix)
struct GemmEpi {
  const float *bias = nullptr;
  const float *addc = nullptr;
  const float *dact = nullptr;
  float *z_out = nullptr;
  int act = 0;
  const float *scale = nullptr, *shift = nullptr;
  float *c_f32 = nullptr;
  bf16 *c_bf16 = nullptr;
  int ldc = 0;
  float alpha = 1.0f;
  float *c2 = nullptr;
  int split = 0, ldc2 = 0;
};

// C[M][N] (float32, ldc) = A B^T with K split into slices computed by
// separate workgroups into work[S][M][ldc] and summed in slice order
// (deterministic). work must hold S M ldc floats; S = splitk_slices(M, N, K).
int splitk_slices(int M, int N, int K);
hipError_t gemm_bf16_splitk(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                            float *C, int ldc, float *work, hipStream_t st);

// XT[c][r] = X[r][c] for bfloat16 X[rows][cols]; rows and cols multiples
// of 4.
hipError_t transpose_bf16(const bf16 *X, int rows, int cols, bf16 *XT, hipStream_t st);

// Requires K, lda, ldb multiples of 8 (16-byte rows) and lda, ldb at most
// 2^20. Returns the launch error, if any.
hipError_t gemm_bf16(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                     const GemmEpi &epi, hipStream_t st);

}  // namespace ms
