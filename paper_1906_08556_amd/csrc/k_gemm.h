// FP32 MFMA GEMM launcher shared by the E-step and M-step host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ivx {

enum { GEMM_STORE = 0, GEMM_ADD_F64 = 1, GEMM_STORE_TP = 2 };

struct GemmArgs {
  const float* A = nullptr;
  const float* B = nullptr;
  void* C = nullptr;
  int64_t lda = 0, ldb = 0, ldc = 0;
  int M = 0, N = 0, K = 0;
  int64_t sA = 0, sB = 0, sC = 0;  // per-batch strides (elements)
  int64_t sS = 0;                  // per-split stride of the FP32 store epilogue
  int ksplit = 1;
  int kchunk = 0;                  // K per split (multiple of 16); ignored when ksplit == 1
  int m_fast = 0;                  // set by gemm_f32: M tiles of one column block consecutive
};

// C = op(A) op(B).  ta / tb select the transposed addressing of A / B, epi one
// of GEMM_STORE, GEMM_ADD_F64, GEMM_STORE_TP.  Returns false (and launches
// nothing) for a combination that is not instantiated.
bool gemm_f32(const GemmArgs& g, bool ta, bool tb, int epi, int batches, hipStream_t s);

// C[m][n] = sum_k A[m][k] B[n][k] (FP32 result) on BF16 MFMA from operands
// pre-split into BF16 high and low parts, K-contiguous (hi*hi + hi*lo +
// lo*hi).  K must be a multiple of 8 (rows padded with zeros).
void gemm_bf16x3_nt(const __bf16* Ahi, const __bf16* Alo, int64_t lda, const __bf16* Bhi,
                    const __bf16* Blo, int64_t ldb, float* C, int64_t ldc, int M, int N, int K,
                    hipStream_t s);
// src [rows][cols] FP32 -> BF16 hi / lo [rows][ldo] (zero padding)
void split_bf16(const float* src, int64_t rows, int64_t cols, int64_t ldo, __bf16* hi, __bf16* lo,
                hipStream_t s);
// src [rows][cols] FP32 -> BF16 hi / lo [cols][ldo], transposed (zero padding)
void split_bf16_transposed(const float* src, int64_t rows, int64_t cols, int64_t ldo, __bf16* hi,
                           __bf16* lo, hipStream_t s);

// C[m][n] += sum_k A[k*lda + m] * B[k*ldb + n] with FP64 products and sums
// (k_gemm64.hip).  A is FP32; B is FP64 (b_is_double) or FP32.
void gemm64_tn(const float* A, int64_t lda, const void* B, bool b_is_double, int64_t ldb,
               double* C, int64_t ldc, int M, int N, int K, hipStream_t s);

}  // namespace ivx
