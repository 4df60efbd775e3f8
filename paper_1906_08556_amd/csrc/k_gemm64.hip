// FP64 MFMA GEMM (v_mfma_f64_16x16x4f64) for the M-step accumulators:
//   C[m][n] += sum_k A[k][m] B[k][n]     (A read transposed: A[k*lda + m])
// with A and B stored as float or double and converted to FP64 on load, so
// every product and sum is FP64.  A_c = sum_u n_c(u) Psi(u) has eigenvalues
// spread over ~10 orders of magnitude when a component is seen in fewer than
// R utterances; FP32 products would already perturb its smallest ones.
//
// 64 x 64 output tile per 256-thread workgroup (2 x 2 waves of 32 x 32, each
// 2 x 2 blocks of 16 x 16), K staged 16 at a time through LDS.
#include "ivx_internal.h"
#include "k_gemm.h"

namespace ivx {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int LDW = 64 + 4;

template <typename TAe, typename TBe>
__global__ void __launch_bounds__(256) k_gemm64_tn(const TAe* __restrict__ A, int64_t lda,
                                                   const TBe* __restrict__ B, int64_t ldb,
                                                   double* __restrict__ C, int64_t ldc, int M,
                                                   int N, int K) {
  __shared__ double As[2][BK][LDW];
  __shared__ double Bs[2][BK][LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // loader: thread covers row k = tid / 16 and 4 consecutive columns
  const int lk = tid >> 4, lc = (tid & 15) * 4;
  double ra[4], rb[4];
  auto load = [&](int k0) {
    const int k = k0 + lk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + lc + e, n = n0 + lc + e;
      ra[e] = (k < K && m < M) ? (double)A[(int64_t)k * lda + m] : 0.0;
      rb[e] = (k < K && n < N) ? (double)B[(int64_t)k * ldb + n] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[buf][lk][lc + e] = ra[e];
      Bs[buf][lk][lc + e] = rb[e];
    }
  };
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load((it + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int k = 4 * s + q16;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[cur][k][wm * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[cur][k][wn * 32 + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
  // v_mfma_f64_16x16x4f64 result layout (measured on gfx950): register r of
  // lane l holds row 4*r + l/16, column l%16 -- unlike the FP32 16x16x4 form,
  // whose rows are 4*(l/16) + r.
  // acc[i][j][r] = C[mbase + 4*r + q16][nbase + l16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * r + q16;
        if (m < M && n < N) C[(int64_t)m * ldc + n] += acc[i][j][r];
      }
    }
}

}  // namespace

void gemm64_tn(const float* A, int64_t lda, const void* B, bool b_is_double, int64_t ldb,
               double* C, int64_t ldc, int M, int N, int K, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM));
  if (b_is_double)
    k_gemm64_tn<float, double><<<grid, 256, 0, s>>>(A, lda, static_cast<const double*>(B), ldb, C,
                                                     ldc, M, N, K);
  else
    k_gemm64_tn<float, float><<<grid, 256, 0, s>>>(A, lda, static_cast<const float*>(B), ldb, C,
                                                    ldc, M, N, K);
}

}  // namespace ivx
