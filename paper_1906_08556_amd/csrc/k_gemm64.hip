// FP64 MFMA GEMM (v_mfma_f64_16x16x4f64) for the M-step accumulators:
//   C[m][n] += sum_k A[k][m] B[k][n]     (A read transposed: A[k*lda + m])
// with A and B stored as float or double and converted to FP64 on load, so
// every product and sum is FP64.  A_c = sum_u n_c(u) Psi(u) has eigenvalues
// spread over ~10 orders of magnitude when a component is seen in fewer than
// R utterances; FP32 products would already perturb its smallest ones.
//
// 64 x 64 output tile per 256-thread workgroup (2 x 2 waves of 32 x 32, each
// 2 x 2 blocks of 16 x 16), K staged 16 at a time through LDS.  The tile
// order streams the larger operand once: with m_fast, consecutive workgroups
// share a column block of B (read once from HBM, then from the shared
// last-level cache by the other M tiles); otherwise they share a row block
// of A.
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
                                                   int N, int K, int m_fast) {
  __shared__ double As[2][BK][LDW];
  __shared__ double Bs[2][BK][LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int m0 = (m_fast ? blockIdx.x : blockIdx.y) * BM;
  const int n0 = (m_fast ? blockIdx.y : blockIdx.x) * BN;
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

// 128 x 32 NJ tile for the large accumulator products: 4 waves of
// 64 x 16 NJ (4 x NJ blocks of 16 x 16), K staged 8 at a time, A loaded as
// float4 and B as double2 / float4 (requires M a multiple of 128, N and the
// leading dimensions multiples of 4, 16-byte aligned bases; columns beyond N
// are zero-filled and not stored).  LDS rows are padded by 16 doubles so that
// the two 16-lane halves of a wave reading adjacent rows fall into opposite
// halves of the banks.  m_fast: the M tiles of one B column block are
// consecutive (B streamed once); otherwise the N tiles of one A row block.
constexpr int GT = 128, TK = 8, TLD = 144;

// four consecutive elements as FP64 (16-byte vector loads)
__device__ inline void load4(const double* p, double& a, double& b, double& c, double& d) {
  const double2 u = *reinterpret_cast<const double2*>(p);
  const double2 v = *reinterpret_cast<const double2*>(p + 2);
  a = u.x;
  b = u.y;
  c = v.x;
  d = v.y;
}
__device__ inline void load4(const float* p, double& a, double& b, double& c, double& d) {
  const float4 u = *reinterpret_cast<const float4*>(p);
  a = u.x;
  b = u.y;
  c = u.z;
  d = u.w;
}

// NJ: 16-column blocks per wave (4: 128 x 128 tile, 2: 128 x 64 tile)
template <int NJ, typename TBe>
__global__ void __launch_bounds__(256, 4) k_gemm64_tn_128(const float* __restrict__ A, int64_t lda,
                                                       const TBe* __restrict__ B, int64_t ldb,
                                                       double* __restrict__ C, int64_t ldc,
                                                       int N, int K, int m_fast) {
  constexpr int BNT = 32 * NJ;           // tile columns
  constexpr int BLD = BNT + 16;          // padded B row
  __shared__ double As[2][TK][TLD];
  __shared__ double Bs[2][TK][BLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int64_t m0 = (int64_t)(m_fast ? blockIdx.x : blockIdx.y) * GT;
  const int64_t n0 = (int64_t)(m_fast ? blockIdx.y : blockIdx.x) * BNT;
  const int lk = tid >> 5, lc = (tid & 31) * 4;  // A loader: row lk, columns lc..lc+3
  // B loader: NJ = 4 as A; NJ = 2: row tid / 16, columns (tid % 16) * 4
  const int bk = NJ == 4 ? lk : (tid >> 4), bc = NJ == 4 ? lc : (tid & 15) * 4;
  const bool bload = (NJ == 4 || tid < 128) && n0 + bc < N;
  const float* ap = A + m0 + lc;
  const TBe* bp = B + n0 + bc;
  float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
  double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
#define G64_LOAD(k0)                                                              \
  do {                                                                            \
    const int k_ = (k0) + lk;                                                     \
    if (k_ < K) {                                                                 \
      const float4 a4 = *reinterpret_cast<const float4*>(ap + (int64_t)k_ * lda); \
      ax = a4.x; ay = a4.y; az = a4.z; aw = a4.w;                                 \
    } else {                                                                      \
      ax = ay = az = aw = 0.f;                                                    \
    }                                                                             \
    const int kb_ = (k0) + bk;                                                    \
    if (bload && kb_ < K) {                                                       \
      load4(bp + (int64_t)kb_ * ldb, b0, b1, b2, b3);                             \
    } else {                                                                      \
      b0 = b1 = b2 = b3 = 0.0;                                                    \
    }                                                                             \
  } while (0)
#define G64_STORE(buf)                                                            \
  do {                                                                            \
    double* a_ = &As[buf][lk][lc];                                                \
    a_[0] = (double)ax; a_[1] = (double)ay; a_[2] = (double)az; a_[3] = (double)aw; \
    if ((NJ == 4 || tid < 128)) {                                                 \
      double* b_ = &Bs[buf][bk][bc];                                              \
      b_[0] = b0; b_[1] = b1; b_[2] = b2; b_[3] = b3;                             \
    }                                                                             \
  } while (0)
  doublex4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int nk = (K + TK - 1) / TK;
  if (nk > 0) {
    G64_LOAD(0);
    G64_STORE(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) G64_LOAD((it + 1) * TK);
#pragma unroll
    for (int s = 0; s < TK / 4; ++s) {
      const int k = 4 * s + q16;
      double av[4], bv[NJ];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[cur][k][wm * 64 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bv[j] = Bs[cur][k][wn * 16 * NJ + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) G64_STORE(cur ^ 1);
    __syncthreads();
  }
#undef G64_LOAD
#undef G64_STORE
  // acc[i][j][r] = C[mbase + 4*r + q16][nbase + l16] (layout as above)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int64_t n = n0 + wn * 16 * NJ + j * 16 + l16;
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 64 + i * 16 + 4 * r + q16;
        C[m * ldc + n] += acc[i][j][r];
      }
    }
}

}  // namespace

void gemm64_tn(const float* A, int64_t lda, const void* B, bool b_is_double, int64_t ldb,
               double* C, int64_t ldc, int M, int N, int K, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  // stream the larger operand once (B bytes vs A bytes over K)
  const double a_bytes = (double)M * 4.0, b_bytes = (double)N * (b_is_double ? 8.0 : 4.0);
  if (M % GT == 0 && N % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
      reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0) {
    const unsigned mt = (unsigned)(M / GT), nt = (unsigned)((N + 63) / 64);
    const int m_fast = (b_bytes > a_bytes && nt <= 65535u) ? 1 : 0;
    if (m_fast || mt <= 65535u) {
      const dim3 grid = m_fast ? dim3(mt, nt) : dim3(nt, mt);
      if (b_is_double)
        k_gemm64_tn_128<2, double><<<grid, 256, 0, s>>>(A, lda, static_cast<const double*>(B),
                                                         ldb, C, ldc, N, K, m_fast);
      else
        k_gemm64_tn_128<2, float><<<grid, 256, 0, s>>>(A, lda, static_cast<const float*>(B),
                                                        ldb, C, ldc, N, K, m_fast);
      return;
    }
  }
  const unsigned mt = (unsigned)((M + BM - 1) / BM), nt = (unsigned)((N + BN - 1) / BN);
  const int m_fast = (b_bytes > a_bytes && nt <= 65535u) ? 1 : 0;
  const dim3 grid = m_fast ? dim3(mt, nt) : dim3(nt, mt);
  if (b_is_double)
    k_gemm64_tn<float, double><<<grid, 256, 0, s>>>(A, lda, static_cast<const double*>(B), ldb, C,
                                                     ldc, M, N, K, m_fast);
  else
    k_gemm64_tn<float, float><<<grid, 256, 0, s>>>(A, lda, static_cast<const float*>(B), ldb, C,
                                                    ldc, M, N, K, m_fast);
}

}  // namespace ivx
