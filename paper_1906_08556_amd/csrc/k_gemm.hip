// Dense FP32 GEMM on MFMA (v_mfma_f32_32x32x2_f32) for the E-step and M-step
// contractions: C = op(A) op(B), M x N x K.
//
//  * 128 x 128 output tile per 256-thread workgroup, 2 x 2 waves of 64 x 64
//    (2 x 2 blocks of 32 x 32 per wave), K staged 16 at a time through LDS
//    with a register double buffer for the next global tile.
//  * op(A)(m, k) = A[m*lda + k] (TA = false) or A[k*lda + m] (TA = true);
//    op(B)(k, n) = B[k*ldb + n] (TB = false) or B[n*ldb + k] (TB = true).
//  * blockIdx.z = batch * ksplit + split; split s covers K range
//    [s*kchunk, min(K, (s+1)*kchunk)).
//  * Epilogues: store FP32 (per split to its own slice), add into FP64
//    (atomic when ksplit > 1), or store FP32 into the tile-packed symmetric
//    layout (lower 16 x 16 tiles only).
#include "ivx_internal.h"
#include "k_gemm.h"

namespace ivx {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef floatx16 floatx16_t;

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDSW = BM + 32;  // LDS row stride (floats) of the [k][m] / [k][n] tiles

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256, 2) k_gemm(GemmArgs g) {
  __shared__ float As[2][BK][LDSW];
  __shared__ float Bs[2][BK][LDSW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const int batch = blockIdx.z / g.ksplit, split = blockIdx.z % g.ksplit;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (EPI == GEMM_STORE_TP) {
    // skip workgroups whose tiles all lie strictly above the diagonal
    const int mlast = min(m0 + BM, g.M) - 1;
    if ((mlast >> 4) < (n0 >> 4)) return;
  }
  const float* A = g.A + batch * g.sA;
  const float* B = g.B + batch * g.sB;
  const int kb = split * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);

  // global tile loader: 8 elements of A and 8 of B per thread
  float ra[8], rb[8];
  auto load = [&](int k0) {
    if (!TA) {  // rows m, 16 consecutive k
      const int m = m0 + (tid >> 1), kk = k0 + (tid & 1) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        ra[e] = (m < g.M && kk + e < ke) ? A[(int64_t)m * g.lda + kk + e] : 0.0f;
    } else {    // rows k, 128 consecutive m
      const int k = k0 + (tid >> 4), mm = m0 + (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        ra[e] = (k < ke && mm + e < g.M) ? A[(int64_t)k * g.lda + mm + e] : 0.0f;
    }
    if (!TB) {  // rows k, 128 consecutive n
      const int k = k0 + (tid >> 4), nn = n0 + (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        rb[e] = (k < ke && nn + e < g.N) ? B[(int64_t)k * g.ldb + nn + e] : 0.0f;
    } else {    // rows n, 16 consecutive k
      const int n = n0 + (tid >> 1), kk = k0 + (tid & 1) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        rb[e] = (n < g.N && kk + e < ke) ? B[(int64_t)n * g.ldb + kk + e] : 0.0f;
    }
  };
  auto store = [&](int buf) {
    if (!TA) {
      const int m = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][kk + e][m] = ra[e];
    } else {
      const int k = tid >> 4, mm = (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][k][mm + e] = ra[e];
    }
    if (!TB) {
      const int k = tid >> 4, nn = (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][k][nn + e] = rb[e];
    } else {
      const int n = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][kk + e][n] = rb[e];
    }
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};

  const int nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load(kb + (it + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int k = 2 * s + h;
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[cur][k][wm * 64 + i * 32 + l32];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[cur][k][wn * 64 + j * 32 + l32];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue: acc[i][j][r] is C[m][n] with m = mbase + 8*(r/4) + 4*h + r%4, n = nbase + l32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i][j][r];
        if (EPI == GEMM_STORE) {
          float* C = static_cast<float*>(g.C) + batch * g.sC + split * g.sS;
          C[(int64_t)m * g.ldc + n] = v;
        } else if (EPI == GEMM_ADD_F64) {
          double* C = static_cast<double*>(g.C) + batch * g.sC;
          double* dst = C + (int64_t)m * g.ldc + n;
          if (g.ksplit > 1)
            atomicAdd(dst, (double)v);
          else
            *dst += (double)v;
        } else {  // GEMM_STORE_TP: m, n are matrix row / column
          const int bi = m >> 4, bj = n >> 4;
          if (bi >= bj) {
            float* C = static_cast<float*>(g.C) + batch * g.sC;
            C[(int64_t)(bi * (bi + 1) / 2 + bj) * 256 + (m & 15) * 16 + (n & 15)] = v;
          }
        }
      }
    }
}

template <bool TA, bool TB, int EPI>
void launch(const GemmArgs& g, int batches, hipStream_t s) {
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM),
            (unsigned)(batches * g.ksplit));
  k_gemm<TA, TB, EPI><<<grid, 256, 0, s>>>(g);
}

}  // namespace

bool gemm_f32(const GemmArgs& g0, bool ta, bool tb, int epi, int batches, hipStream_t s) {
  GemmArgs g = g0;
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.ksplit == 1 || g.kchunk <= 0) {
    g.ksplit = 1;
    g.kchunk = g.K;
  }
  if (g.M <= 0 || g.N <= 0 || batches <= 0) return true;
#define IVX_GEMM_CASE(TA_, TB_, EPI_)                 \
  if (ta == TA_ && tb == TB_ && epi == EPI_) {        \
    launch<TA_, TB_, EPI_>(g, batches, s);            \
    return true;                                      \
  }
  IVX_GEMM_CASE(false, false, GEMM_STORE)
  IVX_GEMM_CASE(true, false, GEMM_ADD_F64)
  IVX_GEMM_CASE(true, false, GEMM_STORE_TP)
  IVX_GEMM_CASE(false, false, GEMM_ADD_F64)
  IVX_GEMM_CASE(false, true, GEMM_STORE)
  IVX_GEMM_CASE(true, false, GEMM_STORE)
#undef IVX_GEMM_CASE
  return false;
}

}  // namespace ivx

// ------------------------------------------------------------ BF16 split form
// C = A B (both row-major, FP32 in memory) on v_mfma_f32_32x32x16_bf16 with
// FP32 accumulation: each operand is split into BF16 high and low parts while
// it is staged in LDS, and hi*hi + hi*lo + lo*hi are accumulated.  Used for
// the precision assembly L(u) = I + N U in the BF16 form.
namespace ivx {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
constexpr int BRS = 40;  // LDS row stride (bf16) of a [row][16 hi | 16 lo] tile row

__global__ void __launch_bounds__(256, 2) k_gemm_bf16x3_nn(GemmArgs g) {
  __shared__ __bf16 As[128 * BRS];  // [m][k hi 0..15 | k lo 0..15]
  __shared__ __bf16 Bs[128 * BRS];  // [n][k hi | k lo]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const int m0 = blockIdx.y * 128, n0 = blockIdx.x * 128;
  const float* A = g.A;
  const float* B = g.B;
  floatx16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16_t{0};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    // A tile: 128 rows x 16 k (thread: row tid/2, 8 consecutive k)
    {
      const int m = m0 + (tid >> 1), kk = (tid & 1) * 8;
      __bf16* d = As + (tid >> 1) * BRS + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float v = (m < g.M && k0 + kk + e < g.K) ? A[(int64_t)m * g.lda + k0 + kk + e] : 0.0f;
        const __bf16 hi = (__bf16)v;
        d[e] = hi;
        d[16 + e] = (__bf16)(v - (float)hi);
      }
    }
    // B tile: 16 k x 128 columns, stored transposed (thread: k = tid/16, 8 consecutive n)
    {
      const int k = tid >> 4, nn = (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int n = n0 + nn + e;
        const float v = (n < g.N && k0 + k < g.K) ? B[(int64_t)(k0 + k) * g.ldb + n] : 0.0f;
        const __bf16 hi = (__bf16)v;
        Bs[(nn + e) * BRS + k] = hi;
        Bs[(nn + e) * BRS + 16 + k] = (__bf16)(v - (float)hi);
      }
    }
    __syncthreads();
    bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const __bf16* a = As + (wm * 64 + i * 32 + l32) * BRS + 8 * h;
      ah[i] = *reinterpret_cast<const bf16x8_t*>(a);
      al[i] = *reinterpret_cast<const bf16x8_t*>(a + 16);
      const __bf16* b = Bs + (wn * 64 + i * 32 + l32) * BRS + 8 * h;
      bh[i] = *reinterpret_cast<const bf16x8_t*>(b);
      bl[i] = *reinterpret_cast<const bf16x8_t*>(b + 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (m < g.M && n < g.N) static_cast<float*>(g.C)[(int64_t)m * g.ldc + n] = acc[i][j][r];
      }
    }
}

}  // namespace

void gemm_bf16x3_nn(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 127) / 128));
  k_gemm_bf16x3_nn<<<grid, 256, 0, s>>>(g);
}

}  // namespace ivx
