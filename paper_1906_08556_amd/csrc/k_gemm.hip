// Dense FP32 GEMM on MFMA (v_mfma_f32_32x32x2_f32) for the E-step and M-step
// contractions: C = op(A) op(B), M x N x K.
//
//  * 256 x 128 output tile per 256-thread workgroup, 2 x 2 waves of 128 x 64
//    (4 x 2 blocks of 32 x 32 per wave: eight independent accumulators), K
//    staged 16 at a time through LDS with a register double buffer for the
//    next global tile.
//  * op(A)(m, k) = A[m*lda + k] (TA = false) or A[k*lda + m] (TA = true);
//    op(B)(k, n) = B[k*ldb + n] (TB = false) or B[n*ldb + k] (TB = true).
//  * blockIdx.z = batch * ksplit + split; split s covers K range
//    [s*kchunk, min(K, (s+1)*kchunk)).
//  * Tile order: the larger operand is streamed once -- with m_fast the M
//    tiles of one column block of B are consecutive, otherwise the N tiles of
//    one row block of A.
//  * Epilogues: store FP32 (per split to its own slice), add into FP64
//    (atomic when ksplit > 1), or store FP32 into the tile-packed symmetric
//    layout (lower 16 x 16 tiles only).
#include "ivx_internal.h"
#include "k_gemm.h"

namespace ivx {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef floatx16 floatx16_t;

constexpr int BM = 256, BN = 128, BK = 16;
constexpr int LDA_S = BM + 32;  // LDS row stride (floats) of the [k][m] tile
constexpr int LDB_S = BN + 32;  // LDS row stride (floats) of the [k][n] tile

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256, 2) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) float As[2][BK][LDA_S];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK][LDB_S];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // wave tile: 128 rows x 64 columns
  const int h = lane >> 5, l32 = lane & 31;
  const int batch = blockIdx.z / g.ksplit, split = blockIdx.z % g.ksplit;
  const int m0 = (g.m_fast ? blockIdx.x : blockIdx.y) * BM;
  const int n0 = (g.m_fast ? blockIdx.y : blockIdx.x) * BN;
  if (EPI == GEMM_STORE_TP) {
    // skip workgroups whose tiles all lie strictly above the diagonal
    const int mlast = min(m0 + BM, g.M) - 1;
    if ((mlast >> 4) < (n0 >> 4)) return;
  }
  const float* A = g.A + batch * g.sA;
  const float* B = g.B + batch * g.sB;
  const int kb = split * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);

  // global tile loader: lanes run along the contiguous dimension of each
  // operand (coalesced), four consecutive elements per load (float4 where
  // the rows are 16-byte aligned), 4 loads of A and 2 of B per thread:
  //  !TA  A[m][k]: m = 64 j + tid / 4,  k = 4 (tid % 4)
  //   TA  A[k][m]: k = 4 j + tid / 64,  m = 4 (tid % 64)
  //  !TB  B[k][n]: k = 8 j + tid / 32,  n = 4 (tid % 32)
  //   TB  B[n][k]: n = 64 j + tid / 4,  k = 4 (tid % 4)
  const bool vecA = g.lda % 4 == 0 && g.sA % 4 == 0 && reinterpret_cast<uintptr_t>(g.A) % 16 == 0;
  const bool vecB = g.ldb % 4 == 0 && g.sB % 4 == 0 && reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
  float4 ra[4], rb[2];
  // nval: how many of the four consecutive elements at p lie in bounds
  auto ld4 = [](const float* p, int nval, bool vec) -> float4 {
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (nval >= 4 && vec) {
      v = *reinterpret_cast<const float4*>(p);
    } else {
      if (nval > 0) v.x = p[0];
      if (nval > 1) v.y = p[1];
      if (nval > 2) v.z = p[2];
      if (nval > 3) v.w = p[3];
    }
    return v;
  };
  // tiles inside both operands with aligned rows: unguarded float4 loads
  const bool inner = vecA && vecB && m0 + BM <= g.M && n0 + BN <= g.N;
  auto load = [&](int k0) {
    if (inner && k0 + BK <= ke) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float* p = !TA ? A + (int64_t)(m0 + 64 * j + (tid >> 2)) * g.lda + k0 + 4 * (tid & 3)
                             : A + (int64_t)(k0 + 4 * j + (tid >> 6)) * g.lda + m0 + 4 * (tid & 63);
        ra[j] = *reinterpret_cast<const float4*>(p);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float* p = !TB ? B + (int64_t)(k0 + 8 * j + (tid >> 5)) * g.ldb + n0 + 4 * (tid & 31)
                             : B + (int64_t)(n0 + 64 * j + (tid >> 2)) * g.ldb + k0 + 4 * (tid & 3);
        rb[j] = *reinterpret_cast<const float4*>(p);
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!TA) {
        const int m = m0 + 64 * j + (tid >> 2), k = k0 + 4 * (tid & 3);
        const int nv = m < g.M ? min(4, ke - k) : 0;
        ra[j] = ld4(A + (int64_t)m * g.lda + k, nv, vecA);
      } else {
        const int k = k0 + 4 * j + (tid >> 6), m = m0 + 4 * (tid & 63);
        const int nv = k < ke ? min(4, g.M - m) : 0;
        ra[j] = ld4(A + (int64_t)k * g.lda + m, nv, vecA);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!TB) {
        const int k = k0 + 8 * j + (tid >> 5), n = n0 + 4 * (tid & 31);
        const int nv = k < ke ? min(4, g.N - n) : 0;
        rb[j] = ld4(B + (int64_t)k * g.ldb + n, nv, vecB);
      } else {
        const int n = n0 + 64 * j + (tid >> 2), k = k0 + 4 * (tid & 3);
        const int nv = n < g.N ? min(4, ke - k) : 0;
        rb[j] = ld4(B + (int64_t)n * g.ldb + k, nv, vecB);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!TA) {
        const int m = 64 * j + (tid >> 2), k = 4 * (tid & 3);
        As[buf][k][m] = ra[j].x;
        As[buf][k + 1][m] = ra[j].y;
        As[buf][k + 2][m] = ra[j].z;
        As[buf][k + 3][m] = ra[j].w;
      } else {
        *reinterpret_cast<float4*>(&As[buf][4 * j + (tid >> 6)][4 * (tid & 63)]) = ra[j];
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!TB) {
        *reinterpret_cast<float4*>(&Bs[buf][8 * j + (tid >> 5)][4 * (tid & 31)]) = rb[j];
      } else {
        const int n = 64 * j + (tid >> 2), k = 4 * (tid & 3);
        Bs[buf][k][n] = rb[j].x;
        Bs[buf][k + 1][n] = rb[j].y;
        Bs[buf][k + 2][n] = rb[j].z;
        Bs[buf][k + 3][n] = rb[j].w;
      }
    }
  };

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
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
      float av[4], bv[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[cur][k][wm * 128 + i * 32 + l32];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[cur][k][wn * 64 + j * 32 + l32];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue: acc[i][j][r] is C[m][n] with m = mbase + 8*(r/4) + 4*h + r%4, n = nbase + l32
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 128 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
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
  const unsigned nt = (unsigned)((g.N + BN - 1) / BN), mt = (unsigned)((g.M + BM - 1) / BM);
  const unsigned z = (unsigned)(batches * g.ksplit);
  const dim3 grid = g.m_fast ? dim3(mt, nt, z) : dim3(nt, mt, z);
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
  // stream the larger operand (per K) once; y-dimension limits apply
  const int64_t mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
  g.m_fast = ((int64_t)g.N > (int64_t)g.M && nt <= 65535) || mt > 65535 ? 1 : 0;
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
// C[m][n] = sum_k A[m][k] B[n][k] (FP32 result) on v_mfma_f32_32x32x16_bf16
// from operands stored pre-split as BF16 high and low parts (v = hi + lo,
// both K-contiguous): hi*hi + hi*lo + lo*hi are accumulated in FP32.  Used
// for the precision assembly L(u) = I + N U in the BF16 form.  128 x 128
// output tile per workgroup, K staged 16 at a time, double-buffered LDS.
namespace ivx {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
constexpr int SR = 24;  // LDS row stride (bf16) of a staged 16-k row (48 B)

__global__ void __launch_bounds__(256, 2)
k_gemm_bf16x3_nt(const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo, int64_t lda,
                 const __bf16* __restrict__ Bhi, const __bf16* __restrict__ Blo, int64_t ldb,
                 float* __restrict__ C, int64_t ldc, int M, int N, int K, int m_fast) {
  // [buf][operand: A hi, A lo, B hi, B lo][128 rows][SR]
  __shared__ __bf16 St[2][4][128 * SR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  // m_fast: the M tiles of one column block of B run consecutively
  const int64_t m0 = (int64_t)(m_fast ? blockIdx.x : blockIdx.y) * 128;
  const int64_t n0 = (int64_t)(m_fast ? blockIdx.y : blockIdx.x) * 128;
  // loader: thread covers row tid / 2 and k half (tid & 1) * 8 of each operand
  const int lr = tid >> 1, lk = (tid & 1) * 8;
  uint4 rg[4];
  auto load = [&](int k0) {
    const int64_t am = m0 + lr, bn = n0 + lr;
    const int k = k0 + lk;
    const bool ka = k < K;  // K is a multiple of 8
    rg[0] = (am < M && ka) ? *reinterpret_cast<const uint4*>(Ahi + am * lda + k) : make_uint4(0, 0, 0, 0);
    rg[1] = (am < M && ka) ? *reinterpret_cast<const uint4*>(Alo + am * lda + k) : make_uint4(0, 0, 0, 0);
    rg[2] = (bn < N && ka) ? *reinterpret_cast<const uint4*>(Bhi + bn * ldb + k) : make_uint4(0, 0, 0, 0);
    rg[3] = (bn < N && ka) ? *reinterpret_cast<const uint4*>(Blo + bn * ldb + k) : make_uint4(0, 0, 0, 0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int o = 0; o < 4; ++o) *reinterpret_cast<uint4*>(&St[buf][o][lr * SR + lk]) = rg[o];
  };
  floatx16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16_t{0};
  const int nk = (K + 15) / 16;
  load(0);
  store(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load((it + 1) * 16);
    bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra = (wm * 64 + i * 32 + l32) * SR + 8 * h;
      const int rb = (wn * 64 + i * 32 + l32) * SR + 8 * h;
      ah[i] = *reinterpret_cast<const bf16x8_t*>(&St[cur][0][ra]);
      al[i] = *reinterpret_cast<const bf16x8_t*>(&St[cur][1][ra]);
      bh[i] = *reinterpret_cast<const bf16x8_t*>(&St[cur][2][rb]);
      bl[i] = *reinterpret_cast<const bf16x8_t*>(&St[cur][3][rb]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t n = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (m < M && n < N) C[m * ldc + n] = acc[i][j][r];
      }
    }
}

// src [rows][cols] FP32 -> hi / lo [rows][ldo] BF16 (cols <= ldo; padding 0)
__global__ void k_split_bf16(const float* __restrict__ src, int64_t rows, int64_t cols,
                             int64_t ldo, __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  const int64_t n = rows * ldo;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldo, c = i - r * ldo;
    const float v = (c < cols) ? src[r * cols + c] : 0.0f;
    const __bf16 vh = (__bf16)v;
    hi[i] = vh;
    lo[i] = (__bf16)(v - (float)vh);
  }
}

// src [rows][cols] FP32 -> hi / lo [cols][ldo] BF16 transposed (rows <= ldo;
// padding 0), through 64 x 64 LDS tiles
__global__ void __launch_bounds__(256)
k_split_bf16_t(const float* __restrict__ src, int64_t rows, int64_t cols, int64_t ldo,
               __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  __shared__ float t[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int rr = e >> 6, cc = e & 63;
    const int64_t r = r0 + rr, c = c0 + cc;
    t[rr][cc] = (r < rows && c < cols) ? src[r * cols + c] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int cc = e >> 6, rr = e & 63;
    const int64_t r = r0 + rr, c = c0 + cc;
    if (c < cols && r < ldo) {
      const float v = t[rr][cc];
      const __bf16 vh = (__bf16)v;
      hi[c * ldo + r] = vh;
      lo[c * ldo + r] = (__bf16)(v - (float)vh);
    }
  }
}

}  // namespace

void split_bf16(const float* src, int64_t rows, int64_t cols, int64_t ldo, __bf16* hi, __bf16* lo,
                hipStream_t s) {
  if (rows <= 0) return;
  k_split_bf16<<<2048, 256, 0, s>>>(src, rows, cols, ldo, hi, lo);
}

void split_bf16_transposed(const float* src, int64_t rows, int64_t cols, int64_t ldo, __bf16* hi,
                           __bf16* lo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((ldo + 63) / 64));
  k_split_bf16_t<<<grid, 256, 0, s>>>(src, rows, cols, ldo, hi, lo);
}

void gemm_bf16x3_nt(const __bf16* Ahi, const __bf16* Alo, int64_t lda, const __bf16* Bhi,
                    const __bf16* Blo, int64_t ldb, float* C, int64_t ldc, int M, int N, int K,
                    hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const unsigned mt = (unsigned)((M + 127) / 128), nt = (unsigned)((N + 127) / 128);
  const int m_fast = (N > M && nt <= 65535u) || mt > 65535u ? 1 : 0;  // stream B once
  const dim3 grid = m_fast ? dim3(mt, nt) : dim3(nt, mt);
  k_gemm_bf16x3_nt<<<grid, 256, 0, s>>>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, M, N, K, m_fast);
}

}  // namespace ivx
