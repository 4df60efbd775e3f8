// E-step (eqs. (3)-(4)) and the M-step accumulators.
//
//  k_tv_prep      per component, FP64: Sigma_c = L L^T, Y_c = L^{-1} T_c,
//                 V_c = Sigma_c^{-1} T_c (both stored FP32), P_c = Sigma_c^{-1}
//                 and log|Sigma_c| (FP64, for the objective).
//  U_c = Y_c^T Y_c = T_c^T Sigma_c^{-1} T_c runs on the FP32 MFMA GEMM with a
//  tile-packed store; L(u) = I + sum_c n_c(u) U_c and the linear term
//  b(u) = p + sum_c V_c^T f_c(u) are two more GEMMs (host code in ivx_tv.hip).
//  k_estep_chol   one workgroup per utterance on the tile-packed L(u):
//                 blocked Cholesky L(u) = G G^T (16 x 16 tiles, trailing
//                 updates on v_mfma_f32_16x16x4_f32), phi = G^{-T} G^{-1} b,
//                 log|L(u)|, and when the covariance is wanted W = G^{-1} and
//                 Phi(u) = W^T W (tile products on MFMA).
#include <cmath>

#include "ivx_internal.h"
#include "ivx_tv.h"

namespace ivx {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int MAXNB = 32;  // tiles per side (R <= 512)

__device__ inline int64_t tile_off(int bi, int bj) { return (int64_t)(bi * (bi + 1) / 2 + bj) * 256; }

// ---------------------------------------------------------------- precompute
__global__ void __launch_bounds__(256)
k_tv_prep(const double* __restrict__ T, const double* __restrict__ Sigma, int D, int R,
          float* __restrict__ Y32, float* __restrict__ V32, double* __restrict__ Psig,
          double* __restrict__ logdet, int* __restrict__ err) {
  extern __shared__ double sm[];
  double* A = sm;           // Sigma -> L, later P
  double* Li = sm + D * D;  // L^{-1}, then 64 zeros
  __shared__ int bad;
  __shared__ double ld;
  const int c = blockIdx.x, t = threadIdx.x;
  for (int i = t; i < D * D; i += 256) A[i] = Sigma[(size_t)c * D * D + i];
  if (t < 64) Li[D * D + t] = 0.0;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    const double djj = A[j * D + j];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (t == 0) bad = 1;
      break;
    }
    const double ljj = sqrt(djj);
    __syncthreads();
    if (t > j && t < D) A[t * D + j] /= ljj;
    if (t == j) A[j * D + j] = ljj;
    __syncthreads();
    if (t > j && t < D) {
      const double lij = A[t * D + j];
      for (int k = j + 1; k <= t; ++k) A[t * D + k] -= lij * A[k * D + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (t == 0) {
      raise_error(err, IVX_ENOTPD, PK_TV_PREP, c);
      logdet[c] = NAN;
    }
    return;
  }
  if (t < D) {
    const int j = t;
    for (int i = 0; i < j; ++i) Li[i * D + j] = 0.0;
    Li[j * D + j] = 1.0 / A[j * D + j];
    for (int i = j + 1; i < D; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += A[i * D + k] * Li[k * D + j];
      Li[i * D + j] = -s / A[i * D + i];
    }
  }
  if (t == 0) {
    double s = 0.0;
    for (int i = 0; i < D; ++i) s += log(A[i * D + i]);
    ld = 2.0 * s;
  }
  __syncthreads();
  // P = L^{-T} L^{-1} (overwrites L)
  for (int e = t; e < D * D; e += 256) {
    const int i = e / D, j = e - i * D;
    double s = 0.0;
    for (int m = (i > j ? i : j); m < D; ++m) s += Li[m * D + i] * Li[m * D + j];
    A[e] = s;
  }
  if (t == 0) logdet[c] = ld;
  __syncthreads();
  for (int e = t; e < D * D; e += 256) Psig[(size_t)c * D * D + e] = A[e];
  // Y = L^{-1} T_c, V = P T_c: thread t holds column r of T_c in registers
  // (D <= 63) and forms all D rows of that column from the LDS copies of
  // L^{-1} and P (same summation order over k as a plain loop).  The k loop
  // has no test: tk[k] = 0 for k >= D and L^{-1} is zero above the diagonal,
  // so the extra terms add exact zeros (the reads past row d stay inside the
  // two matrices and the 64 zeros after them).
  const double* Tc = T + (size_t)c * D * R;
  for (int r = t; r < R; r += 256) {
    double tk[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) tk[k] = (k < D) ? Tc[(size_t)k * R + r] : 0.0;
    for (int d = 0; d < D; ++d) {
      double y = 0.0, v = 0.0;
      const double* Lr = Li + d * D;
      const double* Pr = A + d * D;
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        y += Lr[k] * tk[k];
        v += Pr[k] * tk[k];
      }
      Y32[((size_t)c * D + d) * R + r] = (float)y;
      V32[((size_t)c * D + d) * R + r] = (float)v;
    }
  }
}

// L(u) += I on every diagonal position of the tile-packed layout (padding too)
__global__ void k_add_identity(float* __restrict__ L, int64_t TP, int nb, int64_t U) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = U * nb * 16;
  if (i >= n) return;
  const int64_t u = i / (nb * 16);
  const int d = (int)(i - u * nb * 16);
  const int bk = d >> 4, e = d & 15;
  L[u * TP + tile_off(bk, bk) + e * 17] += 1.0f;
}

// b[u][r] = p[r] + sum_s part[s][u][r]
__global__ void k_reduce_b(const float* __restrict__ part, int nsplit, int64_t sstride, int64_t U,
                           int R, const double* __restrict__ p, float* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= U * R) return;
  double s = p[i % R];
  for (int k = 0; k < nsplit; ++k) s += part[k * sstride + i];
  b[i] = (float)s;
}

__device__ inline void wave_sync() { __builtin_amdgcn_wave_barrier(); }

__device__ inline void decode_tri(int t, int& ii, int& jj) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ii = i;
  jj = t - i * (i + 1) / 2;
}

// -------------------------------------------------- per-utterance E-step core
__global__ void __launch_bounds__(256)
k_estep_chol(int R, int nb, int64_t TP, float* __restrict__ Lb, float* __restrict__ Wb,
             const float* __restrict__ bvec, const double* __restrict__ p,
             float* __restrict__ phi, double* __restrict__ llu, int* __restrict__ info,
             int want_cov, int* __restrict__ err) {
  __shared__ float dg[256];
  __shared__ __attribute__((aligned(16))) float pan[(MAXNB - 1) * 256];
  __shared__ float vec[MAXNB * 16];
  __shared__ float wsc[4][256];
  // reduction scratch, used only after the factorisation: shares the panel's
  // memory (keeps the workgroup under 40 KB of LDS, four per CU)
  double* red = reinterpret_cast<double*>(pan);
  __shared__ int s_bad;
  const int64_t u = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  float* L = Lb + u * TP;
  float* W = Wb + u * TP;
  if (tid == 0) s_bad = 0;
  __syncthreads();

  // ---- blocked Cholesky L = G G^T (G overwrites the lower tiles)
  for (int k = 0; k < nb; ++k) {
    if (wave == 0) {
      float* Lkk = L + tile_off(k, k);
      for (int e = lane; e < 256; e += 64) dg[e] = Lkk[e];
      wave_sync();
      for (int j = 0; j < 16; ++j) {
        const float piv = dg[j * 16 + j];
        if (!(piv > 0.0f) || !isfinite(piv)) {
          if (lane == 0) s_bad = k * 16 + j + 1;
          break;
        }
        const float ljj = sqrtf(piv);
        wave_sync();
        if (lane > j && lane < 16) dg[lane * 16 + j] /= ljj;
        if (lane == j) dg[j * 16 + j] = ljj;
        wave_sync();
        for (int e = lane; e < 256; e += 64) {
          const int i = e >> 4, cc = e & 15;
          if (cc > j && i >= cc) dg[e] -= dg[i * 16 + j] * dg[cc * 16 + j];
        }
        wave_sync();
      }
      for (int e = lane; e < 256; e += 64) {
        const int i = e >> 4, cc = e & 15;
        const float v = (cc <= i) ? dg[e] : 0.0f;
        dg[e] = v;
        Lkk[e] = v;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int m = nb - k - 1;
    // panel tiles (k+1+it, k): X <- X G_kk^{-T}, row by row
    for (int row = tid; row < m * 16; row += 256) {
      const int it = row >> 4, r = row & 15;
      float* src = L + tile_off(k + 1 + it, k) + r * 16;
      float x[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) x[cc] = src[cc];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        float s = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) s -= x[l] * dg[j * 16 + l];
        x[j] = s / dg[j * 16 + j];
        // one column at a time: keeps the LDS reads of later columns from
        // being hoisted into registers
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        src[cc] = x[cc];
        pan[it * 256 + r * 16 + cc] = x[cc];
      }
    }
    __syncthreads();
    // trailing tiles (k+1+ii, k+1+jj), jj <= ii: C -= P_ii P_jj^T
    // four tiles per wave and pass, all loaded before their MFMAs (tiles
    // past the end repeat the pass's first tile and are not stored)
    const int ntile = m * (m + 1) / 2;
    for (int t0 = wave; t0 < ntile; t0 += 16) {
      floatx4 acc[4];
      float* Ct[4];
      int ii[4], jj[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        decode_tri(t0 + 4 * v < ntile ? t0 + 4 * v : t0, ii[v], jj[v]);
        Ct[v] = L + tile_off(k + 1 + ii[v], k + 1 + jj[v]);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[v][r] = Ct[v][(4 * q16 + r) * 16 + l16];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float* Pi = pan + ii[v] * 256;
        const float* Pj = pan + jj[v] * 256;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float a = -Pi[l16 * 16 + 4 * q + q16];
          const float bb = Pj[l16 * 16 + 4 * q + q16];
          acc[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, acc[v], 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (t0 + 4 * v >= ntile) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) Ct[v][(4 * q16 + r) * 16 + l16] = acc[v][r];
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) {
      if (info) info[u] = s_bad;
      raise_error(err, IVX_ENOTPD, PK_ESTEP_CHOL, (int)u);
      llu[u] = 0.0;
    }
    for (int i = tid; i < R; i += 256) phi[u * R + i] = NAN;
    return;
  }
  if (info && tid == 0) info[u] = 0;

  // ---- log|L| = 2 sum log G_ii ; vec = b
  double ls = 0.0;
  for (int i = tid; i < R; i += 256) ls += log((double)L[tile_off(i >> 4, i >> 4) + (i & 15) * 17]);
  red[tid] = ls;
  for (int i = tid; i < nb * 16; i += 256) vec[i] = (i < R) ? bvec[u * R + i] : 0.0f;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double logdet = 2.0 * red[0];
  __syncthreads();

  // ---- forward solve G z = b
  for (int k = 0; k < nb; ++k) {
    if (wave == 0) {
      const float* Gkk = L + tile_off(k, k);
      for (int e = lane; e < 256; e += 64) wsc[0][e] = Gkk[e];
      wave_sync();
      for (int j = 0; j < 16; ++j) {
        const float zj = vec[k * 16 + j] / wsc[0][j * 16 + j];
        wave_sync();
        if (lane == j) vec[k * 16 + j] = zj;
        if (lane > j && lane < 16) vec[k * 16 + lane] -= wsc[0][lane * 16 + j] * zj;
        wave_sync();
      }
    }
    __syncthreads();
    for (int row = tid; row < (nb - k - 1) * 16; row += 256) {
      const int it = row >> 4, r = row & 15;
      const float* G = L + tile_off(k + 1 + it, k) + r * 16;
      float s = 0.0f;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) s += G[cc] * vec[k * 16 + cc];
      vec[(k + 1) * 16 + row] -= s;
    }
    __syncthreads();
  }
  // ---- backward solve G^T phi = z
  for (int k = nb - 1; k >= 0; --k) {
    if (wave == 0) {
      const float* Gkk = L + tile_off(k, k);
      for (int e = lane; e < 256; e += 64) wsc[0][e] = Gkk[e];
      wave_sync();
      for (int j = 15; j >= 0; --j) {
        const float xj = vec[k * 16 + j] / wsc[0][j * 16 + j];
        wave_sync();
        if (lane == j) vec[k * 16 + j] = xj;
        if (lane < j) vec[k * 16 + lane] -= wsc[0][j * 16 + lane] * xj;
        wave_sync();
      }
    }
    __syncthreads();
    for (int idx = tid; idx < k * 16; idx += 256) {
      const int jb = idx >> 4, cc = idx & 15;
      const float* G = L + tile_off(k, jb);
      float s = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) s += G[r * 16 + cc] * vec[k * 16 + r];
      vec[idx] -= s;
    }
    __syncthreads();
  }
  // ---- phi and the utterance's objective share
  double bp = 0.0, pp = 0.0;
  for (int i = tid; i < R; i += 256) {
    const float ph = vec[i];
    phi[u * R + i] = ph;
    bp += (double)bvec[u * R + i] * (double)ph;
    pp += p[i] * p[i];
  }
  red[tid] = bp - pp;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) llu[u] = -0.5 * logdet + 0.5 * red[0];
  if (!want_cov) return;

  // ---- W = G^{-1}: diagonal tiles
  for (int k = wave; k < nb; k += 4) {
    const float* Gkk = L + tile_off(k, k);
    for (int e = lane; e < 256; e += 64) wsc[wave][e] = Gkk[e];
    wave_sync();
    if (lane < 16) {
      const int cc = lane;
      float x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float s = (i == cc) ? 1.0f : 0.0f;
#pragma unroll
        for (int l = 0; l < i; ++l) s -= wsc[wave][i * 16 + l] * x[l];
        x[i] = (i < cc) ? 0.0f : s / wsc[wave][i * 16 + i];
      }
      float* Wkk = W + tile_off(k, k);
#pragma unroll
      for (int i = 0; i < 16; ++i) Wkk[i * 16 + cc] = x[i];
    }
    wave_sync();
  }
  __syncthreads();
  // ---- W off-diagonal tiles, block row by block row:
  //      W_ik = -W_ii sum_{j=k}^{i-1} G_ij W_jk
  for (int i = 1; i < nb; ++i) {
    for (int k = wave; k < i; k += 4) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      // four j steps per pass: all their loads first, then the MFMAs
      for (int j0 = k; j0 < i; j0 += 4) {
        float av[4][4], bv[4][4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = j0 + jj;
          const bool ok = j < i;
          const float* Gij = L + tile_off(i, ok ? j : k);
          const float* Wjk = W + tile_off(ok ? j : k, k);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            av[jj][q] = ok ? Gij[l16 * 16 + 4 * q + q16] : 0.0f;
            bv[jj][q] = ok ? Wjk[(4 * q + q16) * 16 + l16] : 0.0f;
          }
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jj][q], bv[jj][q], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) wsc[wave][(4 * q16 + r) * 16 + l16] = acc[r];
      wave_sync();
      const float* Wii = W + tile_off(i, i);
      floatx4 res = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = -Wii[l16 * 16 + 4 * q + q16];
        const float bb = wsc[wave][(4 * q + q16) * 16 + l16];
        res = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, res, 0, 0, 0);
      }
      wave_sync();
      float* Wik = W + tile_off(i, k);
#pragma unroll
      for (int r = 0; r < 4; ++r) Wik[(4 * q16 + r) * 16 + l16] = res[r];
    }
    __syncthreads();
  }
  // ---- Phi = W^T W into the L buffer: Phi_ij = sum_{k >= i} W_ki^T W_kj
  const int ntile = nb * (nb + 1) / 2;
  for (int t = wave; t < ntile; t += 4) {
    int i, j;
    decode_tri(t, i, j);
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    // four k steps per pass: all their loads first, then the MFMAs
    for (int k0 = i; k0 < nb; k0 += 4) {
      float av[4][4], bv[4][4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = k0 + kk;
        const bool ok = k < nb;
        const float* Wki = W + tile_off(ok ? k : i, i);
        const float* Wkj = W + tile_off(ok ? k : i, j);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[kk][q] = ok ? Wki[(4 * q + q16) * 16 + l16] : 0.0f;
          bv[kk][q] = ok ? Wkj[(4 * q + q16) * 16 + l16] : 0.0f;
        }
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk][q], bv[kk][q], acc, 0, 0, 0);
    }
    float* Pt = L + tile_off(i, j);
#pragma unroll
    for (int r = 0; r < 4; ++r) Pt[(4 * q16 + r) * 16 + l16] = acc[r];
  }
}

// tile t of the tile-packed layout -> its block row / column (t = bi (bi + 1) / 2 + bj)
__device__ inline void tile_decode(int t, int& bi, int& bj) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  bi = i;
  bj = t - i * (i + 1) / 2;
}

// Phi (tile-packed) -> packed upper triangle, row by row.  One workgroup per
// (utterance, tile): the tile is read whole, transposed through LDS, and
// element (i, j), i <= j (lower tile (j, i) at (j & 15, i & 15)) is written
// with lanes along j, i.e. consecutive packed positions of row i.
__global__ void __launch_bounds__(256) k_tp_to_packed(const float* __restrict__ Ptp, int64_t TP,
                                                      int R, float* __restrict__ out) {
  __shared__ float ts[16][17];
  const int64_t u = blockIdx.x;
  const int t = blockIdx.y, tid = threadIdx.x;
  int bi, bj;
  tile_decode(t, bi, bj);
  ts[tid >> 4][tid & 15] = Ptp[u * TP + (int64_t)t * 256 + tid];
  __syncthreads();
  const int cl = tid >> 4, rl = tid & 15;
  const int i = bj * 16 + cl, j = bi * 16 + rl;
  if (j < R && i <= j) {
    const int64_t np = (int64_t)R * (R + 1) / 2;
    out[u * np + (int64_t)i * R - (int64_t)i * (i - 1) / 2 + (j - i)] = ts[rl][cl];
  }
}

// Psi(u) = Phi(u) + phi phi^T in tile-packed FP64 (padding zero); the FP32
// inputs are widened first, so the product phi phi^T is exact.  One
// workgroup per (utterance, tile): packed entries are read with lanes along
// the tile's rows (consecutive positions of one packed row below the
// diagonal), transposed through LDS and the tile written whole.
__global__ void __launch_bounds__(256) k_packed_to_psi(const float* __restrict__ Phi,
                                                       const float* __restrict__ phi, int64_t TP,
                                                       int R, double* __restrict__ Psi) {
  __shared__ double ts[16][17];
  const int64_t u = blockIdx.x;
  const int t = blockIdx.y, tid = threadIdx.x;
  int bi, bj;
  tile_decode(t, bi, bj);
  const int cl = tid >> 4, rl = tid & 15;
  const int r = bi * 16 + rl, c = bj * 16 + cl;
  double v = 0.0;
  if (r < R && c < R) {
    const int i = c < r ? c : r, j = c < r ? r : c;  // i <= j
    const int64_t k = (int64_t)i * R - (int64_t)i * (i - 1) / 2 + (j - i);
    v = (double)Phi[u * ((int64_t)R * (R + 1) / 2) + k] +
        (double)phi[u * R + r] * (double)phi[u * R + c];
  }
  ts[rl][cl] = v;
  __syncthreads();
  Psi[u * TP + (int64_t)t * 256 + tid] = ts[tid >> 4][tid & 15];
}

// Column sums over the utterances, in two passes with a fixed order (results
// do not depend on scheduling): pass 1, blockIdx.y = row chunk s of CSPLIT,
// part[s][col] = sum over the chunk's u of the column, columns [n | phi | Psi]
__global__ void k_colsums_part(const float* __restrict__ n, const float* __restrict__ phi,
                               const double* __restrict__ Psi, int64_t U, int C, int R,
                               int64_t TP, double* __restrict__ part) {
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = C + R + TP;
  if (col >= total) return;
  const int64_t ucnt = (U + CSPLIT - 1) / CSPLIT;
  const int64_t u0 = blockIdx.y * ucnt, u1 = min(U, u0 + ucnt);
  double s = 0.0;
  if (col < C) {
    for (int64_t u = u0; u < u1; ++u) s += n[u * C + col];
  } else if (col < C + R) {
    const int64_t r = col - C;
    for (int64_t u = u0; u < u1; ++u) s += phi[u * R + r];
  } else {
    const int64_t e = col - C - R;
    for (int64_t u = u0; u < u1; ++u) s += Psi[u * TP + e];
  }
  part[blockIdx.y * total + col] = s;
}

// pass 2: N[c] += sum_s part[s][c]; h[r] += ...; H[e] += ...; count += U
__global__ void k_colsums_fin(const double* __restrict__ part, int64_t U, int C, int R, int64_t TP,
                              double* __restrict__ N, double* __restrict__ h,
                              double* __restrict__ H, double* __restrict__ count) {
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = C + R + TP;
  if (col == 0) count[0] += (double)U;
  if (col >= total) return;
  double s = 0.0;
  for (int k = 0; k < CSPLIT; ++k) s += part[k * total + col];
  if (col < C)
    N[col] += s;
  else if (col < C + R)
    h[col - C] += s;
  else
    H[col - C - R] += s;
}

}  // namespace

void launch_tv_prep(ivx_ctx* ctx, hipStream_t s) {
  const size_t lds = sizeof(double) * (2 * ctx->D * ctx->D + 64);
  k_tv_prep<<<ctx->C, 256, lds, s>>>(ctx->T, ctx->Sigma, ctx->D, ctx->R, ctx->Y32, ctx->V32,
                                     ctx->Psig, ctx->sig_logdet, ctx->dev_err);
}

void launch_add_identity(ivx_ctx* ctx, float* L, int64_t U, hipStream_t s) {
  const int nb = (ctx->R + 15) / 16;
  const int64_t n = U * nb * 16;
  if (n <= 0) return;
  k_add_identity<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L, ctx->TP, nb, U);
}

void launch_reduce_b(ivx_ctx* ctx, const float* part, int nsplit, int64_t sstride, int64_t U,
                     float* b, hipStream_t s) {
  const int64_t n = U * ctx->R;
  if (n <= 0) return;
  k_reduce_b<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(part, nsplit, sstride, U, ctx->R, ctx->p, b);
}

void launch_estep_chol(ivx_ctx* ctx, int64_t U, float* Lb, float* Wb, const float* b, float* phi,
                       double* llu, int* info, float* Phi, hipStream_t s) {
  if (U <= 0) return;
  if (!ctx->tune.estep_global && estep_rr_fits(ctx->R)) {
    launch_estep_rr(ctx, U, Lb, b, phi, llu, info, Phi, s);
    return;
  }
  const int nb = (ctx->R + 15) / 16;
  k_estep_chol<<<(unsigned)U, 256, 0, s>>>(ctx->R, nb, ctx->TP, Lb, Wb, b, ctx->p, phi, llu, info,
                                           Phi != nullptr ? 1 : 0, ctx->dev_err);
  if (Phi) launch_tp_to_packed(ctx, Lb, U, Phi, s);
}

void launch_tp_to_packed(ivx_ctx* ctx, const float* Ptp, int64_t U, float* out, hipStream_t s) {
  if (U <= 0) return;
  const unsigned ntile = (unsigned)(ctx->TP / 256);
  k_tp_to_packed<<<dim3((unsigned)U, ntile), 256, 0, s>>>(Ptp, ctx->TP, ctx->R, out);
}

void launch_packed_to_psi(ivx_ctx* ctx, const float* Phi, const float* phi, int64_t U, double* Psi,
                          hipStream_t s) {
  if (U <= 0) return;
  const unsigned ntile = (unsigned)(ctx->TP / 256);
  k_packed_to_psi<<<dim3((unsigned)U, ntile), 256, 0, s>>>(Phi, phi, ctx->TP, ctx->R, Psi);
}

void launch_colsums(ivx_ctx* ctx, const float* n, const float* phi, const double* Psi, int64_t U,
                    const ivx_accum* acc, hipStream_t s) {
  const int64_t total = ctx->C + ctx->R + ctx->TP;
  const unsigned nbx = (unsigned)((total + 255) / 256);
  k_colsums_part<<<dim3(nbx, CSPLIT), 256, 0, s>>>(n, phi, Psi, U, ctx->C, ctx->R, ctx->TP,
                                                   ctx->colpart);
  k_colsums_fin<<<nbx, 256, 0, s>>>(ctx->colpart, U, ctx->C, ctx->R, ctx->TP, acc->N, acc->h,
                                    acc->H, acc->count);
}

}  // namespace ivx
