// FP64 tile kernels for symmetric positive definite matrices in the
// tile-packed layout (16 x 16 lower tiles, row-major tile order, each tile
// row-major), on v_mfma_f64_16x16x4f64.  Used by the M-step solve and the
// minimum-divergence set-up; every function is called by all 256 threads of
// the workgroup.
#pragma once

#include "ivx_internal.h"

namespace ivx {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ inline int64_t tp_off(int bi, int bj) { return (int64_t)(bi * (bi + 1) / 2 + bj) * 256; }

// v_mfma_f64_16x16x4f64 operand layout: lane l holds A[l % 16][k] and
// B[k][l % 16] with k = l / 16 of each 4-wide K step; result register r of
// lane l is C[4 r + l / 16][l % 16].
// acc += s * X Y^T for 16 x 16 row-major tiles given by element accessors
// x(i, k), y(j, k).
template <typename FX, typename FY>
__device__ inline doublex4 mma16_xyt(FX x, FY y, doublex4 acc, double s) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q16 = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double a = s * x(l16, 4 * q + q16);
    const double b = y(l16, 4 * q + q16);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// tiles per wave and pass in the update loops
constexpr int UT = 2;

__device__ inline void tri_decode(int t, int& ii, int& jj) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ii = i;
  jj = t - i * (i + 1) / 2;
}

// Blocked right-looking Cholesky A = G G^T of an nb x nb-tile matrix in
// place (lower tiles).  The inverse of every diagonal tile, W_k = G_kk^{-1}
// (row-major, upper part zero), goes to Winv[k * 256].  LDS: dg [256],
// pan [(nb - 1) * 256].  Returns 0, or 1 + the first row whose pivot was not
// positive (then A is partly overwritten).
__device__ inline int chol_tp64(double* __restrict__ A, int nb, double* __restrict__ Winv,
                                double* dg, double* pan, int* s_bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  if (tid == 0) *s_bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (wave == 0) {
      double* Akk = A + tp_off(k, k);
      for (int e = lane; e < 256; e += 64) dg[e] = Akk[e];
      __builtin_amdgcn_wave_barrier();
      for (int j = 0; j < 16; ++j) {
        const double piv = dg[j * 16 + j];
        if (!(piv > 0.0) || !isfinite(piv)) {
          if (lane == 0) *s_bad = k * 16 + j + 1;
          break;  // piv is the same in every lane: uniform exit
        }
        const double ljj = sqrt(piv);
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < 16) dg[lane * 16 + j] /= ljj;
        if (lane == j) dg[j * 16 + j] = ljj;
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < 256; e += 64) {
          const int i = e >> 4, c = e & 15;
          if (c > j && i >= c) dg[e] -= dg[i * 16 + j] * dg[c * 16 + j];
        }
        __builtin_amdgcn_wave_barrier();
      }
      for (int e = lane; e < 256; e += 64) {
        const int i = e >> 4, c = e & 15;
        const double v = (c <= i) ? dg[e] : 0.0;
        dg[e] = v;
        Akk[e] = v;
      }
      __builtin_amdgcn_wave_barrier();
      // W = G_kk^{-1}: lane j < 16 solves column j by forward substitution
      if (lane < 16 && *s_bad == 0) {
        const int j = lane;
        double w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
          for (int l = 0; l < i; ++l) s -= dg[i * 16 + l] * w[l];
          w[i] = (i >= j) ? s / dg[i * 16 + i] : 0.0;
          // one row at a time: keeps the row's LDS reads from piling up in registers
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Winv[k * 256 + i * 16 + j] = w[i];
      }
    }
    __syncthreads();
    if (*s_bad) return *s_bad;
    const double* W = Winv + k * 256;
    const int m = nb - k - 1;
    // panel: P_i = A_(k+1+i),k W^T, to A and LDS
    for (int it = wave; it < m; it += 4) {
      double* At = A + tp_off(k + 1 + it, k);
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return At[i * 16 + l]; },
                      [&](int j, int l) { return W[j * 16 + l]; }, acc, 1.0);
      // all lanes have read the tile before anyone writes it
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = (4 * r + q16) * 16 + l16;
        At[e] = acc[r];
        pan[it * 256 + e] = acc[r];
      }
    }
    __syncthreads();
    // trailing update: A_(k+1+ii),(k+1+jj) -= P_ii P_jj^T, jj <= ii; each
    // wave takes UT tiles per pass and loads all of them before the MFMAs
    // (tiles past the end repeat the pass's first tile and are not stored)
    const int nt = m * (m + 1) / 2;
    for (int t0 = wave; t0 < nt; t0 += 4 * UT) {
      doublex4 acc[UT];
      double* Ct[UT];
      int ii[UT], jj[UT];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int t = t0 + 4 * u < nt ? t0 + 4 * u : t0;
        tri_decode(t, ii[u], jj[u]);
        Ct[u] = A + tp_off(k + 1 + ii[u], k + 1 + jj[u]);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[u][r] = Ct[u][(4 * r + q16) * 16 + l16];
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const double* Pi = pan + ii[u] * 256;
        const double* Pj = pan + jj[u] * 256;
        acc[u] = mma16_xyt([&](int i, int l) { return Pi[i * 16 + l]; },
                           [&](int j, int l) { return Pj[j * 16 + l]; }, acc[u], -1.0);
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        if (t0 + 4 * u >= nt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) Ct[u][(4 * r + q16) * 16 + l16] = acc[u][r];
      }
    }
    __syncthreads();
  }
  return 0;
}

// Lane-crossing moves of one FP64 value (two 32-bit halves each).
__device__ inline double lane_read64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// value of lane `src` (byte address 4 src)
__device__ inline double lane_perm64(int src4, double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src4, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src4, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// value of lane J of the lane's own 16-lane row (DPP row_newbcast:J)
template <int J>
__device__ inline double row_bcast64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x150 + J, 0xf, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x150 + J, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Factors the diagonal tile held in dg [256] (lower part used) in the
// registers of one wave: G_kk (upper part zero) to Akk and W_kk = G_kk^{-1}
// (row-major, upper part zero) to W.  Lane (c, q) = (lane % 16, lane / 16)
// holds rows 4 r + q (r < 4) of column c of the symmetric trailing matrix
// and of X, the right-hand side of G W = I being reduced alongside.  Step j
// of the right-looking elimination takes the pivot with a lane read,
// 1 / G_jj = rsqrt(pivot) by two Newton steps from the hardware estimate,
// the column-j entries of the lane's own rows with a broadcast inside each
// 16-lane row, and row j (of the trailing matrix and of X) with a permute
// from the row group that holds it; row j of W is then final and stored.
// Rows above the step hold values that are never read again.  Sets *s_bad
// to 1 + the first row whose pivot was not positive.  CM: dg and W are
// stored column-major (element (r, c) at 16 c + r), else row-major; Akk is
// row-major.
template <bool CM = false>
__device__ inline void diag_factor64(const double* dg, double* __restrict__ Akk,
                                     double* __restrict__ W, int row0, int* s_bad) {
  auto ix = [](int r, int cc) { return CM ? cc * 16 + r : r * 16 + cc; };
  // the lane-dependent selects below stay inside the call (hoisting them out
  // of a caller's step loop would hold dozens of scalar masks live)
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int c = lane & 15, q = lane >> 4;
  double a[4], x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * r + q;
    a[r] = dg[c <= i ? ix(i, c) : ix(c, i)];
    x[r] = i == c ? 1.0 : 0.0;
  }
  double my_rinv = 0.0;  // 1 / G_cc
  int bad = 0;
#define IVX_DF64_STEP(j)                                                            \
  {                                                                                 \
    const double piv = lane_read64(a[(j) >> 2], 16 * ((j) & 3) + (j));              \
    if (!(piv > 0.0) || !isfinite(piv)) {                                           \
      bad = (j) + 1;                                                                \
      goto done;                                                                    \
    }                                                                               \
    double ri = __builtin_amdgcn_rsq(piv);                                          \
    ri = fma(0.5 * ri, fma(-piv * ri, ri, 1.0), ri);                                \
    ri = fma(0.5 * ri, fma(-piv * ri, ri, 1.0), ri);                                \
    const double ri2 = ri * ri;                                                     \
    my_rinv = c == (j) ? ri : my_rinv;                                              \
    const int src4 = (16 * ((j) & 3) + c) * 4;                                      \
    const double ajc = lane_perm64(src4, a[(j) >> 2]);                              \
    const double xjc = lane_perm64(src4, x[(j) >> 2]);                              \
    if (q == ((j) & 3)) W[ix((j), c)] = x[(j) >> 2] * ri;                           \
    const double t = c > (j) ? ajc * ri2 : 0.0;                                     \
    const double u = xjc * ri2;                                                     \
    _Pragma("unroll") for (int r = 0; r < 4; ++r) {                                 \
      const double d = row_bcast64<(j)>(a[r]);                                      \
      a[r] = fma(-d, t, a[r]);                                                      \
      x[r] = fma(-d, u, x[r]);                                                      \
    }                                                                               \
  }
  IVX_DF64_STEP(0) IVX_DF64_STEP(1) IVX_DF64_STEP(2) IVX_DF64_STEP(3)
  IVX_DF64_STEP(4) IVX_DF64_STEP(5) IVX_DF64_STEP(6) IVX_DF64_STEP(7)
  IVX_DF64_STEP(8) IVX_DF64_STEP(9) IVX_DF64_STEP(10) IVX_DF64_STEP(11)
  IVX_DF64_STEP(12) IVX_DF64_STEP(13) IVX_DF64_STEP(14) IVX_DF64_STEP(15)
#undef IVX_DF64_STEP
done:
  if (bad) {
    if (lane == 0) *s_bad = row0 + bad;
    return;
  }
  // column c of the trailing matrix at step c is G_ic G_cc for i >= c
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * r + q;
    Akk[i * 16 + c] = i >= c ? a[r] * my_rinv : 0.0;
  }
}

// Left-looking blocked Cholesky A = G G^T with the same contract as
// chol_tp64 (lower tiles in place, W_k = G_kk^{-1} to Winv[k * 256]).  Block
// column k is formed in LDS from the finished columns j < k,
// A_(k+i),k - sum_j G_(k+i),j G_k,j^T on MFMA (each wave two tile rows with
// independent accumulators, the next j's tiles requested before the current
// MFMAs), then its diagonal tile is factored and inverted and the rest
// multiplied by that inverse; the column is written once.  A finished tile
// is read once for every later block column it feeds and never rewritten,
// where the right-looking form reads and writes every trailing tile at each
// step.  LDS: dg [256], pan [nb * 256].
__device__ inline int chol_ll64(double* __restrict__ A, int nb, double* __restrict__ Winv,
                                double* dg, double* pan, int* s_bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int eo = l16 * 16 + q16;  // element (l16, 4 q + q16) is at eo + 4 q
  if (tid == 0) *s_bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const int m1 = nb - k;  // tiles of block column k, the diagonal one first
    for (int it0 = wave; it0 < m1; it0 += 8) {
      const int itA = it0, itB = it0 + 4 < m1 ? it0 + 4 : it0;
      const double* At = A + tp_off(k + itA, k);
      const double* Bt = A + tp_off(k + itB, k);
      doublex4 accA, accB;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accA[r] = At[(4 * r + q16) * 16 + l16];
        accB[r] = Bt[(4 * r + q16) * 16 + l16];
      }
      double ck[4], ca[4], cb[4], nk[4], na[4], nb4[4];
      auto load = [&](int j, double (&gk)[4], double (&ga)[4], double (&gb)[4]) {
        const double* Gk = A + tp_off(k, j);
        const double* Ga = A + tp_off(k + itA, j);
        const double* Gb = A + tp_off(k + itB, j);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          gk[q] = Gk[eo + 4 * q];
          ga[q] = Ga[eo + 4 * q];
          gb[q] = Gb[eo + 4 * q];
        }
      };
      if (k > 0) load(0, ck, ca, cb);
      for (int j = 0; j < k; ++j) {
        if (j + 1 < k) load(j + 1, nk, na, nb4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          accA = __builtin_amdgcn_mfma_f64_16x16x4f64(-ca[q], ck[q], accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f64_16x16x4f64(-cb[q], ck[q], accB, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ck[q] = nk[q];
          ca[q] = na[q];
          cb[q] = nb4[q];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pan[itA * 256 + (4 * r + q16) * 16 + l16] = accA[r];
        if (itB != itA) pan[itB * 256 + (4 * r + q16) * 16 + l16] = accB[r];
      }
    }
    __syncthreads();
    if (wave == 0) {
      for (int e = lane; e < 256; e += 64) dg[e] = pan[e];
      __builtin_amdgcn_wave_barrier();
      diag_factor64(dg, A + tp_off(k, k), Winv + k * 256, k * 16, s_bad);
    }
    __syncthreads();
    if (*s_bad) return *s_bad;
    const double* W = Winv + k * 256;
    // panel: G_(k+i),k = pan_i W_kk^T, written once
    for (int it = 1 + wave; it < m1; it += 4) {
      const double* Pt = pan + it * 256;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return Pt[i * 16 + l]; },
                      [&](int j, int l) { return W[j * 16 + l]; }, acc, 1.0);
      double* Gt = A + tp_off(k + it, k);
#pragma unroll
      for (int r = 0; r < 4; ++r) Gt[(4 * r + q16) * 16 + l16] = acc[r];
    }
    __syncthreads();
  }
  return 0;
}

// Solves (G G^T) X = B in place for B of nrow (<= nb * 16) rows and ncol
// (<= 64) columns, element (r, d) at B[d * ldb + r]; rows >= nrow and
// columns >= ncol are treated as zero and never written.  G and Winv come
// from chol_tp64.  LDS: zb [16 * 64].
__device__ inline void solve_tp64(const double* __restrict__ G, const double* __restrict__ Winv,
                                  int nb, double* __restrict__ B, int64_t ldb, int nrow, int ncol,
                                  double* zb) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  auto bat = [&](int r, int d) -> double {
    return (r < nrow && d < ncol) ? B[(int64_t)d * ldb + r] : 0.0;
  };
  // forward: G Z = B
  for (int k = 0; k < nb; ++k) {
    const double* W = Winv + k * 256;
    {  // Z_k = W_k B_k, column block `wave`
      const int d0 = wave * 16;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return W[i * 16 + l]; },
                      [&](int j, int l) { return bat(k * 16 + l, d0 + j); }, acc, 1.0);
#pragma unroll
      for (int r = 0; r < 4; ++r) zb[(4 * r + q16) * 64 + d0 + l16] = acc[r];
    }
    __syncthreads();
    {
      const int d0 = wave * 16;
      for (int r = 0; r < 4; ++r) {
        const int row = k * 16 + 4 * r + q16, d = d0 + l16;
        if (row < nrow && d < ncol) B[(int64_t)d * ldb + row] = zb[(4 * r + q16) * 64 + d];
      }
    }
    // B_i -= G_ik Z_k for i > k (UT tiles per wave and pass, loads first)
    const int m = nb - k - 1;
    for (int w0 = wave; w0 < 4 * m; w0 += 4 * UT) {
      doublex4 acc[UT];
      double gv[UT][4];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u < 4 * m ? w0 + 4 * u : w0;
        const int it = k + 1 + (w >> 2), d0 = (w & 3) * 16;
        const double* Gt = G + tp_off(it, k);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[u][r] = bat(it * 16 + 4 * r + q16, d0 + l16);
#pragma unroll
        for (int q = 0; q < 4; ++q) gv[u][q] = Gt[l16 * 16 + 4 * q + q16];
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u < 4 * m ? w0 + 4 * u : w0;
        const int d0 = (w & 3) * 16;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-gv[u][q], zb[(4 * q + q16) * 64 + d0 + l16],
                                                        acc[u], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u;
        if (w >= 4 * m) break;
        const int it = k + 1 + (w >> 2), d0 = (w & 3) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = it * 16 + 4 * r + q16, d = d0 + l16;
          if (row < nrow && d < ncol) B[(int64_t)d * ldb + row] = acc[u][r];
        }
      }
    }
    __syncthreads();
  }
  // backward: G^T X = Z
  for (int k = nb - 1; k >= 0; --k) {
    const double* W = Winv + k * 256;
    {  // X_k = W_k^T Z_k
      const int d0 = wave * 16;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return W[l * 16 + i]; },
                      [&](int j, int l) { return bat(k * 16 + l, d0 + j); }, acc, 1.0);
#pragma unroll
      for (int r = 0; r < 4; ++r) zb[(4 * r + q16) * 64 + d0 + l16] = acc[r];
    }
    __syncthreads();
    {
      const int d0 = wave * 16;
      for (int r = 0; r < 4; ++r) {
        const int row = k * 16 + 4 * r + q16, d = d0 + l16;
        if (row < nrow && d < ncol) B[(int64_t)d * ldb + row] = zb[(4 * r + q16) * 64 + d];
      }
    }
    // Z_i -= G_ki^T X_k for i < k (UT tiles per wave and pass, loads first)
    for (int w0 = wave; w0 < 4 * k; w0 += 4 * UT) {
      doublex4 acc[UT];
      double gv[UT][4];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u < 4 * k ? w0 + 4 * u : w0;
        const int it = w >> 2, d0 = (w & 3) * 16;
        const double* Gt = G + tp_off(k, it);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[u][r] = bat(it * 16 + 4 * r + q16, d0 + l16);
#pragma unroll
        for (int q = 0; q < 4; ++q) gv[u][q] = Gt[(4 * q + q16) * 16 + l16];
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u < 4 * k ? w0 + 4 * u : w0;
        const int d0 = (w & 3) * 16;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-gv[u][q], zb[(4 * q + q16) * 64 + d0 + l16],
                                                        acc[u], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int w = w0 + 4 * u;
        if (w >= 4 * k) break;
        const int it = w >> 2, d0 = (w & 3) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = it * 16 + 4 * r + q16, d = d0 + l16;
          if (row < nrow && d < ncol) B[(int64_t)d * ldb + row] = acc[u][r];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace ivx
