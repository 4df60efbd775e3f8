// M-step (factor-analysis EM cited in Sec. 2.1 / Sec. 3.2 step 3), the EM
// objective, and minimum-divergence re-estimation (eqs. (6)-(12)); FP64.
//
//  k_objective_parts  per component: N_c(-D/2 log 2pi - 1/2 log|Sigma_c|)
//                     - 1/2 tr(Sigma_c^{-1} S_c) at the incoming Sigma_c.
//  k_mstep_solve      per component: blocked Cholesky of A_c (tile-packed,
//                     in place), T_c^T = A_c^{-1} Cc_c^T by two blocked
//                     triangular solves (16 right-hand sides at a time), then
//                     Sigma_c = sym((S_c - T_c Cc_c^T) / N_c) kept only if it
//                     is positive definite.
//  k_mindiv_setup     one workgroup: G = H/U - (h/U)(h/U)^T = L_G L_G^T,
//                     g = L_G^{-1} h/U, Householder vector a, p = P2 g and
//                     M = P1^{-1} P2^{-1} = L_G P2.
//  k_apply_M          T_c <- T_c M for all c (FP64 GEMM, LDS tiles).
#include <cmath>

#include "ivx_internal.h"
#include "ivx_tv.h"

namespace ivx {
namespace {

constexpr double kLog2Pi = 1.8378770664093454836;
// Components with N_c below this (no frames: soft counts cluster at integer
// frame counts when posteriors are near one-hot) keep T_c and Sigma_c.
constexpr double kMinCount = 0.5;

__device__ inline int64_t tile_off(int bi, int bj) { return (int64_t)(bi * (bi + 1) / 2 + bj) * 256; }

__device__ inline int64_t packed_idx(int i, int j, int D) {  // i <= j, upper row by row
  return (int64_t)i * D - (int64_t)i * (i - 1) / 2 + (j - i);
}

__device__ inline void decode_tri(int t, int& ii, int& jj) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ii = i;
  jj = t - i * (i + 1) / 2;
}

__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256)
k_objective_parts(const double* __restrict__ N, const double* __restrict__ S,
                  const double* __restrict__ Psig, const double* __restrict__ logdet, int D,
                  double* __restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int Dp = D * (D + 1) / 2;
  double tr = 0.0;
  for (int e = threadIdx.x; e < D * D; e += 256) {
    const int i = e / D, j = e - i * D;
    const int a = i < j ? i : j, b = i < j ? j : i;
    tr += Psig[(size_t)c * D * D + e] * S[(size_t)c * Dp + packed_idx(a, b, D)];
  }
  tr = block_sum(tr, red);
  if (threadIdx.x == 0) part[c] = N[c] * (-0.5 * D * kLog2Pi - 0.5 * logdet[c]) - 0.5 * tr;
}

__global__ void __launch_bounds__(256)
k_objective_finish(const double* __restrict__ part, int C, const double* __restrict__ ll_sum,
                   double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int c = threadIdx.x; c < C; c += 256) s += part[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s + (ll_sum ? ll_sum[0] : 0.0);
}

// one workgroup per component
__global__ void __launch_bounds__(256)
k_mstep_solve(int C, int D, int R, int nb, int64_t TP, double* __restrict__ A,
              const double* __restrict__ Cc, const double* __restrict__ N,
              const double* __restrict__ S, int update_sigma, double* __restrict__ T,
              double* __restrict__ Sigma, int* __restrict__ status, int* __restrict__ err) {
  extern __shared__ double X[];  // max(nb*256, 2*D*D) doubles
  __shared__ double dg[256];
  __shared__ int s_bad;
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double Nc = N[c];
  if (!(Nc >= kMinCount)) {  // no data: keep T_c, Sigma_c
    if (tid == 0) status[c] = 1;
    return;
  }
  double* Ac = A + (int64_t)c * TP;
  if (tid == 0) s_bad = 0;
  // identity on the padded diagonal so the padding factors trivially
  for (int d = R + tid; d < nb * 16; d += 256) Ac[tile_off(d >> 4, d >> 4) + (d & 15) * 17] = 1.0;
  __syncthreads();

  // ---- blocked Cholesky of A_c
  for (int k = 0; k < nb; ++k) {
    if (wave == 0) {
      double* Akk = Ac + tile_off(k, k);
      for (int e = lane; e < 256; e += 64) dg[e] = Akk[e];
      __builtin_amdgcn_wave_barrier();
      for (int j = 0; j < 16; ++j) {
        const double piv = dg[j * 16 + j];
        if (!(piv > 0.0) || !isfinite(piv)) {
          if (lane == 0) s_bad = k * 16 + j + 1;
          break;
        }
        const double ljj = sqrt(piv);
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < 16) dg[lane * 16 + j] /= ljj;
        if (lane == j) dg[j * 16 + j] = ljj;
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < 256; e += 64) {
          const int i = e >> 4, cc = e & 15;
          if (cc > j && i >= cc) dg[e] -= dg[i * 16 + j] * dg[cc * 16 + j];
        }
        __builtin_amdgcn_wave_barrier();
      }
      for (int e = lane; e < 256; e += 64) {
        const int i = e >> 4, cc = e & 15;
        const double v = (cc <= i) ? dg[e] : 0.0;
        dg[e] = v;
        Akk[e] = v;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int m = nb - k - 1;
    for (int row = tid; row < m * 16; row += 256) {
      const int it = row >> 4, r = row & 15;
      double* src = Ac + tile_off(k + 1 + it, k) + r * 16;
      double x[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) x[cc] = src[cc];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double s = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) s -= x[l] * dg[j * 16 + l];
        x[j] = s / dg[j * 16 + j];
      }
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        src[cc] = x[cc];
        X[it * 256 + r * 16 + cc] = x[cc];
      }
    }
    __syncthreads();
    const int ntile = m * (m + 1) / 2;
    const int i = tid >> 4, j = tid & 15;
    for (int t = 0; t < ntile; ++t) {
      int ii, jj;
      decode_tri(t, ii, jj);
      const double* Pi = X + ii * 256;
      const double* Pj = X + jj * 256;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 16; ++l) s += Pi[i * 16 + l] * Pj[j * 16 + l];
      Ac[tile_off(k + 1 + ii, k + 1 + jj) + i * 16 + j] -= s;
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) {
      status[c] = 3;
      raise_error(err, IVX_ENOTPD, PK_MSTEP, c);
    }
    return;
  }

  // ---- T_c^T = A_c^{-1} Cc_c^T, 16 columns (feature dims) at a time
  const double* Ccc = Cc + (int64_t)c * D * R;
  double* Tc = T + (int64_t)c * D * R;
  for (int d0 = 0; d0 < D; d0 += 16) {
    for (int e = tid; e < nb * 256; e += 256) {
      const int r = e >> 4, jc = e & 15;
      X[e] = (r < R && d0 + jc < D) ? Ccc[(int64_t)(d0 + jc) * R + r] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {  // forward: G z = b
      if (tid < 16) {
        const double* Gkk = Ac + tile_off(k, k);
        const int jc = tid;
        for (int l = 0; l < 16; ++l) {
          double s = X[(k * 16 + l) * 16 + jc];
          for (int q = 0; q < l; ++q) s -= Gkk[l * 16 + q] * X[(k * 16 + q) * 16 + jc];
          X[(k * 16 + l) * 16 + jc] = s / Gkk[l * 16 + l];
        }
      }
      __syncthreads();
      for (int e = tid; e < (nb - k - 1) * 256; e += 256) {
        const int row = (k + 1) * 16 + (e >> 4), jc = e & 15;
        const double* G = Ac + tile_off(row >> 4, k) + (row & 15) * 16;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l) s += G[l] * X[(k * 16 + l) * 16 + jc];
        X[row * 16 + jc] -= s;
      }
      __syncthreads();
    }
    for (int k = nb - 1; k >= 0; --k) {  // backward: G^T x = z
      if (tid < 16) {
        const double* Gkk = Ac + tile_off(k, k);
        const int jc = tid;
        for (int l = 15; l >= 0; --l) {
          double s = X[(k * 16 + l) * 16 + jc];
          for (int q = l + 1; q < 16; ++q) s -= Gkk[q * 16 + l] * X[(k * 16 + q) * 16 + jc];
          X[(k * 16 + l) * 16 + jc] = s / Gkk[l * 16 + l];
        }
      }
      __syncthreads();
      for (int e = tid; e < k * 256; e += 256) {
        const int row = e >> 4, jc = e & 15;  // row in blocks < k
        const double* G = Ac + tile_off(k, row >> 4) + (row & 15);
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) s += G[r * 16] * X[(k * 16 + r) * 16 + jc];
        X[row * 16 + jc] -= s;
      }
      __syncthreads();
    }
    for (int e = tid; e < 16 * R; e += 256) {
      const int jc = e / R, r = e - jc * R;
      if (d0 + jc < D) Tc[(int64_t)(d0 + jc) * R + r] = X[r * 16 + jc];
    }
    __syncthreads();
  }
  if (!update_sigma) {
    if (tid == 0) status[c] = 0;
    return;
  }
  // ---- Sigma_c = sym((S_c - T_c Cc_c^T) / N_c), kept if positive definite
  const int Dp = D * (D + 1) / 2;
  double* Ms = X;          // [D][D] symmetric candidate
  double* Lc = X + D * D;  // [D][D] Cholesky scratch
  for (int e = tid; e < D * D; e += 256) {
    const int a = e / D, b = e - a * D;
    if (a > b) continue;
    double s1 = 0.0, s2 = 0.0;
    for (int r = 0; r < R; ++r) {
      s1 += Tc[(int64_t)a * R + r] * Ccc[(int64_t)b * R + r];
      s2 += Tc[(int64_t)b * R + r] * Ccc[(int64_t)a * R + r];
    }
    const double v = (S[(int64_t)c * Dp + packed_idx(a, b, D)] - 0.5 * (s1 + s2)) / Nc;
    Ms[a * D + b] = v;
    Ms[b * D + a] = v;
    Lc[a * D + b] = v;
    Lc[b * D + a] = v;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    const double djj = Lc[j * D + j];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (tid == 0) s_bad = 1;
      break;
    }
    const double ljj = sqrt(djj);
    __syncthreads();
    if (tid > j && tid < D) Lc[tid * D + j] /= ljj;
    if (tid == j) Lc[j * D + j] = ljj;
    __syncthreads();
    if (tid > j && tid < D) {
      const double lij = Lc[tid * D + j];
      for (int k = j + 1; k <= tid; ++k) Lc[tid * D + k] -= lij * Lc[k * D + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) status[c] = 2;
    return;
  }
  for (int e = tid; e < D * D; e += 256) Sigma[(int64_t)c * D * D + e] = Ms[e];
  if (tid == 0) status[c] = 0;
}

// Minimum-divergence set-up, one workgroup of 256 threads.
__global__ void __launch_bounds__(256)
k_mindiv_setup(int R, int nb, const double* __restrict__ hsum, const double* __restrict__ Htp,
               const double* __restrict__ count, double* __restrict__ G, double* __restrict__ M,
               double* __restrict__ vec, double* __restrict__ p, int* __restrict__ err) {
  __shared__ double red[256];
  __shared__ double sc[4];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const double U = count[0];
  double* hb = vec;         // h / U
  double* g = vec + R;      // L_G^{-1} h / U
  double* a = vec + 2 * R;  // Householder vector
  double* v = vec + 3 * R;  // L_G a
  for (int i = tid; i < R; i += 256) hb[i] = hsum[i] / U;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e - i * R;
    const int bi = i >> 4, bj = j >> 4;
    const double Hij = (bi >= bj) ? Htp[tile_off(bi, bj) + (i & 15) * 16 + (j & 15)]
                                  : Htp[tile_off(bj, bi) + (j & 15) * 16 + (i & 15)];
    G[e] = Hij / U - hb[i] * hb[j];
  }
  __syncthreads();
  // Cholesky of G (lower, in place), column by column
  for (int j = 0; j < R; ++j) {
    const double djj = G[(int64_t)j * R + j];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (tid == 0) bad = 1;
      break;
    }
    const double ljj = sqrt(djj);
    __syncthreads();
    for (int i = j + 1 + tid; i < R; i += 256) G[(int64_t)i * R + j] /= ljj;
    if (tid == 0) G[(int64_t)j * R + j] = ljj;
    __syncthreads();
    const int m = R - j - 1;
    const int64_t ne = (int64_t)m * (m + 1) / 2;
    for (int64_t e = tid; e < ne; e += 256) {
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while ((int64_t)ii * (ii + 1) / 2 > e) --ii;
      const int kk = (int)(e - (int64_t)ii * (ii + 1) / 2);
      const int row = j + 1 + ii, col = j + 1 + kk;
      G[(int64_t)row * R + col] -= G[(int64_t)row * R + j] * G[(int64_t)col * R + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {  // leave T and p unchanged: M = I
    if (tid == 0) raise_error(err, IVX_ENOTPD, PK_MINDIV);
    for (int e = tid; e < R * R; e += 256) M[e] = (e / R == e % R) ? 1.0 : 0.0;
    return;
  }
  // g = L^{-1} hb (forward substitution; the dot products are block reductions)
  for (int i = 0; i < R; ++i) {
    double s = 0.0;
    for (int k = tid; k < i; k += 256) s += G[(int64_t)i * R + k] * g[k];
    s = block_sum(s, red);
    if (tid == 0) g[i] = (hb[i] - s) / G[(int64_t)i * R + i];
    __syncthreads();
  }
  double s2 = 0.0;
  for (int i = 1 + tid; i < R; i += 256) s2 += g[i] * g[i];
  s2 = block_sum(s2, red);
  if (tid == 0) {
    const double tail = sqrt(s2);
    const double gn = sqrt(s2 + g[0] * g[0]);
    double alpha = 0.0;
    if (tail > 1e-12 * gn) {
      const double one_minus = (g[0] > 0.0) ? s2 / (gn * (gn + g[0])) : 1.0 - g[0] / gn;
      alpha = 1.0 / sqrt(2.0 * one_minus);
    }
    sc[0] = gn;
    sc[1] = alpha;
  }
  __syncthreads();
  const double gn = sc[0], alpha = sc[1];
  // a = alpha h~ + beta e_1, beta = -alpha (a = 0 means P2 = I)
  for (int i = tid; i < R; i += 256) a[i] = alpha * (g[i] / gn) - ((i == 0) ? alpha : 0.0);
  __syncthreads();
  // p = P2 g = g - 2 a (a^T g);  v = L a
  double ag = 0.0;
  for (int i = tid; i < R; i += 256) ag += a[i] * g[i];
  ag = block_sum(ag, red);
  for (int i = tid; i < R; i += 256) {
    p[i] = g[i] - 2.0 * a[i] * ag;
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += G[(int64_t)i * R + k] * a[k];
    v[i] = s;
  }
  __syncthreads();
  // M = L_G P2 = L_G - 2 (L_G a) a^T
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e - i * R;
    M[e] = ((j <= i) ? G[e] : 0.0) - 2.0 * v[i] * a[j];
  }
}

// Tn[rows x R] = T[rows x R] * M[R x R], 64 x 64 tiles, 4 x 4 outputs per thread
__global__ void __launch_bounds__(256)
k_apply_M(const double* __restrict__ T, const double* __restrict__ M, int64_t rows, int R,
          double* __restrict__ Tn) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int c0 = blockIdx.x * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < R; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int rr = e >> 4, kk = e & 15;
      const int64_t row = r0 + rr;
      As[kk][rr] = (row < rows && k0 + kk < R) ? T[row * R + k0 + kk] : 0.0;
      const int k2 = e >> 6, cc = e & 63;
      Bs[k2][cc] = (k0 + k2 < R && c0 + cc < R) ? M[(int64_t)(k0 + k2) * R + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = r0 + ty * 4 + i;
    if (row >= rows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + tx * 4 + j;
      if (col < R) Tn[row * R + col] = acc[i][j];
    }
  }
}

}  // namespace

void launch_objective(ivx_ctx* ctx, const double* N, const double* S, const double* ll_sum,
                      double* objective, hipStream_t s) {
  k_objective_parts<<<ctx->C, 256, 0, s>>>(N, S, ctx->Psig, ctx->sig_logdet, ctx->D, ctx->obj_part);
  k_objective_finish<<<1, 256, 0, s>>>(ctx->obj_part, ctx->C, ll_sum, objective);
}

void launch_mstep_solve(ivx_ctx* ctx, const ivx_accum* acc, const double* S, int update_sigma,
                        int* status, hipStream_t s) {
  const int nb = (ctx->R + 15) / 16;
  size_t nx = (size_t)nb * 256;
  if ((size_t)2 * ctx->D * ctx->D > nx) nx = (size_t)2 * ctx->D * ctx->D;
  k_mstep_solve<<<ctx->C, 256, nx * sizeof(double), s>>>(ctx->C, ctx->D, ctx->R, nb, ctx->TP,
                                                         acc->A, acc->Cc, acc->N, S, update_sigma,
                                                         ctx->T, ctx->Sigma, status, ctx->dev_err);
}

void launch_mindiv(ivx_ctx* ctx, const ivx_accum* acc, hipStream_t s) {
  const int nb = (ctx->R + 15) / 16;
  k_mindiv_setup<<<1, 256, 0, s>>>(ctx->R, nb, acc->h, acc->H, acc->count, ctx->Gmat, ctx->Mmat,
                                   ctx->mvec, ctx->p, ctx->dev_err);
  const int64_t rows = (int64_t)ctx->C * ctx->D;
  dim3 grid((unsigned)((ctx->R + 63) / 64), (unsigned)((rows + 63) / 64));
  k_apply_M<<<grid, 256, 0, s>>>(ctx->T, ctx->Mmat, rows, ctx->R, ctx->Tnew);
  // copy back on the stream (no host-side pointer swap, so a captured graph
  // replays correctly)
  hipMemcpyAsync(ctx->T, ctx->Tnew, sizeof(double) * rows * ctx->R, hipMemcpyDeviceToDevice, s);
}

}  // namespace ivx
