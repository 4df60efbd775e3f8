// UBM preparation (FP64), TV initialisation and the realignment mean update.
//
// For every component c the frame log-likelihood is a quadratic form in the
// augmented feature x~ = [1, x - s] (s: a global mean shift):
//   log w_c N(x; mu_c, Sigma_c) = x~^T Q_c x~,
//   Q_c = [[g_c, b_c^T / 2], [b_c / 2, -P_c / 2]],  P_c = Sigma_c^{-1},
//   b_c = P_c (mu_c - s),  g_c = log w_c - D/2 log 2pi - 1/2 log|Sigma_c|
//                               - 1/2 (mu_c - s)^T P_c (mu_c - s).
// Written over the (D+1)(D+2)/2 products x~_a x~_b (a <= b) it is one dot
// product per (frame, component); W holds those coefficients (off-diagonal
// entries of Q doubled).  The exact rescoring uses L_c^{-1} and the constant
// log w_c - D/2 log 2pi - sum_i log L_c[i,i] with L_c = chol(Sigma_c).
#include <climits>
#include <cmath>

#include "ivx_internal.h"

namespace ivx {
namespace {

constexpr double kLog2Pi = 1.8378770664093454836;

__global__ void __launch_bounds__(64) k_ubm_shift(const double* __restrict__ w,
                                                  const double* __restrict__ mu, int C, int D,
                                                  float* __restrict__ shift) {
  const int d = threadIdx.x;
  if (d >= D) return;
  double s = 0.0, sw = 0.0;
  for (int c = 0; c < C; ++c) {
    s += w[c] * mu[(size_t)c * D + d];
    sw += w[c];
  }
  shift[d] = (float)(s / sw);
}

// One 64-thread workgroup per component (D <= 63).  LDS: L and L^{-1}, D x D
// doubles each.
__global__ void __launch_bounds__(64) k_ubm_prepare(
    const double* __restrict__ w, const double* __restrict__ mu, const double* __restrict__ cov,
    const float* __restrict__ shift, int C, int D, int K, int Kpad,
    const uint16_t* __restrict__ pairs, float* __restrict__ Wexp, __bf16* __restrict__ W16,
    double* __restrict__ linv_out, float* __restrict__ linv32r_out,
    double* __restrict__ cst_out, int* __restrict__ err) {
  extern __shared__ double sm[];
  double* A = sm;           // [D][D], becomes L (lower triangle)
  double* Li = sm + D * D;  // [D][D], L^{-1} (lower triangle)
  __shared__ double y[64], bv[64], red[64];
  __shared__ int bad;
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  // chunk-major layout: coefficient (c, k) at ((k / 8) * Cpad + c) * 8 + k % 8
  const int Cpad = gridDim.x;
  auto wat = [&](int k) -> float& { return Wexp[((size_t)(k >> 3) * Cpad + c) * 8 + (k & 7)]; };
  // BF16 copy, [Kpad/16][Cpad][32]: 16 high parts then 16 low parts per chunk
  auto put = [&](int k, float v) {
    wat(k) = v;
    const __bf16 hi = (__bf16)v;
    __bf16* q = W16 + ((size_t)(k >> 4) * Cpad + c) * 32;
    q[k & 15] = hi;
    q[16 + (k & 15)] = (__bf16)(v - (float)hi);
  };
  if (c >= C) {  // padding rows of the frame GEMM: never a candidate
    for (int k = t; k < Kpad; k += 64) put(k, (k == 0) ? -1e30f : 0.0f);
    return;
  }
  for (int i = t; i < D * D; i += 64) A[i] = cov[(size_t)c * D * D + i];
  if (t == 0) bad = 0;
  __syncthreads();
  // Cholesky, right-looking, one column per step
  for (int j = 0; j < D; ++j) {
    const double djj = A[j * D + j];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (t == 0) bad = 1;
      break;  // djj is read by every thread: uniform exit
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
      raise_error(err, IVX_ENOTPD, PK_UBM, c);
    }
    for (int k = t; k < Kpad; k += 64) put(k, (k == 0) ? -1e30f : 0.0f);
    if (t == 0) cst_out[c] = -INFINITY;
    return;
  }
  // L^{-1}: thread j owns column j (forward substitution)
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
  __syncthreads();
  // y = L^{-1}(mu - s),  b = L^{-T} y = P (mu - s)
  if (t < D) {
    double s = 0.0;
    for (int k = 0; k <= t; ++k) s += Li[t * D + k] * (mu[(size_t)c * D + k] - (double)shift[k]);
    y[t] = s;
  }
  __syncthreads();
  if (t < D) {
    double s = 0.0;
    for (int k = t; k < D; ++k) s += Li[k * D + t] * y[k];
    bv[t] = s;
  }
  red[t] = (t < D) ? (y[t] * y[t]) : 0.0;
  __syncthreads();
  if (t == 0) {
    double quad = 0.0, hld = 0.0;
    for (int i = 0; i < D; ++i) {
      quad += red[i];
      hld += log(A[i * D + i]);
    }
    const double base = log(w[c]) - 0.5 * D * kLog2Pi - hld;
    cst_out[c] = base;
    red[0] = base - 0.5 * quad;  // g_c
  }
  __syncthreads();
  const double g = red[0];
  // L^{-1} packed: column j holds rows j..D-1
  const int Dp = D * (D + 1) / 2;
  for (int j = 0; j < D; ++j) {
    const int col = j * D - j * (j - 1) / 2;
    if (t >= j && t < D) linv_out[(size_t)c * Dp + col + (t - j)] = Li[t * D + j];
  }
  // FP32 copy packed by rows (row i: columns 0..i) for the learned-selection filter
  for (int i = 0; i < D; ++i)
    if (t <= i) linv32r_out[(size_t)c * Dp + i * (i + 1) / 2 + t] = (float)Li[i * D + t];
  // expanded coefficients
  for (int k = t; k < Kpad; k += 64) {
    double v = 0.0;
    if (k < K) {
      const int pr = pairs[k];
      const int a = pr & 0xff, b = pr >> 8;
      if (a == 0 && b == 0) {
        v = g;
      } else if (a == 0) {
        v = bv[b - 1];
      } else {
        const int i = a - 1, jj = b - 1;
        double P = 0.0;
        for (int m = (i > jj ? i : jj); m < D; ++m) P += Li[m * D + i] * Li[m * D + jj];
        v = (i == jj) ? -0.5 * P : -P;
      }
    }
    put(k, (float)v);
  }
}

__global__ void k_init_tv(const double* __restrict__ T_rand, const double* __restrict__ mu,
                          const double* __restrict__ cov, double p0, int C, int D, int R,
                          double* __restrict__ T, double* __restrict__ Sigma,
                          double* __restrict__ p) {
  const int64_t nT = (int64_t)C * D * R, nS = (int64_t)C * D * D;
  const int64_t n = nT > nS ? nT : nS;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nT) T[i] = (i % R == 0) ? mu[i / R] / p0 : T_rand[i];
    if (i < nS) Sigma[i] = cov[i];
    if (i < R) p[i] = (i == 0) ? p0 : 0.0;
  }
}

// Standard initialisation (Sec. 2.1): T <- T_rand, Sigma <- UBM covariances,
// p <- 0, bias m <- UBM means (FP64 and its FP32 copy).
__global__ void k_init_tv_standard(const double* __restrict__ T_rand,
                                   const double* __restrict__ mu, const double* __restrict__ cov,
                                   int C, int D, int R, double* __restrict__ T,
                                   double* __restrict__ Sigma, double* __restrict__ p,
                                   double* __restrict__ bias, float* __restrict__ bias32) {
  const int64_t nT = (int64_t)C * D * R, nS = (int64_t)C * D * D;
  const int64_t n = nT > nS ? nT : nS;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nT) T[i] = T_rand[i];
    if (i < nS) Sigma[i] = cov[i];
    if (i < R) p[i] = 0.0;
    if (i < (int64_t)C * D) {
      bias[i] = mu[i];
      bias32[i] = (float)mu[i];
    }
  }
}

__global__ void k_bias32(const double* __restrict__ bias, int64_t n, float* __restrict__ bias32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bias32[i] = (float)bias[i];
}

// ldense[c][j][i] = L_c^-1[i][j] for j <= i < D, else 0 (dense column-major
// copy of the column-packed FP64 factor, for the sorted exact rescoring)
__global__ void k_linv_dense(const double* __restrict__ linv, int C, int D,
                             double* __restrict__ ldense) {
  const int Dp = D * (D + 1) / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)C * 4096;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e >> 12), j = (int)((e >> 6) & 63), i = (int)(e & 63);
    double v = 0.0;
    if (j < D && i < D && j <= i) v = linv[(size_t)c * Dp + j * D - j * (j - 1) / 2 + (i - j)];
    ldense[e] = v;
  }
}

__global__ void k_update_means(const double* __restrict__ T, const double* __restrict__ p, int C,
                               int D, int R, double* __restrict__ mu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < C * D) mu[i] = p[0] * T[(size_t)i * R];
}

}  // namespace

void launch_ubm_prepare(ivx_ctx* ctx, hipStream_t s) {
  k_ubm_shift<<<1, 64, 0, s>>>(ctx->w, ctx->mu, ctx->C, ctx->D, ctx->shift);
  const size_t lds = 2 * sizeof(double) * ctx->D * ctx->D;
  k_ubm_prepare<<<ctx->Cpad, 64, lds, s>>>(ctx->w, ctx->mu, ctx->cov, ctx->shift, ctx->C, ctx->D,
                                           ctx->K, ctx->Kpad, ctx->pairs, ctx->Wexp, ctx->W16,
                                           ctx->linv, ctx->linv32r, ctx->cst, ctx->dev_err);
  k_linv_dense<<<2048, 256, 0, s>>>(ctx->linv, ctx->C, ctx->D, ctx->ldense);
}

void launch_init_tv(ivx_ctx* ctx, const double* T_rand, double p0, hipStream_t s) {
  k_init_tv<<<1024, 256, 0, s>>>(T_rand, ctx->mu, ctx->cov, p0, ctx->C, ctx->D, ctx->R, ctx->T,
                                 ctx->Sigma, ctx->p);
}

void launch_init_tv_standard(ivx_ctx* ctx, const double* T_rand, hipStream_t s) {
  k_init_tv_standard<<<1024, 256, 0, s>>>(T_rand, ctx->mu, ctx->cov, ctx->C, ctx->D, ctx->R,
                                          ctx->T, ctx->Sigma, ctx->p, ctx->bias, ctx->bias32);
}

void launch_bias32(ivx_ctx* ctx, hipStream_t s) {
  const int64_t n = (int64_t)ctx->C * ctx->D;
  k_bias32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ctx->bias, n, ctx->bias32);
}

void launch_update_means(ivx_ctx* ctx, hipStream_t s) {
  const int n = ctx->C * ctx->D;
  k_update_means<<<(n + 255) / 256, 256, 0, s>>>(ctx->T, ctx->p, ctx->C, ctx->D, ctx->R, ctx->mu);
  launch_ubm_prepare(ctx, s);
}

}  // namespace ivx
