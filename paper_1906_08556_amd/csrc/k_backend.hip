// Scoring back-end of Sec. 4.1 on the GPU: centring / whitening / length
// normalisation, class scatter, LDA, two-covariance PLDA and trial scoring.
//
//  k_class_sums      per-class sums and counts (FP64 atomics)
//  gemm64_tn         second moment X^T X (FP64 MFMA, k_gemm64.hip)
//  k_scatter         Sw, Sb (divisor N) from the second moment and class sums
//  k_jacobi_rows/cols  symmetric eigendecomposition by cyclic Jacobi with
//                    round-robin ordering: n/2 disjoint rotations per step,
//                    rows (one workgroup per pair) then columns and
//                    eigenvectors (one workgroup per row); the host checks
//                    the off-diagonal norm after every sweep
//  k_dgemm           small FP64 products (n <= 512) through LDS tiles
//  k_lnorm           y = W (x - mean) scaled to unit length, one wave per row
//  k_plda_score      llr of (z1, z2) in the space where W = I and B = diag(psi)
#include <algorithm>
#include <cmath>

#include "ivx_backend.h"

namespace ivx {
namespace {

__global__ void __launch_bounds__(256)
k_class_sums(const float* __restrict__ X, int64_t n, int dim, const int* __restrict__ labels,
             int K, double* __restrict__ sums, double* __restrict__ counts,
             int* __restrict__ bad) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int k = labels ? labels[i] : 0;
  if (k < 0 || k >= K) {
    if (threadIdx.x == 0) atomicAdd(bad, 1);
    return;
  }
  for (int d = threadIdx.x; d < dim; d += blockDim.x)
    atomicAdd(&sums[(size_t)k * dim + d], (double)X[i * dim + d]);
  if (threadIdx.x == 0) atomicAdd(&counts[k], 1.0);
}

// Sw = (M2 - G) / N, Sb = (G - N m m^T) / N with G = sum_k s_k s_k^T / n_k and
// m = sum_k s_k / N (classes without members contribute nothing).
__global__ void __launch_bounds__(256)
k_scatter(const double* __restrict__ M2, const double* __restrict__ sums,
          const double* __restrict__ counts, int K, int dim, double* __restrict__ Sw,
          double* __restrict__ Sb, double* __restrict__ mean) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)dim * dim) return;
  const int i = (int)(e / dim), j = (int)(e - (int64_t)i * dim);
  double G = 0.0, si = 0.0, sj = 0.0, N = 0.0;
  for (int k = 0; k < K; ++k) {
    const double nk = counts[k];
    if (nk <= 0.0) continue;
    const double a = sums[(size_t)k * dim + i], b = sums[(size_t)k * dim + j];
    G += a * b / nk;
    si += a;
    sj += b;
    N += nk;
  }
  const double mi = si / N, mj = sj / N;
  Sw[e] = (M2[e] - G) / N;
  Sb[e] = (G - N * mi * mj) / N;
  if (i == j && mean) mean[i] = mi;
}

// Round-robin pairing of n (even) indices, step r in [0, n-1): pair 0 is
// (n-1, r); pair k >= 1 is ((r + k) mod (n-1), (r - k) mod (n-1)).
__device__ inline void rr_pair(int n, int r, int k, int& p, int& q) {
  const int m = n - 1;
  if (k == 0) {
    p = r;
    q = m;
  } else {
    p = (r + k) % m;
    q = (r - k + m) % m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// One step of the cyclic Jacobi method on the symmetric A [n][n] (n even):
// the n/2 disjoint pairs of round-robin step r rotate at once,
// A <- J^T A J, V <- V J.  k_jacobi_rows: one workgroup per pair computes its
// rotation from the 2 x 2 block, stores it, and applies J^T to rows p and q.
// k_jacobi_cols: one workgroup per row i applies every pair's rotation to
// columns p and q of A and V.
__global__ void __launch_bounds__(256)
k_jacobi_rows(double* __restrict__ A, int n, int r, double2* __restrict__ rot) {
  __shared__ double s_c, s_s;
  int p, q;
  rr_pair(n, r, blockIdx.x, p, q);
  if (threadIdx.x == 0) {
    const double apq = A[(size_t)p * n + q];
    double c = 1.0, t = 0.0;
    if (apq != 0.0) {
      const double theta = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
      t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      c = 1.0 / sqrt(t * t + 1.0);
    }
    s_c = c;
    s_s = t * c;
    rot[blockIdx.x] = make_double2(c, t * c);
  }
  __syncthreads();
  const double c = s_c, sv = s_s;
  if (sv == 0.0) return;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double ap = A[(size_t)p * n + j], aq = A[(size_t)q * n + j];
    A[(size_t)p * n + j] = c * ap - sv * aq;
    A[(size_t)q * n + j] = sv * ap + c * aq;
  }
}

__global__ void __launch_bounds__(256)
k_jacobi_cols(double* __restrict__ A, double* __restrict__ V, int n, int r,
              const double2* __restrict__ rot) {
  const int i = blockIdx.x;
  for (int k = threadIdx.x; k < n / 2; k += 256) {
    const double2 cs = rot[k];
    if (cs.y == 0.0) continue;
    int p, q;
    rr_pair(n, r, k, p, q);
    double* a = A + (size_t)i * n;
    const double ap = a[p], aq = a[q];
    a[p] = cs.x * ap - cs.y * aq;
    a[q] = cs.y * ap + cs.x * aq;
    double* v = V + (size_t)i * n;
    const double vp = v[p], vq = v[q];
    v[p] = cs.x * vp - cs.y * vq;
    v[q] = cs.y * vp + cs.x * vq;
  }
}

// part[b] = partial sums of the squared off-diagonal (and, with diag, all)
// entries of A [n][n]; one value per workgroup, two slots per workgroup.
__global__ void __launch_bounds__(256)
k_offnorm_part(const double* __restrict__ A, int n, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * 256) {
    const double v = A[e] * A[e];
    all += v;
    if (e / n != e % n) off += v;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_eye_diag(double* __restrict__ V, int n, const double* __restrict__ A,
                           double* __restrict__ w, int mode) {
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * 256) {
    if (mode == 0)
      V[e] = (e / n == e % n) ? 1.0 : 0.0;
    else if (e < n)
      w[e] = A[e * n + e];
  }
}

// C[M][N] = sum_k op(A)[m][k] op(B)[k][n] - colsub[n], FP64 sums, 16 x 16 tiles.
// op(A)[m][k] = A[m*lda + k] (ta = 0) or A[k*lda + m] (ta = 1); same for B.
template <typename TA>
__global__ void __launch_bounds__(256)
k_dgemm(const TA* __restrict__ A, int64_t lda, int ta, const double* __restrict__ B, int64_t ldb,
        int tb, void* __restrict__ Cv, int64_t ldc, int c_float, int M, int N, int K,
        const double* __restrict__ colsub) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t m = (int64_t)blockIdx.y * 16 + ty;
  const int nn = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int64_t mm = (int64_t)blockIdx.y * 16 + ty;
      const int kk = k0 + tx;
      double v = 0.0;
      if (mm < M && kk < K) v = (double)(ta ? A[(int64_t)kk * lda + mm] : A[mm * lda + kk]);
      As[ty][tx] = v;
      const int kb = k0 + ty, nb = blockIdx.x * 16 + tx;
      double u = 0.0;
      if (kb < K && nb < N) u = tb ? B[(int64_t)nb * ldb + kb] : B[(int64_t)kb * ldb + nb];
      Bs[ty][tx] = u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  if (m < M && nn < N) {
    if (colsub) acc -= colsub[nn];
    if (c_float)
      static_cast<float*>(Cv)[m * ldc + nn] = (float)acc;
    else
      static_cast<double*>(Cv)[m * ldc + nn] = acc;
  }
}

// Wh[:, j] = Q[:, j] / sqrt(lam_j) for the columns j < dim of Q [ld][ld]
// (trans: stored transposed, Wh[j][i]); an eigenvalue <= floor * max makes
// the matrix singular: flagged.
__global__ void __launch_bounds__(256)
k_whiten_cols(const double* __restrict__ Q, int ld, const double* __restrict__ lam, int dim,
              double floor_rel, int trans, double* __restrict__ Wh, int* __restrict__ bad) {
  __shared__ double s_max;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < dim; ++j) mx = fmax(mx, lam[j]);
    s_max = mx;
  }
  __syncthreads();
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < (int64_t)dim * dim;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / dim), j = (int)(e - (int64_t)i * dim);
    const double l = lam[j];
    const int64_t o = trans ? (int64_t)j * dim + i : e;
    if (!(l > floor_rel * s_max)) {
      if (i == 0) atomicAdd(bad, 1);
      Wh[o] = 0.0;
    } else {
      Wh[o] = Q[(size_t)i * ld + j] / sqrt(l);
    }
  }
}

// Ranks of w [n] in decreasing order (ties: lower index first); idx[rank] = i
// for the first `keep` ranks, among the first `valid` entries only.
__global__ void __launch_bounds__(256)
k_rank_desc(const double* __restrict__ w, int valid, int keep, int* __restrict__ idx) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < valid; i += gridDim.x * 256) {
    const double v = w[i];
    int r = 0;
    for (int j = 0; j < valid; ++j) r += (w[j] > v) || (w[j] == v && j < i);
    if (r < keep) idx[r] = i;
  }
}

// out[i][r] = src[i][idx[r]] (i < rows, r < keep), FP64; vals[r] = w[idx[r]]
__global__ void __launch_bounds__(256)
k_gather_cols(const double* __restrict__ src, int ld, const int* __restrict__ idx, int rows,
              int keep, const double* __restrict__ w, double* __restrict__ out,
              double* __restrict__ vals) {
  const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (e < (int64_t)rows * keep) {
    const int i = (int)(e / keep), r = (int)(e - (int64_t)i * keep);
    out[e] = src[(size_t)i * ld + idx[r]];
  }
  if (vals && e < keep) vals[e] = w[idx[e]];
}

// y = W (x - mean) (W optional) scaled to unit length; one wave per row,
// four rows per workgroup, the centred and whitened rows staged in LDS.
constexpr int LN_MAX = 512;
__global__ void __launch_bounds__(256)
k_lnorm(const float* __restrict__ X, int64_t n, int dim, const double* __restrict__ mean,
        const double* __restrict__ W, float* __restrict__ Y) {
  __shared__ double t[4][LN_MAX];
  __shared__ double y[4][LN_MAX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wv;
  const bool active = row < n;
  if (active)
    for (int d = lane; d < dim; d += 64)
      t[wv][d] = (double)X[row * dim + d] - (mean ? mean[d] : 0.0);
  __syncthreads();
  double ss = 0.0;
  if (active) {
    for (int i = lane; i < dim; i += 64) {
      double a = t[wv][i];
      if (W) {
        const double* wi = W + (size_t)i * dim;
        a = 0.0;
        for (int d = 0; d < dim; ++d) a += wi[d] * t[wv][d];
      }
      y[wv][i] = a;
      ss += a * a;
    }
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
  if (active) {
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    for (int i = lane; i < dim; i += 64) Y[row * dim + i] = (float)(y[wv][i] * inv);
  }
}

// Per-dimension PLDA score coefficients from psi (between-speaker variances
// in the space where the within-speaker covariance is I): with s = psi + 1,
// det = s^2 - psi^2:  a = -(s / det - 1 / s) / 2,  b = psi / det,
// c = sum (-log(det) / 2 + log s).
__global__ void __launch_bounds__(256)
k_plda_coef(const double* __restrict__ psi, int d, double* __restrict__ coef) {
  __shared__ double red[256];
  double c = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double p = fmax(psi[i], 0.0), s = p + 1.0, det = s * s - p * p;
    coef[i] = -0.5 * (s / det - 1.0 / s);
    coef[d + i] = p / det;
    c += -0.5 * log(det) + log(s);
  }
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) coef[2 * d] = red[0];
}

// scores[t] = c + sum_i a_i (z1_i^2 + z2_i^2) + b_i z1_i z2_i for the pair
// (Z1[trials[2t]], Z2[trials[2t+1]]); one wave per trial.
__global__ void __launch_bounds__(256)
k_plda_score(const float* __restrict__ Z1, int64_t n1, const float* __restrict__ Z2, int64_t n2,
             int d, const double* __restrict__ coef, const int* __restrict__ trials, int64_t T,
             float* __restrict__ scores, int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  const int i = trials[2 * t], j = trials[2 * t + 1];
  if (i < 0 || i >= n1 || j < 0 || j >= n2) {
    if (lane == 0) {
      atomicAdd(bad, 1);
      scores[t] = NAN;
    }
    return;
  }
  const float* z1 = Z1 + (int64_t)i * d;
  const float* z2 = Z2 + (int64_t)j * d;
  double s = 0.0;
  for (int k = lane; k < d; k += 64) {
    const double a = z1[k], b = z2[k];
    s += coef[k] * (a * a + b * b) + coef[d + k] * a * b;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) scores[t] = (float)(s + coef[2 * d]);
}

// dst [n][n] = the symmetric part of src [dim][dim], zero-padded to n >= dim
__global__ void __launch_bounds__(256)
k_pad_sym(const double* __restrict__ src, int dim, double* __restrict__ dst, int n) {
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    dst[e] = (i < dim && j < dim) ? 0.5 * (src[(size_t)i * dim + j] + src[(size_t)j * dim + i])
                                  : 0.0;
  }
}

__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

// ------------------------------------------------------------------ launchers

void be_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill_zero<<<(unsigned)nb, 256, 0, s>>>(p, n);
}

void be_class_sums(const float* X, int64_t n, int dim, const int* labels, int K, double* sums,
                   double* counts, int* bad, hipStream_t s) {
  if (n > 0) k_class_sums<<<(unsigned)n, 128, 0, s>>>(X, n, dim, labels, K, sums, counts, bad);
}

void be_scatter(const double* M2, const double* sums, const double* counts, int K, int dim,
                double* Sw, double* Sb, double* mean, hipStream_t s) {
  const int64_t e = (int64_t)dim * dim;
  k_scatter<<<(unsigned)((e + 255) / 256), 256, 0, s>>>(M2, sums, counts, K, dim, Sw, Sb, mean);
}

constexpr int kOffParts = 64;

int be_jacobi(double* A, double* V, int n, int max_sweeps, double tol, double* w, double2* rot,
              double* part, hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  const unsigned gb = (unsigned)std::min<int64_t>((nn + 255) / 256, 1024);
  k_eye_diag<<<gb, 256, 0, s>>>(V, n, A, w, 0);
  double host[2 * kOffParts];
  double fro = -1.0;
  int sweep = 0;
  for (;; ++sweep) {
    k_offnorm_part<<<kOffParts, 256, 0, s>>>(A, n, part);
    if (hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return -1;
    double off = 0.0, all = 0.0;
    for (int b = 0; b < kOffParts; ++b) {
      off += host[2 * b];
      all += host[2 * b + 1];
    }
    if (fro < 0.0) fro = std::sqrt(all);
    if (!(std::sqrt(off) > tol * fro)) break;
    if (sweep >= max_sweeps) return -2;
    for (int r = 0; r < n - 1; ++r) {
      k_jacobi_rows<<<n / 2, 256, 0, s>>>(A, n, r, rot);
      k_jacobi_cols<<<n, 256, 0, s>>>(A, V, n, r, rot);
    }
  }
  k_eye_diag<<<1, 256, 0, s>>>(V, n, A, w, 1);
  return sweep;
}

void be_dgemm(const void* A, bool a_float, int64_t lda, bool ta, const double* B, int64_t ldb,
              bool tb, void* C, int64_t ldc, bool c_float, int M, int N, int K,
              const double* colsub, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16));
  if (a_float)
    k_dgemm<float><<<grid, 256, 0, s>>>(static_cast<const float*>(A), lda, ta, B, ldb, tb, C, ldc,
                                       c_float, M, N, K, colsub);
  else
    k_dgemm<double><<<grid, 256, 0, s>>>(static_cast<const double*>(A), lda, ta, B, ldb, tb, C,
                                        ldc, c_float, M, N, K, colsub);
}

void be_whiten_cols(const double* Q, int ld, const double* lam, int dim, double floor_rel,
                    bool trans, double* Wh, int* bad, hipStream_t s) {
  const int64_t e = (int64_t)dim * dim;
  int64_t nb = (e + 255) / 256;
  if (nb > 1024) nb = 1024;
  k_whiten_cols<<<(unsigned)nb, 256, 0, s>>>(Q, ld, lam, dim, floor_rel, trans ? 1 : 0, Wh, bad);
}

void be_pad_sym(const double* src, int dim, double* dst, int n, hipStream_t s) {
  const int64_t e = (int64_t)n * n;
  int64_t nb = (e + 255) / 256;
  if (nb > 1024) nb = 1024;
  k_pad_sym<<<(unsigned)nb, 256, 0, s>>>(src, dim, dst, n);
}

void be_rank_desc(const double* w, int valid, int keep, int* idx, hipStream_t s) {
  k_rank_desc<<<(unsigned)((valid + 255) / 256), 256, 0, s>>>(w, valid, keep, idx);
}

void be_gather_cols(const double* src, int ld, const int* idx, int rows, int keep,
                    const double* w, double* out, double* vals, hipStream_t s) {
  const int64_t e = (int64_t)rows * keep;
  k_gather_cols<<<(unsigned)((e + 255) / 256), 256, 0, s>>>(src, ld, idx, rows, keep, w, out,
                                                            vals);
}

void be_lnorm(const float* X, int64_t n, int dim, const double* mean, const double* W, float* Y,
              hipStream_t s) {
  if (n > 0) k_lnorm<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(X, n, dim, mean, W, Y);
}

void be_plda_coef(const double* psi, int d, double* coef, hipStream_t s) {
  k_plda_coef<<<1, 256, 0, s>>>(psi, d, coef);
}

void be_plda_score(const float* Z1, int64_t n1, const float* Z2, int64_t n2, int d,
                   const double* coef, const int* trials, int64_t T, float* scores, int* bad,
                   hipStream_t s) {
  if (T > 0)
    k_plda_score<<<(unsigned)((T + 3) / 4), 256, 0, s>>>(Z1, n1, Z2, n2, d, coef, trials, T,
                                                         scores, bad);
}

}  // namespace ivx
