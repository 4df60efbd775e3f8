// M-step (factor-analysis EM cited in Sec. 2.1 / Sec. 3.2 step 3), the EM
// objective, and minimum-divergence re-estimation (eqs. (6)-(12)); FP64.
//
//  k_objective_parts  per component: N_c(-D/2 log 2pi - 1/2 log|Sigma_c|)
//                     - 1/2 tr(Sigma_c^{-1} S_c) at the incoming Sigma_c.
//  k_mstep_solve      per component: blocked Cholesky of A_c (tile-packed,
//                     in place, FP64 MFMA updates), T_c^T = A_c^{-1} Cc_c^T
//                     by two blocked triangular solves over all D right-hand
//                     sides, then Sigma_c = sym((S_c - T_c Cc_c^T) / N_c) kept
//                     only if it is positive definite.
//  k_mindiv_setup     one workgroup: G = H/U - (h/U)(h/U)^T = L_G L_G^T,
//                     g = L_G^{-1} h/U, Householder vector a, p = P2 g and
//                     M = P1^{-1} P2^{-1} = L_G P2.
//                     Standard formulation (Sec. 3.1): M = P1^{-1} = L_G
//                     alone, p stays 0.
//  k_bias_update      standard formulation, optional (Sec. 5):
//                     m_c <- m_c + T_c h/U with the T of the M-step.
//  k_apply_M          T_c <- T_c M for all c (FP64 MFMA GEMM, LDS tiles).
#include <cmath>

#include "ivx_internal.h"
#include "ivx_tv.h"
#include "k_chol64.h"

namespace ivx {
namespace {

constexpr double kLog2Pi = 1.8378770664093454836;
// Components with N_c below this (no frames: soft counts cluster at integer
// frame counts when posteriors are near one-hot) keep T_c and Sigma_c.
constexpr double kMinCount = 0.5;

__device__ inline int64_t packed_idx(int i, int j, int D) {  // i <= j, upper row by row
  return (int64_t)i * D - (int64_t)i * (i - 1) / 2 + (j - i);
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

// Sigma_c = sym((S_c - P) / N_c) with P = T_c Cc_c^T given in big[0..4096)
// ([64][64], row-major), stored only if it is positive definite (status 0;
// else status 2 and Sigma_c unchanged).  Called by all threads of the
// workgroup (any multiple of 64, at least D) after P is complete.  LDS: big
// [4096 + D * D].
__device__ __noinline__ void sigma_finish(int c, int D, double Nc, const double* __restrict__ S,
                                          double* __restrict__ Sigma, double* big, int* s_bad,
                                          int* __restrict__ status) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int l16 = lane & 15, q16 = lane >> 4, nt = blockDim.x;
  double* Cb = big;          // [64][64] T_c Cc_c^T
  double* Ms = big + 4096;   // [D][D] candidate
  const int Dp = D * (D + 1) / 2;
  for (int e = tid; e < D * D; e += nt) {
    const int a = e / D, b = e - a * D;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    Ms[e] = (S[(int64_t)c * Dp + packed_idx(lo, hi, D)] - 0.5 * (Cb[a * 64 + b] + Cb[b * 64 + a])) / Nc;
  }
  __syncthreads();
  // positive definiteness: blocked Cholesky of Ms on 16 x 16 tiles in LDS
  // (lower tiles, tile-packed, padded with the identity), the diagonal tiles
  // factored in one wave's registers, panels and updates on MFMA
  const int nbD = (D + 15) >> 4;  // <= 4
  double* Pt = Cb;                // [10][256]
  double* Wk = Cb + 10 * 256;     // [256] G_kk^{-1}
  double* Lk = Wk + 256;          // [256] G_kk (not needed further)
  for (int e = tid; e < nbD * (nbD + 1) / 2 * 256; e += nt) {
    const int t = e >> 8, w = e & 255;
    const int bi = t >= 6 ? 3 : t >= 3 ? 2 : t >= 1 ? 1 : 0, bj = t - bi * (bi + 1) / 2;
    const int i = bi * 16 + (w >> 4), j = bj * 16 + (w & 15);
    Pt[e] = (i < D && j < D) ? Ms[i * D + j] : (i == j ? 1.0 : 0.0);
  }
  if (tid == 0) *s_bad = 0;
  __syncthreads();
  for (int k = 0; k < nbD; ++k) {
    if (wave == 0) diag_factor64(Pt + tp_off(k, k), Lk, Wk, 16 * k, s_bad);
    __syncthreads();
    if (*s_bad) break;
    for (int it = k + 1 + wave; it < nbD; it += nw) {
      double* At = Pt + tp_off(it, k);
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return At[i * 16 + l]; },
                      [&](int j, int l) { return Wk[j * 16 + l]; }, acc, 1.0);
      __builtin_amdgcn_wave_barrier();  // the tile is read whole before it is replaced
#pragma unroll
      for (int r = 0; r < 4; ++r) At[(4 * r + q16) * 16 + l16] = acc[r];
    }
    __syncthreads();
    const int m = nbD - k - 1;
    for (int t = wave; t < m * (m + 1) / 2; t += nw) {
      int ii, jj;
      tri_decode(t, ii, jj);
      double* Ct = Pt + tp_off(k + 1 + ii, k + 1 + jj);
      const double* Pi = Pt + tp_off(k + 1 + ii, k);
      const double* Pj = Pt + tp_off(k + 1 + jj, k);
      doublex4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = Ct[(4 * r + q16) * 16 + l16];
      acc = mma16_xyt([&](int i, int l) { return Pi[i * 16 + l]; },
                      [&](int j, int l) { return Pj[j * 16 + l]; }, acc, -1.0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ct[(4 * r + q16) * 16 + l16] = acc[r];
    }
    __syncthreads();
  }
  __syncthreads();
  if (*s_bad) {
    if (tid == 0) status[c] = 2;
    return;
  }
  for (int e = tid; e < D * D; e += nt) Sigma[(int64_t)c * D * D + e] = Ms[e];
  if (tid == 0) status[c] = 0;
}

// The Sigma_c update after T_c has been written to device memory:
// T_c Cc_c^T on MFMA into big[0..4096), then sigma_finish.
__device__ __noinline__ void sigma_update(int c, int D, int R, double Nc, const double* __restrict__ Tc,
                             const double* __restrict__ Ccc, const double* __restrict__ S,
                             double* __restrict__ Sigma, double* big, int* s_bad,
                             int* __restrict__ status) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  double* Cb = big;          // [64][64] T_c Cc_c^T
  for (int t = wave; t < 16; t += nw) {
    const int ta = t >> 2, tb = t & 3;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < R; r0 += 16) {
      acc = mma16_xyt(
          [&](int i, int l) {
            const int a = ta * 16 + i, r = r0 + l;
            return (a < D && r < R) ? Tc[(int64_t)a * R + r] : 0.0;
          },
          [&](int j, int l) {
            const int b = tb * 16 + j, r = r0 + l;
            return (b < D && r < R) ? Ccc[(int64_t)b * R + r] : 0.0;
          },
          acc, 1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Cb[(ta * 16 + 4 * r + q16) * 64 + tb * 16 + l16] = acc[r];
  }
  __syncthreads();
  sigma_finish(c, D, Nc, S, Sigma, big, s_bad, status);
}


// One workgroup per component: blocked FP64 Cholesky of A_c on MFMA
// (chol_tp64), T_c^T = A_c^{-1} Cc_c^T with all D right-hand sides at once
// (solve_tp64, in place in T_c), then Sigma_c = sym((S_c - T_c Cc_c^T) / N_c)
// with T_c Cc_c^T on MFMA, kept only if it is positive definite.  T_c and
// Sigma_c are untouched when A_c is not positive definite.
__global__ void __launch_bounds__(256, 2)
k_mstep_solve(int C, int D, int R, int nb, int64_t TP, double* __restrict__ A,
              const double* __restrict__ Cc, const double* __restrict__ N,
              const double* __restrict__ S, int update_sigma, double* __restrict__ T,
              double* __restrict__ Sigma, double* __restrict__ Winv_all,
              int* __restrict__ status, int* __restrict__ err, int left) {
  extern __shared__ double sm[];
  double* dg = sm;            // [256]
  double* zb = sm + 256;      // [16 * 64]
  double* big = sm + 1280;    // max(nb * 256, 4096 + D * D)
  __shared__ int s_bad;
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  const double Nc = N[c];
  if (!(Nc >= kMinCount)) {  // no data: keep T_c, Sigma_c
    if (tid == 0) status[c] = 1;
    return;
  }
  double* Ac = A + (int64_t)c * TP;
  double* Winv = Winv_all + (int64_t)c * nb * 256;
  // identity on the padded diagonal so the padding factors trivially
  for (int d = R + tid; d < nb * 16; d += 256) Ac[tp_off(d >> 4, d >> 4) + (d & 15) * 17] = 1.0;
  __syncthreads();
  const int bad = left ? chol_ll64(Ac, nb, Winv, dg, big, &s_bad)
                       : chol_tp64(Ac, nb, Winv, dg, big, &s_bad);
  if (bad) {
    if (tid == 0) {
      status[c] = 3;
      raise_error(err, IVX_ENOTPD, PK_MSTEP, c);
    }
    return;
  }
  // T_c^T = A_c^{-1} Cc_c^T: right-hand sides copied into T_c ([D][R])
  const double* Ccc = Cc + (int64_t)c * D * R;
  double* Tc = T + (int64_t)c * D * R;
  for (int e = tid; e < D * R; e += 256) Tc[e] = Ccc[e];
  __syncthreads();
  solve_tp64(Ac, Winv, nb, Tc, R, R, D, zb);
  if (!update_sigma) {
    if (tid == 0) status[c] = 0;
    return;
  }
  sigma_update(c, D, R, Nc, Tc, Ccc, S, Sigma, big, &s_bad, status);
}

// The same M-step with the right-hand sides held in registers, one
// workgroup of 8 waves per component.  The 64 x R block of right-hand sides
// B = Cc_c^T (D padded to 64) is split into 16 x 16 tiles; wave w keeps the
// tiles of column block w % 4 and row blocks i = w / 4 + 2 s (s < 13) as
// FP64 MFMA fragments.  Block column k of the Cholesky factor is formed
// left-looking in LDS (A_ik - sum_{j<k} G_ij G_kj^T from the finished
// columns in device memory, block row k of G staged in LDS), its diagonal
// tile factored and inverted in one wave's registers while the other waves
// stage block row k + 1, the column written once, and the forward-solve step
// for block row k runs on it while it is still in LDS: Z_k = G_kk^{-1} B_k,
// then B_i -= G_ik Z_k (i > k), which overlaps the next column's formation.
// The backward solve G^T X = Z then reads each tile of G once.  The
// right-hand sides never leave the registers between the read of Cc_c and
// the write of T_c, and T_c Cc_c^T for the Sigma update is formed from them
// there.
constexpr int MR_NW = 8;
constexpr int MR_NS = 13;     // right-hand-side slots per wave (nb <= 26)
constexpr int MR_MAXNB = 25;  // R <= 400
constexpr size_t MR_LDS_DOUBLES = 2 * MR_MAXNB * 256 + 16 * 64 + (MR_MAXNB - 1) * 256;

__global__ void __launch_bounds__(MR_NW * 64)
k_mstep_rr(int C, int D, int R, int nb, int64_t TP, double* __restrict__ A,
           const double* __restrict__ Cc, const double* __restrict__ N,
           const double* __restrict__ S, int update_sigma, double* __restrict__ T,
           double* __restrict__ Sigma, int* __restrict__ status, int* __restrict__ err) {
  extern __shared__ double sm[];
  double* pan = sm;                     // [nb][256] block column k (tile it = row k + it)
  double* pan2 = sm + MR_MAXNB * 256;   // [nb][256] G_(k+it),k (tiles 1 .. nb-k-1) for the
                                        // forward update, and W_j = G_jj^{-1} (row-major) of
                                        // every step j <= k in tile wtile(j)
  double* zb = pan2 + MR_MAXNB * 256;   // [16][64] Z_k, then X_k
  double* rowk = zb + 16 * 64;          // [nb - 1][256] block row k of G
  __shared__ int s_bad;
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, q16 = lane >> 4;
  const double Nc = N[c];
  if (!(Nc >= kMinCount)) {  // no data: keep T_c, Sigma_c
    if (tid == 0) status[c] = 1;
    return;
  }
  double* Ac = A + (int64_t)c * TP;
  const double* Ccc = Cc + (int64_t)c * D * R;
  // identity on the padded diagonal so the padding factors trivially
  for (int d = R + tid; d < nb * 16; d += MR_NW * 64) Ac[tp_off(d >> 4, d >> 4) + (d & 15) * 17] = 1.0;
  // right-hand sides: slot s = row block ib + 2 s, column block db;
  // register r = B[16 i + 4 r + q16][16 db + l16] = Cc_c[16 db + l16][16 i + 4 r + q16]
  const int ib = wave >> 2, db = wave & 3, dcol = 16 * db + l16;
  doublex4 bt[MR_NS];
#pragma unroll
  for (int s = 0; s < MR_NS; ++s) {
    const int i = ib + 2 * s;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * i + 4 * r + q16;
      bt[s][r] = (i < nb && row < R && dcol < D) ? Ccc[(int64_t)dcol * R + row] : 0.0;
    }
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();

  // The LDS tiles (pan, pan2, rowk) are stored column-major (element (r, c)
  // at 16 c + r), so that the reads of an MFMA operand fragment (row l16 of
  // the tile in lane l16) fall in consecutive words; tiles in device memory
  // are row-major.
  // pan2 tile of W_k: tile 0 for k = 0, else nb - k (the panel tiles of step
  // k are 1 .. nb - k - 1, and W_k is written after step k - 1's last use
  // of tile nb - k)
  const auto wtile = [nb](int k) { return k == 0 ? 0 : nb - k; };
  for (int k = 0; k < nb; ++k) {
    const int m1 = nb - k;  // tiles of block column k, the diagonal one first
    // ---- block column k: A_(k+it),k - sum_{j<k} G_(k+it),j G_k,j^T, with
    //      block row k of G (shared by every row's sum) already in rowk; each
    //      wave keeps the tiles of the next three j in flight while it
    //      multiplies the current one (contraction index 4 q16 + q: lane
    //      (l16, q16) reads four consecutive doubles of row l16 of a tile).
    //      No barrier before it: it writes pan only, and the previous step's
    //      forward update reads pan2 and zb.
    const int ro = l16 * 16 + 4 * q16;
    if (m1 > MR_NW) {
      // two rows per wave, independent accumulators (a wave with one row
      // computes it twice and stores it once)
      for (int it0 = wave; it0 < m1; it0 += 2 * MR_NW) {
        const int itA = it0, itB = it0 + MR_NW < m1 ? it0 + MR_NW : it0;
        const double* At = Ac + tp_off(k + itA, k);
        const double* Bt = Ac + tp_off(k + itB, k);
        doublex4 accA, accB;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accA[r] = At[(4 * r + q16) * 16 + l16];
          accB[r] = Bt[(4 * r + q16) * 16 + l16];
        }
        double2 a0[2], b0[2], a1[2], b1[2], a2[2], b2[2];
        auto load = [&](int j, double2 (&ga)[2], double2 (&gb)[2]) {
          const double2* Ga = reinterpret_cast<const double2*>(Ac + tp_off(k + itA, j) + ro);
          const double2* Gb = reinterpret_cast<const double2*>(Ac + tp_off(k + itB, j) + ro);
          ga[0] = Ga[0];
          ga[1] = Ga[1];
          gb[0] = Gb[0];
          gb[1] = Gb[1];
        };
        auto step = [&](int j, const double2 (&ga)[2], const double2 (&gb)[2]) {
          const double* Kr = rowk + j * 256 + 64 * q16 + l16;  // G_kj[l16][4 q16 + n] at Kr[16 n]
          const double k0 = Kr[0], k1 = Kr[16], k2 = Kr[32], k3 = Kr[48];
          accA = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[0].x, k0, accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f64_16x16x4f64(-gb[0].x, k0, accB, 0, 0, 0);
          accA = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[0].y, k1, accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f64_16x16x4f64(-gb[0].y, k1, accB, 0, 0, 0);
          accA = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[1].x, k2, accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f64_16x16x4f64(-gb[1].x, k2, accB, 0, 0, 0);
          accA = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[1].y, k3, accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f64_16x16x4f64(-gb[1].y, k3, accB, 0, 0, 0);
        };
        if (k > 0) load(0, a0, b0);
        if (k > 1) load(1, a1, b1);
        if (k > 2) load(2, a2, b2);
        for (int j = 0; j < k; j += 3) {
          step(j, a0, b0);
          if (j + 3 < k) load(j + 3, a0, b0);
          if (j + 1 < k) {
            step(j + 1, a1, b1);
            if (j + 4 < k) load(j + 4, a1, b1);
          }
          if (j + 2 < k) {
            step(j + 2, a2, b2);
            if (j + 5 < k) load(j + 5, a2, b2);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pan[itA * 256 + l16 * 16 + 4 * r + q16] = accA[r];
          if (itB != itA) pan[itB * 256 + l16 * 16 + 4 * r + q16] = accB[r];
        }
      }
    } else {
      // at most one row per wave: the waves of row it = w % m1 split its
      // sum over j into equal ranges; the partial sums of the waves w >= m1
      // go to the free panel slots MR_NW + w and are added in a fixed order
      const int it = wave % m1, p = wave / m1, P = (MR_NW - 1 - it) / m1 + 1;
      const int j0 = p * k / P, j1 = (p + 1) * k / P;
      const double* At = Ac + tp_off(k + it, k);
      doublex4 acc0;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc0[r] = p == 0 ? At[(4 * r + q16) * 16 + l16] : 0.0;
      double2 g0[2], g1[2], g2[2];
      auto load1 = [&](int j, double2 (&g)[2]) {
        const double2* G = reinterpret_cast<const double2*>(Ac + tp_off(k + it, j) + ro);
        g[0] = G[0];
        g[1] = G[1];
      };
      auto step1 = [&](int j, const double2 (&g)[2], doublex4& acc) {
        const double* Kr = rowk + j * 256 + 64 * q16 + l16;  // G_kj[l16][4 q16 + n] at Kr[16 n]
        const double k0 = Kr[0], k1 = Kr[16], k2 = Kr[32], k3 = Kr[48];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-g[0].x, k0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-g[0].y, k1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-g[1].x, k2, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-g[1].y, k3, acc, 0, 0, 0);
      };
      if (j0 < j1) load1(j0, g0);
      if (j0 + 1 < j1) load1(j0 + 1, g1);
      if (j0 + 2 < j1) load1(j0 + 2, g2);
      for (int j = j0; j < j1; j += 3) {
        step1(j, g0, acc0);
        if (j + 3 < j1) load1(j + 3, g0);
        if (j + 1 < j1) {
          step1(j + 1, g1, acc0);
          if (j + 4 < j1) load1(j + 4, g1);
        }
        if (j + 2 < j1) {
          step1(j + 2, g2, acc0);
          if (j + 5 < j1) load1(j + 5, g2);
        }
      }
      double* dst = pan + (p == 0 ? it : MR_NW + wave) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[l16 * 16 + 4 * r + q16] = acc0[r];
      __syncthreads();
      for (int e = tid; e < m1 * 256; e += MR_NW * 64) {
        const int t = e >> 8, np = (MR_NW - 1 - t) / m1 + 1;
        double v = pan[e];
        for (int q = 1; q < np; ++q) v += pan[(MR_NW + t + q * m1) * 256 + (e & 255)];
        pan[e] = v;
      }
    }
    __syncthreads();
    // W_k to pan2 tile wtile(k), which no panel tile of this or a later
    // step uses; the other waves stage block row k + 1 of G (the tiles of
    // the finished columns; tile k comes from the panel below)
    if (wave == 0) {
      diag_factor64<true>(pan, Ac + tp_off(k, k), pan2 + wtile(k) * 256, k * 16, &s_bad);
    } else if (k + 1 < nb) {
      for (int e = tid - 64; e < k * 128; e += (MR_NW - 1) * 64) {
        const int j = e >> 7, w = e & 127;
        const double2 v = reinterpret_cast<const double2*>(Ac + tp_off(k + 1, j))[w];
        const int r = w >> 3, cc = 2 * (w & 7);  // elements (r, cc), (r, cc + 1)
        rowk[j * 256 + cc * 16 + r] = v.x;
        rowk[j * 256 + cc * 16 + 16 + r] = v.y;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const double* W = pan2 + wtile(k) * 256;
    // ---- panel G_(k+it),k = pan_it W^T (to pan2 and device memory; tile 1
    //      also to rowk as the last tile of the next block row), and
    //      Z_k = W B_k by the owners of row block k
    for (int it = 1 + wave; it < m1; it += MR_NW) {
      const double* Pt = pan + it * 256;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16_xyt([&](int i, int l) { return Pt[l * 16 + i]; },
                      [&](int j, int l) { return W[l * 16 + j]; }, acc, 1.0);
      double* Gt = Ac + tp_off(k + it, k);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Gt[(4 * r + q16) * 16 + l16] = acc[r];
        pan2[it * 256 + l16 * 16 + 4 * r + q16] = acc[r];
        if (it == 1) rowk[k * 256 + l16 * 16 + 4 * r + q16] = acc[r];
      }
    }
    if (ib == (k & 1)) {
#pragma unroll
      for (int s = 0; s < MR_NS; ++s) {
        if (s == (k >> 1)) {
          doublex4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            z = __builtin_amdgcn_mfma_f64_16x16x4f64(W[(4 * q + q16) * 16 + l16], bt[s][q], z, 0, 0, 0);
          bt[s] = z;
#pragma unroll
          for (int r = 0; r < 4; ++r) zb[(4 * r + q16) * 64 + dcol] = z[r];
        }
      }
    }
    __syncthreads();
    // ---- B_i -= G_ik Z_k for i > k.  No barrier after it: the next step
    //      writes only pan until its first barrier.
#pragma unroll
    for (int s = 0; s < MR_NS; ++s) {
      const int i = ib + 2 * s;
      if (i > k && i < nb) {
        const double* Gt = pan2 + (i - k) * 256;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bt[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-Gt[(4 * q + q16) * 16 + l16], zb[(4 * q + q16) * 64 + dcol],
                                                       bt[s], 0, 0, 0);
      }
    }
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) {
      status[c] = 3;
      raise_error(err, IVX_ENOTPD, PK_MSTEP, c);
    }
    return;
  }
  // ---- backward solve G^T X = Z: X_k = W_k^T Z_k, then Z_i -= G_ki^T X_k (i < k)
  for (int k = nb - 1; k >= 0; --k) {
    const double* W = pan2 + wtile(k) * 256;
    if (ib == (k & 1)) {
#pragma unroll
      for (int s = 0; s < MR_NS; ++s) {
        if (s == (k >> 1)) {
          doublex4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            x = __builtin_amdgcn_mfma_f64_16x16x4f64(W[l16 * 16 + 4 * q + q16], bt[s][q], x, 0, 0, 0);
          bt[s] = x;
#pragma unroll
          for (int r = 0; r < 4; ++r) zb[(4 * r + q16) * 64 + dcol] = x[r];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MR_NS; ++s) {
      const int i = ib + 2 * s;
      if (i < k) {
        const double* Gt = Ac + tp_off(k, i);
        double g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = Gt[(4 * q + q16) * 16 + l16];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bt[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-g[q], zb[(4 * q + q16) * 64 + dcol], bt[s],
                                                       0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ---- T_c[d][r] = X[r][d]
  double* Tc = T + (int64_t)c * D * R;
  if (dcol < D) {
#pragma unroll
    for (int s = 0; s < MR_NS; ++s) {
      const int i = ib + 2 * s;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + 4 * r + q16;
        if (i < nb && row < R) Tc[(int64_t)dcol * R + row] = bt[s][r];
      }
    }
  }
  if (!update_sigma) {
    if (tid == 0) status[c] = 0;
    return;
  }
  // ---- T_c Cc_c^T from the X fragments: wave (ib, db) sums over its row
  //      blocks for the output tiles (db, tb), tb < 4 (A operand: the slot's
  //      fragment as it stands, B operand: Cc_c^T read from device memory);
  //      the halves ib = 0 and 1 are added in LDS in a fixed order.  pan and
  //      pan2 are free after the backward solve.
  doublex4 pc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) pc[tb] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < MR_NS; ++s) {
    const int i = ib + 2 * s;
    if (i < nb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + 4 * r + q16;
        double cv[4];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
          const int b = 16 * tb + l16;
          cv[tb] = (row < R && b < D) ? Ccc[(int64_t)b * R + row] : 0.0;
        }
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
          pc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bt[s][r], cv[tb], pc[tb], 0, 0, 0);
      }
    }
  }
  double* Pb = sm + (ib ? 8192 : 0);
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Pb[(16 * db + 4 * r + q16) * 64 + 16 * tb + l16] = pc[tb][r];
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += MR_NW * 64) sm[e] += sm[8192 + e];
  __syncthreads();
  sigma_finish(c, D, Nc, S, Sigma, sm, &s_bad, status);
}

// Minimum-divergence set-up, one workgroup of 256 threads:
//   G = H/U - (h/U)(h/U)^T (tile-packed) = L_G L_G^T  (chol_tp64, MFMA)
//   g = L_G^{-1} h/U, Householder vector a from g, p = P2 g,
//   M = P1^{-1} P2^{-1} = L_G P2 = L_G - 2 (L_G a) a^T   ([R][R] row-major).
// Standard formulation: M = L_G and nothing else (p is not touched).
// On failure M = I, p is left unchanged and h/U (vec[0..R)) is set to 0.
__global__ void __launch_bounds__(256)
k_mindiv_setup(int R, int nb, const double* __restrict__ hsum, const double* __restrict__ Htp,
               const double* __restrict__ count, int standard, double* __restrict__ G,
               double* __restrict__ Winv, double* __restrict__ M, double* __restrict__ vec,
               double* __restrict__ p, int* __restrict__ err) {
  extern __shared__ double sm[];
  double* dg = sm;          // [256]
  double* pan = sm + 256;   // [(nb - 1) * 256]
  __shared__ double red[256];
  __shared__ double sc[4];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const double U = count[0];
  double* hb = vec;         // h / U
  double* g = vec + R;      // L_G^{-1} h / U
  double* a = vec + 2 * R;  // Householder vector
  double* v = vec + 3 * R;  // L_G a
  for (int i = tid; i < R; i += 256) hb[i] = hsum[i] / U;
  __syncthreads();
  // G in the tile-packed layout, identity on the padded diagonal
  const int64_t ntp = (int64_t)nb * (nb + 1) / 2 * 256;
  for (int64_t e = tid; e < ntp; e += 256) {
    const int t = (int)(e >> 8), w = (int)(e & 255);
    int bi, bj;
    tri_decode(t, bi, bj);
    const int i = bi * 16 + (w >> 4), j = bj * 16 + (w & 15);
    double v0;
    if (i < R && j < R)
      v0 = Htp[e] / U - hb[i] * hb[j];
    else
      v0 = (i == j) ? 1.0 : 0.0;
    G[e] = v0;
  }
  __syncthreads();
  const int bad = chol_tp64(G, nb, Winv, dg, pan, &s_bad);
  if (bad) {  // leave T and p unchanged: M = I
    if (tid == 0) raise_error(err, IVX_ENOTPD, PK_MINDIV, bad - 1);
    for (int e = tid; e < R * R; e += 256) M[e] = (e / R == e % R) ? 1.0 : 0.0;
    for (int i = tid; i < R; i += 256) hb[i] = 0.0;
    return;
  }
  if (standard) {  // M = P1^{-1} = L_G
    for (int e = tid; e < R * R; e += 256) {
      const int i = e / R, j = e - i * R;
      M[e] = (j <= i) ? G[tp_off(i >> 4, j >> 4) + (i & 15) * 16 + (j & 15)] : 0.0;
    }
    return;
  }
  // g = L^{-1} hb, blocked: g_k = W_k r_k, then r_i -= L_ik g_k (i > k)
  for (int i = tid; i < R; i += 256) g[i] = hb[i];  // r
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid < 16) {
      double s = 0.0;
      for (int l = 0; l < 16; ++l) {
        const int r = k * 16 + l;
        if (r < R) s += Winv[k * 256 + tid * 16 + l] * g[r];
      }
      red[tid] = s;
    }
    __syncthreads();
    if (tid < 16 && k * 16 + tid < R) g[k * 16 + tid] = red[tid];
    __syncthreads();
    for (int i = (k + 1) * 16 + tid; i < R; i += 256) {
      const double* Lt = G + tp_off(i >> 4, k) + (i & 15) * 16;
      double s = 0.0;
      for (int l = 0; l < 16; ++l) s += Lt[l] * g[k * 16 + l];
      g[i] -= s;
    }
    __syncthreads();
  }
  double s2 = 0.0;
  for (int i = 1 + tid; i < R; i += 256) s2 += g[i] * g[i];
  red[tid] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    const double ss = red[0];
    const double tail = sqrt(ss);
    const double gn = sqrt(ss + g[0] * g[0]);
    double alpha = 0.0;
    if (tail > 1e-12 * gn) {
      const double one_minus = (g[0] > 0.0) ? ss / (gn * (gn + g[0])) : 1.0 - g[0] / gn;
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
  double ag = 0.0;
  for (int i = tid; i < R; i += 256) ag += a[i] * g[i];
  red[tid] = ag;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  ag = red[0];
  // p = P2 g = g - 2 a (a^T g);  v = L a
  for (int i = tid; i < R; i += 256) {
    p[i] = g[i] - 2.0 * a[i] * ag;
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += G[tp_off(i >> 4, k >> 4) + (i & 15) * 16 + (k & 15)] * a[k];
    v[i] = s;
  }
  __syncthreads();
  // M = L_G P2 = L_G - 2 (L_G a) a^T
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e - i * R;
    const double lij = (j <= i) ? G[tp_off(i >> 4, j >> 4) + (i & 15) * 16 + (j & 15)] : 0.0;
    M[e] = lij - 2.0 * v[i] * a[j];
  }
}

// bias[row] += T[row, :] . hb over rows = C * D, one wave per row
__global__ void __launch_bounds__(256)
k_bias_update(const double* __restrict__ T, const double* __restrict__ hb, int64_t rows, int R,
              double* __restrict__ bias) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const double* t = T + row * R;
  double s = 0.0;
  for (int r = lane; r < R; r += 64) s += t[r] * hb[r];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) bias[row] += s;
}

// Tn[rows x R] = T[rows x R] * M[R x R], 64 x 64 tiles, 4 x 4 outputs per thread
__global__ void __launch_bounds__(256)
k_apply_M(const double* __restrict__ T, const double* __restrict__ M, int64_t rows, int R,
          double* __restrict__ Tn) {
  // 64 x 64 output tile; wave w computes the 32 x 32 quarter (w / 2, w % 2)
  // as 2 x 2 blocks of v_mfma_f64_16x16x4f64, K staged 16 at a time.  LDS
  // rows are padded to 80 doubles so that the four K rows a wave reads at
  // once fall into alternate halves of the banks.
  constexpr int AL = 64 + 16;
  __shared__ double As[16][AL];  // [k][row]
  __shared__ double Bs[16][AL];  // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int wm = w >> 1, wn = w & 1;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int c0 = blockIdx.x * 64;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
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
    for (int ks = 0; ks < 16; ks += 4) {
      const int k = ks + q16;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[k][wm * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[k][wn * 32 + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[i][j][r] = Tn[r0 + 32 wm + 16 i + 4 r + q16][c0 + 32 wn + 16 j + l16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = c0 + wn * 32 + j * 16 + l16;
      if (col >= R) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + i * 16 + 4 * r + q16;
        if (row < rows) Tn[row * R + col] = acc[i][j][r];
      }
    }
}

}  // namespace

void launch_objective(ivx_ctx* ctx, const double* N, const double* S, const double* ll_sum,
                      double* objective, hipStream_t s) {
  k_objective_parts<<<ctx->C, 256, 0, s>>>(N, S, ctx->Psig, ctx->sig_logdet, ctx->D, ctx->obj_part);
  k_objective_finish<<<1, 256, 0, s>>>(ctx->obj_part, ctx->C, ll_sum, objective);
}

size_t mstep_lds_bytes(int R, int D);

bool mstep_set_attributes() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mstep_solve),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)mstep_lds_bytes(480, 63)) == hipSuccess &&
         hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mstep_rr),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(MR_LDS_DOUBLES * sizeof(double))) == hipSuccess;
}

size_t mstep_lds_bytes(int R, int D) {
  const int nb = (R + 15) / 16;
  size_t nbig = (size_t)nb * 256;  // the left-looking form keeps a whole block column
  if ((size_t)4096 + (size_t)D * D > nbig) nbig = (size_t)4096 + (size_t)D * D;
  return sizeof(double) * (1280 + nbig);
}

void launch_mstep_solve(ivx_ctx* ctx, const ivx_accum* acc, const double* S, int update_sigma,
                        int* status, hipStream_t s) {
  const int nb = (ctx->R + 15) / 16;
  if (!ctx->tune.mstep_global && nb <= MR_MAXNB) {
    k_mstep_rr<<<ctx->C, MR_NW * 64, MR_LDS_DOUBLES * sizeof(double), s>>>(
        ctx->C, ctx->D, ctx->R, nb, ctx->TP, acc->A, acc->Cc, acc->N, S, update_sigma, ctx->T,
        ctx->Sigma, status, ctx->dev_err);
    return;
  }
  k_mstep_solve<<<ctx->C, 256, mstep_lds_bytes(ctx->R, ctx->D), s>>>(
      ctx->C, ctx->D, ctx->R, nb, ctx->TP, acc->A, acc->Cc, acc->N, S, update_sigma, ctx->T,
      ctx->Sigma, ctx->Winv, status, ctx->dev_err, ctx->tune.mstep_left);
}

ivx_status launch_mindiv(ivx_ctx* ctx, const ivx_accum* acc, bool standard, bool update_mean,
                         hipStream_t s) {
  const int nb = (ctx->R + 15) / 16;
  k_mindiv_setup<<<1, 256, sizeof(double) * 256 * nb, s>>>(
      ctx->R, nb, acc->h, acc->H, acc->count, standard ? 1 : 0, ctx->Gmat, ctx->Winv, ctx->Mmat,
      ctx->mvec, ctx->p, ctx->dev_err);
  const int64_t rows = (int64_t)ctx->C * ctx->D;
  if (standard && update_mean) {  // reads T before the whitened copy replaces it
    k_bias_update<<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(ctx->T, ctx->mvec, rows, ctx->R,
                                                            ctx->bias);
    launch_bias32(ctx, s);
  }
  dim3 grid((unsigned)((ctx->R + 63) / 64), (unsigned)((rows + 63) / 64));
  k_apply_M<<<grid, 256, 0, s>>>(ctx->T, ctx->Mmat, rows, ctx->R, ctx->Tnew);
  // copy back on the stream (no host-side pointer swap, so a captured graph
  // replays correctly)
  if (hipMemcpyAsync(ctx->T, ctx->Tnew, sizeof(double) * rows * ctx->R, hipMemcpyDeviceToDevice,
                     s) != hipSuccess) {
    set_error("tv_mindiv: queueing the copy of the updated T failed");
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

}  // namespace ivx
