// Baum-Welch statistics (Sec. 2) from the sparse per-frame posterior lists.
//
//  n_c(u), f_c(u): a map from frame to utterance (k_frame_utt, which also
//    checks the offsets), then every kept posterior entry is added to its
//    (utterance, component) row of 64-bit fixed-point sums (k_nf.h; from the
//    posterior lists in k_nf_accum, or inside the rescoring pass of the
//    all-component posteriors), and k_nf_finish converts the sums to FP32
//    n and f (zeros included) and resets them.
//  S_c = sum_t gamma_tc x_t x_t^T (FP64 totals): the (frame, component)
//    posterior entries are bucketed by component with a counting sort
//    (per-block histograms, a scan, a scatter); one workgroup per component
//    then forms (gamma X)^T X on FP64 MFMA over its entries.
//  Standard formulation (Sec. 2): with a bias m set, every term is centred
//    before it is accumulated, f~_c(u) = sum_t gamma_tc (x_t - m_c) and
//    S~_c = sum_t gamma_tc (x_t - m_c)(x_t - m_c)^T (the frames staged as
//    FP64 x - m_c), so no large uncentred sums are formed and cancelled.
#include <algorithm>

#include "ivx_internal.h"
#include "k_nf.h"

namespace ivx {
namespace {

constexpr int HB = 8192;       // frames per histogram block

// One workgroup per utterance: checks its offsets (0 = utt_off[0] <= ... <=
// utt_off[U] = F) and writes the utterance index of each of its frames.
__global__ void __launch_bounds__(256)
k_frame_utt(const int64_t* __restrict__ utt_off, int64_t U, int64_t F, int* __restrict__ umap,
            int* __restrict__ err) {
  const int64_t u = blockIdx.x;
  const int64_t t0 = utt_off[u], t1 = utt_off[u + 1];
  const bool bad = (t0 > t1) || (t0 < 0) || (t1 > F) || (u == 0 && t0 != 0) ||
                   (u == U - 1 && t1 != F);
  if (bad) {
    if (threadIdx.x == 0) raise_error(err, IVX_EINVAL, PK_STATS_NF, (int)u);
    return;
  }
  for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) umap[t] = (int)u;
}

// n/f from the posterior lists, one wave per frame (frames of one workgroup
// consecutive): the kept entries of frame g are added to the fixed-point
// sums of its utterance (nf_add_entry).
__global__ void __launch_bounds__(256)
k_nf_accum(const float* __restrict__ X, int64_t F, int D, int C, const int* __restrict__ post_idx,
           const float* __restrict__ post_val, const int* __restrict__ umap, int64_t U,
           const float* __restrict__ mb, unsigned long long* __restrict__ acc,
           int* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= F) return;
  const int u = umap[g];
  if (u < 0 || u >= U) return;  // offsets rejected by k_frame_utt
  const int id = (lane < KP) ? post_idx[g * KP + lane] : -1;
  const float gv = (lane < KP) ? post_val[g * KP + lane] : 0.0f;
  const float xv = (lane >= 1 && lane <= D) ? X[g * D + (lane - 1)] : 0.0f;
  uint64_t mask = __ballot(id >= 0 && id < C);
  while (mask) {
    const int sl = __ffsll((unsigned long long)mask) - 1;
    mask &= mask - 1;
    nf_add_entry(acc, (int64_t)u * C, D, lane, xv, mb, __shfl(id, sl), (double)__shfl(gv, sl),
                 err);
  }
}

// n[u][c] and f[u][c][:] from the fixed-point sums, which are reset to zero
// for the next call; every (u, c) is written, zeros included.
__global__ void __launch_bounds__(256)
k_nf_finish(int64_t U, int C, int D, unsigned long long* __restrict__ acc, float* __restrict__ n,
            float* __restrict__ f) {
  const int DS = D + 1;
  const int64_t total = U * C * DS;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const long long v = (long long)acc[i];
    acc[i] = 0ull;
    const float val = (float)((double)v * kFixInv);
    const int64_t row = i / DS;
    const int col = (int)(i - row * DS);
    if (col == 0)
      n[row] = val;
    else
      f[row * D + col - 1] = val;
  }
}

// hist[b][c] = number of posterior entries of component c in frame block b
__global__ void __launch_bounds__(256)
k_hist(int64_t F, int C, const int* __restrict__ post_idx, int* __restrict__ hist) {
  extern __shared__ int hl[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) hl[c] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)b * HB * KP;
  const int64_t e1 = min(F * KP, e0 + (int64_t)HB * KP);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = post_idx[e];
    if (c >= 0) atomicAdd(&hl[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) hist[(size_t)b * C + c] = hl[c];
}

// Turns hist into exclusive offsets in (component, block) order and writes
// coff[c] = first entry of component c (coff[C] = total).  One workgroup.
__global__ void __launch_bounds__(1024) k_hist_scan(int nb, int C, int* __restrict__ hist,
                                                     int* __restrict__ coff) {
  __shared__ int tot[1024];
  __shared__ int wsum[16];
  // per-component totals; each thread owns components c = tid, tid+1024, ...
  int carry = 0;
  for (int cbase = 0; cbase < C; cbase += 1024) {
    const int c = cbase + threadIdx.x;
    int s = 0;
    if (c < C)
      for (int b = 0; b < nb; ++b) s += hist[(size_t)b * C + c];
    tot[threadIdx.x] = s;
    __syncthreads();
    // inclusive scan of tot (Hillis-Steele)
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = (threadIdx.x >= o) ? tot[threadIdx.x - o] : 0;
      __syncthreads();
      tot[threadIdx.x] += v;
      __syncthreads();
    }
    const int excl = carry + ((threadIdx.x > 0) ? tot[threadIdx.x - 1] : 0);
    if (c < C) {
      coff[c] = excl;
      int run = excl;
      for (int b = 0; b < nb; ++b) {
        const int v = hist[(size_t)b * C + c];
        hist[(size_t)b * C + c] = run;
        run += v;
      }
    }
    const int last = tot[1023];
    __syncthreads();
    carry += last;
  }
  if (threadIdx.x == 0) coff[C] = carry;
  (void)wsum;
}

__global__ void __launch_bounds__(256)
k_scatter(int64_t F, int C, const int* __restrict__ post_idx, const float* __restrict__ post_val,
          const int* __restrict__ base, int2* __restrict__ ent) {
  extern __shared__ int cur[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) cur[c] = base[(size_t)b * C + c];
  __syncthreads();
  const int64_t e0 = (int64_t)b * HB * KP;
  const int64_t e1 = min(F * KP, e0 + (int64_t)HB * KP);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = post_idx[e];
    if (c >= 0) {
      const int pos = atomicAdd(&cur[c], 1);
      ent[pos] = make_int2((int)(e / KP), __float_as_int(post_val[e]));
    }
  }
}

// S_c += sum over the component's entries of gamma x x^T (centred on mb[c]
// when mb is given) as an FP64 MFMA product (gamma X)^T X over the entries,
// 64 entries staged at a time in LDS.  Output 64 x 64 (D <= 63, zero
// padded): wave w computes rows 16w..16w+15 as four 16 x 16 blocks of
// v_mfma_f64_16x16x4f64; the upper triangle (i <= j < D) is added to S_acc.
constexpr int SE = 64;      // entries per LDS stage
constexpr int SLD = 64 + 4; // padded row (doubles)
typedef double sdoublex4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_S_mfma(const float* __restrict__ X, int D, const int* __restrict__ coff,
         const int2* __restrict__ ent, const double* __restrict__ mb, double* __restrict__ S_acc) {
  __shared__ double xs[SE][SLD];  // entry e, feature d: x (or x - m_c)
  __shared__ double gs[SE];       // gamma of entry e
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, q16 = lane >> 4;
  const int e0 = coff[c], e1 = coff[c + 1];
  const double* mc = mb ? mb + (size_t)c * D : nullptr;
  sdoublex4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = sdoublex4{0.0, 0.0, 0.0, 0.0};
  // stage loader: thread tid stages feature d = tid % 64 of entries
  // e = tid / 64 + 4 it; the next stage is requested before the current
  // stage's MFMAs and written to LDS after them
  constexpr int NIT = SE * 64 / 256;
  const int dl = tid & 63, el = tid >> 6;
  float xr[NIT];
  float gr = 0.0f;
  int nr = 0;
  auto gload = [&](int eb) {
    nr = min(SE, e1 - eb);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = el + 4 * it;
      xr[it] = (e < nr && dl < D) ? X[(int64_t)ent[eb + e].x * D + dl] : 0.0f;
    }
    gr = (tid < nr) ? __int_as_float(ent[eb + tid].y) : 0.0f;
  };
  if (e0 < e1) gload(e0);
  for (int eb = e0; eb < e1; eb += SE) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = el + 4 * it;
      double v = 0.0;
      if (e < nr && dl < D) {
        v = (double)xr[it];
        if (mc) v -= mc[dl];
      }
      xs[e][dl] = v;
    }
    if (tid < SE) gs[tid] = (double)gr;
    __syncthreads();
    if (eb + SE < e1) gload(eb + SE);
#pragma unroll 4
    for (int k = 0; k < SE; k += 4) {
      const int e = k + q16;
      const double a = gs[e] * xs[e][16 * w + l16];  // A[m][k] = gamma_e x_e[m]
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xs[e][16 * j + l16], acc[j], 0, 0, 0);
    }
  }
  // acc[j][r] = S[16 w + 4 r + q16][16 j + l16]
  const int Dp = D * (D + 1) / 2;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + 4 * r + q16, jj = 16 * j + l16;
      if (i < D && jj < D && i <= jj)
        S_acc[(size_t)c * Dp + i * D - i * (i - 1) / 2 + (jj - i)] += acc[j][r];
    }
}

__global__ void __launch_bounds__(256) k_sum_partial(const double* __restrict__ x, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_final(const double* __restrict__ part, int np,
                                                   double* __restrict__ acc) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += sh[0];
}

}  // namespace

NfTarget launch_frame_utt(ivx_ctx* ctx, const int64_t* utt_off, int64_t U, int64_t F,
                          hipStream_t s) {
  if (U > 0) k_frame_utt<<<(unsigned)U, 256, 0, s>>>(utt_off, U, F, ctx->umap, ctx->dev_err);
  return NfTarget{ctx->umap, U, ctx->standard ? ctx->bias32 : nullptr, ctx->nf_acc};
}

void launch_nf_accum(ivx_ctx* ctx, const float* X, int64_t F, const int* post_idx,
                     const float* post_val, const NfTarget& nf, hipStream_t s) {
  if (F <= 0 || nf.U <= 0) return;
  k_nf_accum<<<(unsigned)((F + 3) / 4), 256, 0, s>>>(X, F, ctx->D, ctx->C, post_idx, post_val,
                                                     nf.umap, nf.U, nf.mb, nf.acc, ctx->dev_err);
}

void launch_nf_finish(ivx_ctx* ctx, int64_t U, float* n, float* f, hipStream_t s) {
  if (U <= 0) return;
  const int64_t total = U * ctx->C * (ctx->D + 1);
  const int64_t nb = std::min<int64_t>((total + 255) / 256, 8192);
  k_nf_finish<<<(unsigned)nb, 256, 0, s>>>(U, ctx->C, ctx->D, ctx->nf_acc, n, f);
}

void launch_stats_S(ivx_ctx* ctx, const float* X, int64_t F, double* S_acc, hipStream_t s) {
  if (F <= 0) return;
  const int nb = (int)((F + HB - 1) / HB);
  const size_t ldsc = sizeof(int) * ctx->C;
  k_hist<<<nb, 256, ldsc, s>>>(F, ctx->C, ctx->post_idx, ctx->hist);
  k_hist_scan<<<1, 1024, 0, s>>>(nb, ctx->C, ctx->hist, ctx->coff);
  k_scatter<<<nb, 256, ldsc, s>>>(F, ctx->C, ctx->post_idx, ctx->post_val, ctx->hist, ctx->ent);
  k_S_mfma<<<ctx->C, 256, 0, s>>>(X, ctx->D, ctx->coff, ctx->ent,
                                  ctx->standard ? ctx->bias : nullptr, S_acc);
}

void launch_hist_scan(int nb, int C, int* hist, int* coff, hipStream_t s) {
  k_hist_scan<<<1, 1024, 0, s>>>(nb, C, hist, coff);
}

void launch_sum_f64(ivx_ctx* ctx, const double* x, int64_t n, double* acc, hipStream_t s) {
  if (n <= 0) return;
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  k_sum_partial<<<nb, 256, 0, s>>>(x, n, ctx->partial);
  k_sum_final<<<1, 256, 0, s>>>(ctx->partial, nb, acc);
}

}  // namespace ivx
