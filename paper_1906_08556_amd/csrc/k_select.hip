// Learned Gaussian selection: a small network proposes k components per
// frame, their exact full-covariance log-likelihoods are computed, and frames
// whose proposals carry too little of the network's own probability mass take
// the all-component path.  It stands where the paper's preselection with a
// diagonal-covariance UBM stands (Sec. 4.2: 20 components per frame picked
// cheaply, then scored with the full covariances).
//
// Inference (per chunk of frames):
//   k_mlp_nt<true>   h1 = relu(W1 x_hat + b1)    x_hat standardised, BF16 MFMA
//   k_mlp_nt<false>  h2 = relu(W2 h1 + b2)
//   k_mlp_l3         z  = W3 h2 + b3, one 128-component chunk at a time; each
//                    chunk goes through LDS and every frame keeps a running
//                    top-k (ties to the lower index) and a running log-sum-exp
// then over all frames:
//   k_sel_hist / scan / k_sel_scatter   (frame, proposal) pairs by component
//   k_sel_score      FP32 shifted-form score of every pair: one component per
//                    wave pass, its L^-1 read through the scalar cache
//   k_sel_thr / k_kept_hist / scan / k_kept_scatter / k_exact_sorted
//                    FP64 exact scores of the proposals within the margin of
//                    the frame's best, again bucketed by component
//   k_sel_finalize   posteriors renormalised over the kept proposals
//   fallback frames  gathered and sent through the all-component kernels
//
// Training runs in FP32 on the FP32 GEMM (k_gemm.hip) with the helpers below.
#include <algorithm>
#include <cmath>

#include "ivx_internal.h"
#include "k_exact.h"
#include "k_gemm.h"

namespace ivx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int MT = 128;       // frames per MLP workgroup
constexpr int NT = 128;       // output features (components) per MLP tile
constexpr int KT = 32;        // K per LDS stage
constexpr int LDK = KT + 8;   // LDS row stride (bf16)
constexpr int ZS = NT + 1;    // LDS row stride (floats) of a staged logit chunk
constexpr int HBS = 8192;     // frames per histogram block

__device__ inline uint4 pack8(const float* v) {
  bf16x8 b;
#pragma unroll
  for (int e = 0; e < 8; ++e) b[e] = (__bf16)v[e];
  return *reinterpret_cast<uint4*>(&b);
}

// One 128 x 32 bf16 stage of an operand whose rows are K-contiguous: thread t
// covers row t/2 and k in [16 (t&1), 16 (t&1) + 16).  Rows >= nrows read 0.
struct RowLoader {
  uint4 r[2];
  __device__ void load_bf16(const __bf16* __restrict__ P, int64_t ld, int64_t row0, int64_t nrows,
                            int k0) {
    const int tid = threadIdx.x;
    const int64_t row = row0 + (tid >> 1);
    const int kk = k0 + (tid & 1) * 16;
    if (row < nrows) {
      const uint4* p = reinterpret_cast<const uint4*>(P + row * ld + kk);
      r[0] = p[0];
      r[1] = p[1];
    } else {
      r[0] = r[1] = make_uint4(0, 0, 0, 0);
    }
  }
  // standardised FP32 features: (x - mean) * istd, features >= D read 0
  __device__ void load_x(const float* __restrict__ X, int D, int64_t row0, int64_t nrows, int k0,
                         const float* __restrict__ mean, const float* __restrict__ istd) {
    const int tid = threadIdx.x;
    const int64_t row = row0 + (tid >> 1);
    const int kk = k0 + (tid & 1) * 16;
    float v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int d = kk + e;
      v[e] = (row < nrows && d < D) ? (X[row * D + d] - mean[d]) * istd[d] : 0.0f;
    }
    r[0] = pack8(v);
    r[1] = pack8(v + 8);
  }
  __device__ void store(__bf16* S) const {
    const int tid = threadIdx.x;
    uint4* d = reinterpret_cast<uint4*>(S + (tid >> 1) * LDK + (tid & 1) * 16);
    d[0] = r[0];
    d[1] = r[1];
  }
};

// acc[i][j] += A(rows wm*64 + i*32 ..) * B(rows wn*64 + j*32 ..)^T over one
// staged K = 32; the B operand's rows are the output columns.
__device__ inline void mma_stage(const __bf16* As, const __bf16* Bs, floatx16 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int sub = 0; sub < 2; ++sub) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(As + (wm * 64 + i * 32 + l32) * LDK + sub * 16 + 8 * h);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn * 64 + j * 32 + l32) * LDK + sub * 16 + 8 * h);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// Out[row][n] = relu(sum_k A[row][k] W[n][k] + b[n]) in BF16 for one
// 128 x 128 tile.  FROM_X: A is the standardised feature matrix (K = 64, D
// features and zero padding); else A is a BF16 [rows][K] activation.
template <bool FROM_X>
__global__ void __launch_bounds__(256, 2)
k_mlp_nt(const float* __restrict__ X, int D, const float* __restrict__ mean,
         const float* __restrict__ istd, const __bf16* __restrict__ Ain, int64_t rows, int K,
         const __bf16* __restrict__ W, const float* __restrict__ bias, int N,
         __bf16* __restrict__ Out) {
  __shared__ __bf16 As[2][MT * LDK];
  __shared__ __bf16 Bs[2][NT * LDK];
  const int64_t m0 = (int64_t)blockIdx.y * MT;
  const int n0 = blockIdx.x * NT;
  RowLoader la, lb;
  auto load = [&](int k0) {
    if (FROM_X)
      la.load_x(X, D, m0, rows, k0, mean, istd);
    else
      la.load_bf16(Ain, K, m0, rows, k0);
    lb.load_bf16(W, K, n0, N, k0);
  };
  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};
  const int nk = K / KT;
  load(0);
  la.store(As[0]);
  lb.store(Bs[0]);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load((it + 1) * KT);
    mma_stage(As[cur], Bs[cur], acc);
    if (it + 1 < nk) {
      la.store(As[cur ^ 1]);
      lb.store(Bs[cur ^ 1]);
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = n0 + wn * 64 + j * 32 + l32;
    if (n >= N) continue;
    const float bn = bias[n];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (m < rows) Out[m * N + n] = (__bf16)fmaxf(acc[i][j][r] + bn, 0.0f);
      }
  }
}

// z = W3 h2 + b3 chunk by chunk (128 components), with a running top-KM and
// log-sum-exp per frame.  The components are the MFMA's M operand and the
// frames its N operand, so lane (wave wm, wn; half h; l32) ends every chunk
// holding, for its frames f_j = wn*64 + j*32 + l32 (j = 0, 1), the 32 logits
// of components wm*64 + i*32 + 8*(r/4) + 4h + r%4 (i = 0, 1; r = 0..15), in
// increasing component order.  Each of a frame's four holders (wm, h) keeps
// a sorted top-KM list of its own components in registers (a logit enters
// only above the holder's current KM-th, so after the first chunks inserts
// are rare; equal logits keep the lower component first) and an online
// log-sum-exp.  At the end the four lists go to LDS and every entry's rank
// in the union is counted; ranks below k give the proposals.
// Writes for frame g = row0 + m0 + f: prop[g][0..k) (largest first, ties to
// the lower index), mass[g] = sum over the proposals of softmax(z), fb[g] =
// mass < min_mass, and appends fallback frames to fb_list (counters[0]);
// counters[1] += k per kept frame.  Zout (optional) receives z [rows][C].
template <int KM>
__global__ void __launch_bounds__(256)
k_mlp_l3(const __bf16* __restrict__ H2, int64_t rows, int64_t row0, int K,
         const __bf16* __restrict__ W3, const float* __restrict__ b3, int C, int Cpad, int k,
         float min_mass, int* __restrict__ prop, float* __restrict__ mass, int* __restrict__ fb,
         int* __restrict__ fb_list, int* __restrict__ counters, float* __restrict__ Zout) {
  extern __shared__ float smem[];
  // GEMM stages (bf16): [2][128 * LDK] components, then [2][128 * LDK] frames;
  // after the last chunk the same memory holds the lists [4][128][KM]
  __bf16* As0 = reinterpret_cast<__bf16*>(smem);
  __bf16* Bs0 = As0 + 2 * NT * LDK;
  float* lvs = smem;                                          // [4][MT][KM]
  int* lis = reinterpret_cast<int*>(lvs + 4 * MT * KM);       // [4][MT][KM]
  float* lse_p = reinterpret_cast<float*>(lis + 4 * MT * KM); // [4][MT][2] (max, sum)
  float* mpart = lse_p + 4 * MT * 2;                          // [4][MT]
  int* wg = reinterpret_cast<int*>(mpart + 4 * MT);           // [2]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 5, l32 = lane & 31;
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  float lv[2][KM];
  int li[2][KM];
  float rm[2], rs[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    rm[j] = -INFINITY;
    rs[j] = 0.0f;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
      lv[j][q] = -INFINITY;
      li[j][q] = -1;
    }
  }
  const int nk = K / KT;
  for (int c0 = 0; c0 < Cpad; c0 += NT) {
    // biases of this lane's 32 components of the chunk, loaded before the K
    // loop so that their latency hides behind it (padding components: -inf)
    float bb[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = c0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        bb[i][r] = (c < C) ? b3[c] : -INFINITY;
      }
    RowLoader la, lb;
    auto load = [&](int kk) {
      la.load_bf16(W3, K, c0, Cpad, kk);
      lb.load_bf16(H2, K, m0, rows, kk);
    };
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};
    load(0);
    la.store(As0);
    lb.store(Bs0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      if (it + 1 < nk) load((it + 1) * KT);
      mma_stage(As0 + cur * NT * LDK, Bs0 + cur * MT * LDK, acc);
      if (it + 1 < nk) {
        la.store(As0 + (cur ^ 1) * NT * LDK);
        lb.store(Bs0 + (cur ^ 1) * MT * LDK);
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t fr = m0 + wn * 64 + j * 32 + l32;
      if (fr >= rows) continue;
      // the chunk's 32 logits of this holder; log-sum-exp rescaled once
      float vv[2][16];
      float cmax = -INFINITY;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          vv[i][r] = acc[i][j][r] + bb[i][r];
          cmax = fmaxf(cmax, vv[i][r]);
        }
      if (Zout) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int c = c0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            if (c < C) Zout[fr * C + c] = vv[i][r];
          }
      }
      if (cmax > -INFINITY) {
        const float nm = fmaxf(rm[j], cmax);
        float add = 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) add += __expf(vv[i][r] - nm);
        rs[j] = rs[j] * __expf(rm[j] - nm) + add;
        rm[j] = nm;
      }
      // only a chunk whose best logit beats the holder's KM-th can change
      // the list
      if (cmax > lv[j][KM - 1]) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float v = vv[i][r];
            const int c = c0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            if (v > lv[j][KM - 1]) {
              // compare-shift insert; every comparison reads the old list
#pragma unroll
              for (int q = KM - 1; q > 0; --q) {
                // values, not addresses, are selected (a select between two
                // array addresses would move the lists to scratch memory)
                const float vp = lv[j][q - 1], vq = lv[j][q];
                const int ip = li[j][q - 1], iq = li[j][q];
                const bool up = v > vp;
                const bool at = v > vq;
                lv[j][q] = up ? vp : (at ? v : vq);
                li[j][q] = up ? ip : (at ? c : iq);
              }
              if (v > lv[j][0]) {
                lv[j][0] = v;
                li[j][0] = c;
              }
            }
          }
      }
    }
  }
  // lists and log-sum-exp partials of the four holders to LDS (the GEMM
  // stages are dead: the loop ended with a barrier)
  const int hold = wm * 2 + h;
  if (tid == 0) wg[0] = 0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int f = wn * 64 + j * 32 + l32;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
      lvs[(hold * MT + f) * KM + q] = lv[j][q];
      lis[(hold * MT + f) * KM + q] = li[j][q];
    }
    lse_p[(hold * MT + f) * 2] = rm[j];
    lse_p[(hold * MT + f) * 2 + 1] = rs[j];
  }
  __syncthreads();
  // rank of each own entry among the four lists; entries ranked below k are
  // the proposals
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int f = wn * 64 + j * 32 + l32;
    const int64_t fr = m0 + f;
    float M = -INFINITY;
#pragma unroll
    for (int o = 0; o < 4; ++o) M = fmaxf(M, lse_p[(o * MT + f) * 2]);
    float S = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const float mo = lse_p[(o * MT + f) * 2], so = lse_p[(o * MT + f) * 2 + 1];
      if (so > 0.0f) S += so * __expf(mo - M);
    }
    const float lse = M + __logf(S);
    float ms = 0.0f;
    if (fr < rows) {
#pragma unroll
      for (int q = 0; q < KM; ++q) {
        const float v = lv[j][q];
        const int c = li[j][q];
        if (c < 0) continue;  // list shorter than KM (fewer components)
        int rank = q;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          if (o == hold) continue;
          const float* ov = lvs + (o * MT + f) * KM;
          const int* oi = lis + (o * MT + f) * KM;
          for (int p = 0; p < KM; ++p) {
            const int oc = oi[p];
            if (oc < 0) break;
            const float ow = ov[p];
            if (ow > v || (ow == v && oc < c))
              ++rank;
            else
              break;  // the other list is sorted: no later entry beats v
          }
        }
        if (rank < k) {
          prop[(row0 + fr) * k + rank] = c;
          ms += __expf(v - lse);
        }
      }
    }
    mpart[hold * MT + f] = ms;
  }
  __syncthreads();
  int local = -1;
  if (tid < MT && m0 + tid < rows) {
    const int f = tid;
    const float ms = mpart[f] + mpart[MT + f] + mpart[2 * MT + f] + mpart[3 * MT + f];
    const int64_t g = row0 + m0 + f;
    mass[g] = ms;
    const bool isfb = !(ms >= min_mass);
    fb[g] = isfb ? 1 : 0;
    if (isfb) local = atomicAdd(&wg[0], 1);
  }
  __syncthreads();
  if (tid == 0) {
    const int nfb = wg[0];
    const int nrow = (int)min<int64_t>(MT, rows - m0);
    wg[1] = nfb ? atomicAdd(&counters[0], nfb) : 0;
    atomicAdd(&counters[1], (nrow - nfb) * k);
  }
  __syncthreads();
  if (local >= 0) fb_list[wg[1] + local] = (int)(row0 + m0 + tid);
}

// ------------------------------------------------- pruned alignment (Sec. 4.2)
// Diagonal-UBM log-likelihoods as one expanded-feature product per (frame,
// component): with x' = x - shift and mu' = mu - shift,
//   log w_c N(x; mu_c, diag(Sigma_c)) = g_c + sum_d b_cd x'_d + sum_d a_cd x'_d^2,
//   a = -1 / (2 s^2), b = mu' / s^2,
//   g = log w_c - D/2 log 2pi - 1/2 sum_d log s^2_cd - 1/2 sum_d mu'^2 / s^2,
// over the features (1, x'_1..x'_D, x'_1^2..x'_D^2).  Coefficients are stored
// chunk-major like the full-covariance ones: (c, k) at ((k/8) Cpad + c) 8 + k%8.
__global__ void k_diag_prepare(const double* __restrict__ w, const double* __restrict__ mu,
                               const double* __restrict__ cov, const float* __restrict__ shift,
                               int C, int Cpad, int D, int Kd8, float* __restrict__ Wd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Cpad) return;
  auto at = [&](int k) -> float& { return Wd[((size_t)(k >> 3) * Cpad + c) * 8 + (k & 7)]; };
  if (c >= C) {  // padding components: never among the best
    for (int k = 0; k < Kd8; ++k) at(k) = (k == 0) ? -1e30f : 0.0f;
    return;
  }
  double g = log(w[c]) - 0.5 * D * 1.8378770664093454836;
  for (int d = 0; d < D; ++d) {
    const double s2 = cov[((size_t)c * D + d) * D + d];
    const double m = mu[(size_t)c * D + d] - (double)shift[d];
    g -= 0.5 * log(s2) + 0.5 * m * m / s2;
    at(1 + d) = (float)(m / s2);
    at(1 + D + d) = (float)(-0.5 / s2);
  }
  at(0) = (float)g;
  for (int k = 1 + 2 * D; k < Kd8; ++k) at(k) = 0.0f;
}

// Diagonal-UBM scores of every (frame, component) on FP32 MFMA and the k best
// components per frame (ties to the lower index).  One workgroup per 128
// frames loops over all components 128 at a time (W chunks of 8 features
// staged through LDS as in k_frame_tile); after each 128-component tile the
// two lane-halves holding a frame insert the tile's scores that beat their
// KM-th into a sorted list in registers; at the end the two lists are merged
// by counting ranks in LDS.  prop[t][0..k): the k best, best first.
template <int KM>
__global__ void __launch_bounds__(256)
k_diag_topk(const float* __restrict__ X, int64_t F, int D, const float* __restrict__ shift,
            const float* __restrict__ Wd, int C, int Cpad, int Kd8,
            const uint16_t* __restrict__ pairs, int k, int* __restrict__ prop) {
  constexpr int FR = 32, FTD = 128, CTD = 128, NCBD = CTD / 32, WLDD = 12;
  extern __shared__ float smem[];
  float* Ws = smem;                                            // [2][CTD][WLDD]
  float* xs = smem + 2 * CTD * WLDD;                           // [FTD][D+1]
  uint32_t* prs = reinterpret_cast<uint32_t*>(xs + FTD * (D + 1));
  float* lvs = smem;                                           // after the loop: [2][FTD][KM]
  int* lis = reinterpret_cast<int*>(lvs + 2 * FTD * KM);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int DS = D + 1;
  const int64_t f0 = (int64_t)blockIdx.x * FTD;
  const int nq = Kd8 / 8;
  for (int i = tid; i < Kd8 / 2; i += 256) prs[i] = reinterpret_cast<const uint32_t*>(pairs)[i];
  for (int i = tid; i < FTD * DS; i += 256) {
    const int fr = i / DS, a = i - fr * DS;
    const int64_t g = f0 + fr;
    float v = (a == 0) ? 1.0f : 0.0f;
    if (a > 0 && g < F) v = X[g * D + (a - 1)] - shift[a - 1];
    xs[i] = v;
  }
  float lv[KM];
  int li[KM];
#pragma unroll
  for (int q = 0; q < KM; ++q) {
    lv[q] = -INFINITY;
    li[q] = -1;
  }
  const float* xw = xs + (wave * FR + l32) * DS;
  for (int c0 = 0; c0 < Cpad; c0 += CTD) {
    // two threads stage the 8 coefficients of one component
    float4 r0;
    auto gload = [&](int q) {
      r0 = *reinterpret_cast<const float4*>(Wd + ((size_t)q * Cpad + c0 + (tid >> 1)) * 8 +
                                             (tid & 1) * 4);
    };
    auto sstore = [&](int buf) {
      *reinterpret_cast<float4*>(Ws + (buf * CTD + (tid >> 1)) * WLDD + (tid & 1) * 4) = r0;
    };
    __syncthreads();  // the previous tile's stages are consumed
    gload(0);
    sstore(0);
    __syncthreads();
    floatx16 acc[NCBD];
#pragma unroll
    for (int cb = 0; cb < NCBD; ++cb) acc[cb] = floatx16{0};
    for (int q = 0; q < nq; ++q) {
      const int cur = q & 1;
      if (q + 1 < nq) gload(q + 1);
      const float* wb = Ws + (cur * CTD + l32) * WLDD + 4 * h;
      float4 wv[NCBD];
#pragma unroll
      for (int cb = 0; cb < NCBD; ++cb) wv[cb] = *reinterpret_cast<const float4*>(wb + cb * 32 * WLDD);
      const uint32_t pw0 = prs[4 * q + 2 * h], pw1 = prs[4 * q + 2 * h + 1];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const uint32_t pr = ((s2 < 2) ? pw0 : pw1) >> ((s2 & 1) * 16);
        const float bv = xw[pr & 0xff] * xw[(pr >> 8) & 0xff];
#pragma unroll
        for (int cb = 0; cb < NCBD; ++cb) {
          const float av = (s2 == 0) ? wv[cb].x : (s2 == 1) ? wv[cb].y : (s2 == 2) ? wv[cb].z : wv[cb].w;
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[cb], 0, 0, 0);
        }
      }
      if (q + 1 < nq) sstore(cur ^ 1);
      __syncthreads();
    }
    float tmax = -INFINITY;
#pragma unroll
    for (int cb = 0; cb < NCBD; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) tmax = fmaxf(tmax, acc[cb][r]);
    if (tmax > lv[KM - 1]) {
#pragma unroll
      for (int cb = 0; cb < NCBD; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float v = acc[cb][r];
          const int c = c0 + cb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
          if (c < C && v > lv[KM - 1]) {
#pragma unroll
            for (int q = KM - 1; q > 0; --q) {
              const float vp = lv[q - 1], vq = lv[q];
              const int ip = li[q - 1], iq = li[q];
              const bool up = v > vp;
              const bool atq = v > vq;
              lv[q] = up ? vp : (atq ? v : vq);
              li[q] = up ? ip : (atq ? c : iq);
            }
            if (v > lv[0]) {
              lv[0] = v;
              li[0] = c;
            }
          }
        }
    }
  }
  __syncthreads();  // stages dead: the lists reuse the memory
  const int f = wave * FR + l32;
#pragma unroll
  for (int q = 0; q < KM; ++q) {
    lvs[(h * FTD + f) * KM + q] = lv[q];
    lis[(h * FTD + f) * KM + q] = li[q];
  }
  __syncthreads();
  const int64_t g = f0 + f;
  if (g < F) {
    const float* ov = lvs + ((h ^ 1) * FTD + f) * KM;
    const int* oi = lis + ((h ^ 1) * FTD + f) * KM;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
      const float v = lv[q];
      const int c = li[q];
      if (c < 0) continue;
      int rank = q;
      for (int p = 0; p < KM; ++p) {
        const int oc = oi[p];
        if (oc < 0) break;
        const float ow = ov[p];
        if (ow > v || (ow == v && oc < c))
          ++rank;
        else
          break;
      }
      if (rank < k) prop[g * k + rank] = c;
    }
  }
}

// hist[b][c]: proposals of component c among the kept frames of block b
__global__ void __launch_bounds__(256)
k_sel_hist(int64_t F, int k, int C, const int* __restrict__ prop, const int* __restrict__ fb,
           int* __restrict__ hist) {
  extern __shared__ int hl[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) hl[c] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)b * HBS * k;
  const int64_t e1 = min(F * k, e0 + (int64_t)HBS * k);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    if (fb && fb[e / k]) continue;
    const int c = prop[e];
    if (c >= 0 && c < C) atomicAdd(&hl[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) hist[(size_t)b * C + c] = hl[c];
}

__global__ void __launch_bounds__(256)
k_sel_scatter(int64_t F, int k, int C, const int* __restrict__ prop, const int* __restrict__ fb,
              const int* __restrict__ base, int2* __restrict__ ent) {
  extern __shared__ int cur[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) cur[c] = base[(size_t)b * C + c];
  __syncthreads();
  const int64_t e0 = (int64_t)b * HBS * k;
  const int64_t e1 = min(F * k, e0 + (int64_t)HBS * k);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    if (fb && fb[e / k]) continue;
    const int c = prop[e];
    if (c >= 0 && c < C) {
      const int pos = atomicAdd(&cur[c], 1);
      ent[pos] = make_int2((int)e, c);
    }
  }
}

// thr[g] = (largest filter score of the frame's k proposals) - margin: the
// proposals at or above it are scored exactly (the test of k_sel_finalize)
__global__ void __launch_bounds__(256)
k_sel_thr(int64_t F, int k, const float* __restrict__ score, float margin,
          float* __restrict__ thr) {
  const int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (g >= F) return;
  float M = -INFINITY;
  for (int s = 0; s < k; ++s) M = fmaxf(M, score[g * k + s]);
  thr[g] = M - margin;
}

__device__ inline int sel_kept(int64_t e, int k, int C, const int* __restrict__ prop,
                               const int* __restrict__ fb, const float* __restrict__ score,
                               const float* __restrict__ thr) {
  const int64_t g = e / k;
  if (fb && fb[g]) return -1;
  const int c = prop[e];
  return (c >= 0 && c < C && score[e] >= thr[g]) ? c : -1;
}

// bucket the kept (frame, proposal) slots by component (as k_sel_hist /
// k_sel_scatter, restricted to the slots within the margin)
__global__ void __launch_bounds__(256)
k_kept_hist(int64_t F, int k, int C, const int* __restrict__ prop, const int* __restrict__ fb,
            const float* __restrict__ score, const float* __restrict__ thr,
            int* __restrict__ hist) {
  extern __shared__ int hl[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) hl[c] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)b * HBS * k;
  const int64_t e1 = min(F * k, e0 + (int64_t)HBS * k);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = sel_kept(e, k, C, prop, fb, score, thr);
    if (c >= 0) atomicAdd(&hl[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) hist[(size_t)b * C + c] = hl[c];
}

__global__ void __launch_bounds__(256)
k_kept_scatter(int64_t F, int k, int C, const int* __restrict__ prop, const int* __restrict__ fb,
               const float* __restrict__ score, const float* __restrict__ thr,
               const int* __restrict__ base, int2* __restrict__ ent) {
  extern __shared__ int cur[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < C; c += 256) cur[c] = base[(size_t)b * C + c];
  __syncthreads();
  const int64_t e0 = (int64_t)b * HBS * k;
  const int64_t e1 = min(F * k, e0 + (int64_t)HBS * k);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = sel_kept(e, k, C, prop, fb, score, thr);
    if (c >= 0) ent[atomicAdd(&cur[c], 1)] = make_int2((int)e, c);
  }
}

// FP32 shifted-form score cst_c - 1/2 ||L_c^-1 (x - mu_c)||^2 of every
// (frame, proposal) pair, pairs sorted by component.  The wave handles one
// component at a time (a wave-uniform index), so mu_c and L_c^-1 (FP32, rows
// packed: row i holds columns 0..i) come through the scalar cache.  Used only
// to pick the pairs that get the exact FP64 score.
__global__ void __launch_bounds__(256)
k_sel_score(const float* __restrict__ X, int D, int k, const int* __restrict__ coff, int C,
            const int2* __restrict__ ent, int64_t cap, const double* __restrict__ mu,
            const float* __restrict__ linv32r, const double* __restrict__ cst,
            float* __restrict__ score) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = coff[C];
  const bool valid = e < total && e < cap;
  const int2 en = valid ? ent[e] : make_int2(0, -1);
  const int Dp = D * (D + 1) / 2;
  bool todo = valid;
  float my = 0.0f;  // stored after the loop: no store may precede the scalar loads
  float xr[64];
  {
    const float* xp = X + (int64_t)(valid ? en.x / k : 0) * D;
#pragma unroll
    for (int j = 0; j < 64; ++j) xr[j] = (valid && j < D) ? xp[j] : 0.0f;
  }
  while (true) {
    const uint64_t pend = __ballot(todo);
    if (pend == 0) break;
    const int src = __ffsll((unsigned long long)pend) - 1;
    const int cu = __builtin_amdgcn_readfirstlane(__shfl(en.y, src));
    // every lane computes component cu (uniform control flow keeps the
    // loads of mu_c and L_c scalar); the lanes that hold it keep the result
    const double* mc = mu + (size_t)cu * D;
    const float* L = linv32r + (size_t)cu * Dp;
    float dv[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) dv[j] = (j < D) ? (float)((double)xr[j] - mc[j]) : 0.0f;
    float q = 0.0f;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      if (i < D) {
        const float* Li = L + i * (i + 1) / 2;
        float y = 0.0f;
#pragma unroll
        for (int j = 0; j <= i; ++j) y = fmaf(Li[j], dv[j], y);
        q = fmaf(y, y, q);
      }
    }
    if (todo && en.y == cu) {
      todo = false;
      my = (float)cst[cu] - 0.5f * q;
    }
  }
  if (valid) score[en.x] = my;
}

// One wave per frame: FP64 exact scores of the proposals within `margin` of
// the frame's best filter score, posteriors renormalised over them, the KP
// largest kept.  Fallback frames are left to the all-component path.
__global__ void __launch_bounds__(256)
k_sel_finalize(const float* __restrict__ X, int64_t F, int D, int C, int k,
               const int* __restrict__ prop, const int* __restrict__ fb,
               const float* __restrict__ score, const double* __restrict__ lscore, float margin,
               float prune, int* __restrict__ post_idx, float* __restrict__ post_val,
               double* __restrict__ frame_ll, int* __restrict__ err) {
  __shared__ double lsh[4][32];
  __shared__ int ish[4][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = (int64_t)blockIdx.x * 4 + wave;
  if (g >= F) return;  // wave-uniform
  if (fb && fb[g]) return;
  int c = -1;
  float sc = -INFINITY;
  if (lane < k) {
    c = prop[g * k + lane];
    sc = score[g * k + lane];
    if (c < 0 || c >= C) c = -1;
  }
  float M = sc;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) M = fmaxf(M, __shfl_xor(M, o));
  const float thr = M - margin;
  const int cin = (c >= 0 && sc >= thr) ? c : -1;
  int m = 0;
  for (int s = 0; s < k; ++s) {
    const int cs = __shfl(cin, s);
    if (cs < 0) continue;
    const double l = lscore[g * k + s];  // exact FP64 (k_exact_sorted)
    if (lane == 0) {  // sorted insertion, largest first
      int pos = m;
      while (pos > 0 && lsh[wave][pos - 1] < l) {
        lsh[wave][pos] = lsh[wave][pos - 1];
        ish[wave][pos] = ish[wave][pos - 1];
        --pos;
      }
      lsh[wave][pos] = l;
      ish[wave][pos] = cs;
    }
    ++m;
  }
  __builtin_amdgcn_wave_barrier();
  double se = 0.0;
  const double mx = (m > 0) ? lsh[wave][0] : -INFINITY;
  for (int s = 0; s < m; ++s) se += exp(lsh[wave][s] - mx);
  const double lse = mx + log(se);
  // pruning (prune > 0): posteriors below `prune` are dropped and the rest
  // renormalised; the list is sorted, so the kept entries are a prefix
  int mk = m < KP ? m : KP;
  double norm = 1.0;
  if (prune > 0.0f) {
    int np = 0;
    double kept = 0.0;
    for (int s = 0; s < m; ++s) {
      const double gs = exp(lsh[wave][s] - lse);
      if (gs >= (double)prune) {
        ++np;
        kept += gs;
      }
    }
    if (lane == 0 && np > KP) raise_error(err, IVX_ECAPACITY, PK_SEL_SCORE, (int)g);
    mk = np < KP ? np : KP;
    norm = kept;
  }
  if (lane == 0) {
    if (!isfinite(lse)) raise_error(err, IVX_ENUMERIC, PK_SEL_SCORE, (int)g);
    if (prune <= 0.0f && m > KP) {
      double kept = 0.0;
      for (int s = 0; s < KP; ++s) kept += exp(lsh[wave][s] - lse);
      if (1.0 - kept > kMaxDroppedMass) raise_error(err, IVX_ECAPACITY, PK_SEL_SCORE, (int)g);
    }
  }
  if (lane < KP) {
    int id = -1;
    float v = 0.0f;
    if (lane < mk) {
      id = ish[wave][lane];
      v = (float)(exp(lsh[wave][lane] - lse) / norm);
    }
    if (post_idx) post_idx[g * KP + lane] = id;
    if (post_val) post_val[g * KP + lane] = v;
  }
  if (lane == 0 && frame_ll) frame_ll[g] = lse;
}

__global__ void k_gather_rows(const float* __restrict__ X, int D, const int* __restrict__ list,
                              const int* __restrict__ count, int64_t cap, float* __restrict__ out) {
  const int64_t n = min<int64_t>(count[0], cap) * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / D, d = i - r * D;
    out[i] = X[(int64_t)list[r] * D + d];
  }
}

__global__ void k_zero_f64(double* __restrict__ p) {
  if (threadIdx.x == 0) p[0] = 0.0;
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// FP32 master parameters -> the BF16 inference layouts.
__global__ void k_sel_pack(const float* __restrict__ param, int D, int H1, int H2, int C, int Cpad,
                           int64_t oW1, int64_t oW2, int64_t oW3, int64_t ob3,
                           __bf16* __restrict__ W1b, __bf16* __restrict__ W2b,
                           __bf16* __restrict__ W3b, float* __restrict__ b3p) {
  const int64_t n1 = (int64_t)H1 * 64, n2 = (int64_t)H2 * H1, n3 = (int64_t)Cpad * H2;
  const int64_t tot = n1 + n2 + n3 + Cpad;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      const int64_t r = i / 64, d = i % 64;
      W1b[i] = (__bf16)((d < D) ? param[oW1 + r * D + d] : 0.0f);
    } else if (i < n1 + n2) {
      const int64_t j = i - n1;
      W2b[j] = (__bf16)param[oW2 + j];
    } else if (i < n1 + n2 + n3) {
      const int64_t j = i - n1 - n2;
      const int64_t c = j / H2;
      W3b[j] = (__bf16)((c < C) ? param[oW3 + j] : 0.0f);
    } else {
      const int64_t c = i - n1 - n2 - n3;
      b3p[c] = (c < C) ? param[ob3 + c] : 0.0f;
    }
  }
}

// ------------------------------------------------------------------ training
__global__ void k_train_gather(const float* __restrict__ X, int D, const int64_t* __restrict__ fidx,
                               int B, int64_t F, const float* __restrict__ mean,
                               const float* __restrict__ istd, float* __restrict__ xs,
                               int* __restrict__ err) {
  const int64_t n = (int64_t)B * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / D, d = i - b * D;
    int64_t t = fidx[b];
    if (t < 0 || t >= F) {
      if (d == 0) raise_error(err, IVX_EINVAL, PK_SEL_TRAIN, (int)b);
      t = 0;
    }
    xs[i] = (X[t * D + d] - mean[d]) * istd[d];
  }
}

// a[b][n] += bias[n]; h = relu(a) (or h = a when relu == 0)
__global__ void k_bias_act(float* __restrict__ a, int64_t B, int N, const float* __restrict__ bias,
                           int relu, float* __restrict__ h) {
  const int64_t n = B * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = a[i] + bias[i % N];
    a[i] = v;
    if (h) h[i] = relu ? fmaxf(v, 0.0f) : v;
  }
}

__device__ inline float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per training row: dz = (softmax(z) * sum(gamma) - gamma) / B and
// the row's cross-entropy -sum_c gamma_c log q_c / B (into loss_part[b]).
__global__ void __launch_bounds__(256)
k_softmax_xent(const float* __restrict__ z, int B, int C, int64_t F,
               const int64_t* __restrict__ fidx,
               const int* __restrict__ post_idx, const float* __restrict__ post_val,
               float* __restrict__ dz, double* __restrict__ loss_part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + wave;
  if (b >= B) return;  // wave-uniform
  const float* zr = z + (int64_t)b * C;
  float* dr = dz + (int64_t)b * C;
  float mx = -INFINITY;
  for (int c = lane; c < C; c += 64) mx = fmaxf(mx, zr[c]);
  mx = wave_max_f(mx);
  float se = 0.0f;
  for (int c = lane; c < C; c += 64) se += expf(zr[c] - mx);
  se = wave_sum_f(se);
  const float lse = mx + logf(se);
  int64_t t = fidx[b];
  if (t < 0 || t >= F) t = 0;  // reported by k_train_gather
  int ci = -1;
  float gv = 0.0f;
  if (lane < KP) {
    ci = post_idx[t * KP + lane];
    gv = (ci >= 0 && ci < C) ? post_val[t * KP + lane] : 0.0f;
    if (ci >= C) ci = -1;
  }
  const float gs = wave_sum_f(gv);
  const float inv = 1.0f / (float)B;
  for (int c = lane; c < C; c += 64) dr[c] = expf(zr[c] - lse) * gs * inv;
  __builtin_amdgcn_wave_barrier();
  __threadfence_block();
  if (ci >= 0) dr[ci] -= gv * inv;
  const double part = (ci >= 0) ? -(double)gv * ((double)zr[ci] - (double)lse) : 0.0;
  double tot = part;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o);
  if (lane == 0) loss_part[b] = tot / (double)B;
}

__global__ void k_relu_grad(float* __restrict__ d, const float* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!(a[i] > 0.0f)) d[i] = 0.0f;
}

// Column sums of d [B][N] in two deterministic passes: 32 row blocks write
// partial sums, then one thread per column adds them.
constexpr int CS_PARTS = 32;
__global__ void k_colsum_part(const float* __restrict__ d, int B, int N, float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int p = blockIdx.y;
  const int b0 = (int)((int64_t)B * p / CS_PARTS), b1 = (int)((int64_t)B * (p + 1) / CS_PARTS);
  float s = 0.0f;
  for (int b = b0; b < b1; ++b) s += d[(int64_t)b * N + n];
  part[(int64_t)p * N + n] = s;
}

__global__ void k_colsum_final(const float* __restrict__ part, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int p = 0; p < CS_PARTS; ++p) s += part[(int64_t)p * N + n];
  out[n] = s;
}

// Adam (Kingma and Ba, 2015) on the flat FP32 parameter vector.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Global feature mean and standard deviation (FP64 sums), one thread per dim.
__global__ void __launch_bounds__(256)
k_feature_stats(const float* __restrict__ X, int64_t F, int D, float* __restrict__ mean,
                float* __restrict__ stdv) {
  __shared__ double s1[256], s2[256];
  const int d = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t t = threadIdx.x; t < F; t += 256) {
    const double x = X[t * D + d];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)F;
    const double var = s2[0] / (double)F - mu * mu;
    mean[d] = (float)mu;
    stdv[d] = (float)sqrt(var > 0.0 ? var : 0.0);
  }
}

__global__ void k_inv_std(const float* __restrict__ stdv, int D, float* __restrict__ istd,
                          int* __restrict__ err) {
  const int d = threadIdx.x;
  if (d >= D) return;
  const float s = stdv[d];
  if (!(s > 0.0f) || !isfinite(s)) {
    raise_error(err, IVX_EINVAL, PK_SEL_TRAIN, d);
    istd[d] = 0.0f;
  } else {
    istd[d] = 1.0f / s;
  }
}

size_t l3_lds_bytes(int km) {
  const size_t stages = sizeof(__bf16) * 2 * (MT + NT) * LDK;
  const size_t lists = sizeof(float) * 4 * MT * km * 2 + sizeof(float) * 4 * MT * 3 + 2 * sizeof(int);
  return std::max(stages, lists);
}

int l3_km(int k) { return k <= 8 ? 8 : (k <= 20 ? 20 : 32); }

size_t diag_lds_bytes(int D, int Kd8, int km) {
  const size_t stage = sizeof(float) * (2 * 128 * 12 + 128 * (D + 1)) + sizeof(uint16_t) * Kd8;
  const size_t lists = sizeof(float) * 2 * 128 * km * 2;
  return std::max(stage, lists);
}

}  // namespace

bool select_set_attributes() {
  bool ok = true;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_diag_topk<32>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)diag_lds_bytes(63, 128, 32)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_diag_topk<20>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)diag_lds_bytes(63, 128, 20)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_diag_topk<8>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)diag_lds_bytes(63, 128, 8)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_l3<8>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)l3_lds_bytes(8)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_l3<20>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)l3_lds_bytes(20)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_l3<32>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)l3_lds_bytes(32)) == hipSuccess;
  return ok;
}

// ------------------------------------------------------------------ launchers
void launch_selector_pack(ivx_ctx* ctx, hipStream_t s) {
  Selector& S = *ctx->sel;
  k_sel_pack<<<2048, 256, 0, s>>>(S.param, ctx->D, S.H1, S.H2, ctx->C, ctx->Cpad, S.oW1, S.oW2,
                                  S.oW3, S.ob3, S.W1b, S.W2b, S.W3b, S.b3p);
}

void launch_feature_stats(ivx_ctx* ctx, const float* X, int64_t F, float* mean, float* stdv,
                          hipStream_t s) {
  k_feature_stats<<<ctx->D, 256, 0, s>>>(X, F, ctx->D, mean, stdv);
}

void launch_selector_inv_std(ivx_ctx* ctx, hipStream_t s) {
  Selector& S = *ctx->sel;
  k_inv_std<<<1, 64, 0, s>>>(S.stdv, ctx->D, S.istd, ctx->dev_err);
}

// MLP forward over frames [0, F) with proposals, masses and the fallback
// list; optional copies of h1, h2 (BF16 bits) and z for inspection.  Returns
// false when one of those copies could not be queued.
bool launch_selector_mlp(ivx_ctx* ctx, const float* X, int64_t F, uint16_t* h1_out,
                         uint16_t* h2_out, float* z_out, hipStream_t s) {
  Selector& S = *ctx->sel;
  k_fill_i32<<<1, 64, 0, s>>>(S.counters, 4, 0);
  for (int64_t r0 = 0; r0 < F; r0 += S.chunk) {
    const int64_t rows = std::min<int64_t>(S.chunk, F - r0);
    const unsigned mb = (unsigned)((rows + MT - 1) / MT);
    {
      ProfScope ps(ctx, PK_SEL_MLP, s);
      k_mlp_nt<true><<<dim3(S.H1 / NT, mb), 256, 0, s>>>(X + r0 * ctx->D, ctx->D, S.mean, S.istd,
                                                         nullptr, rows, 64, S.W1b, S.param + S.ob1,
                                                         S.H1, S.h1b);
      k_mlp_nt<false><<<dim3(S.H2 / NT, mb), 256, 0, s>>>(nullptr, ctx->D, nullptr, nullptr,
                                                          S.h1b, rows, S.H1, S.W2b,
                                                          S.param + S.ob2, S.H2, S.h2b);
      const int km = l3_km(S.k);
      float* zo = z_out ? z_out + r0 * ctx->C : nullptr;
#define IVX_L3(KMV)                                                                          \
  k_mlp_l3<KMV><<<mb, 256, l3_lds_bytes(KMV), s>>>(S.h2b, rows, r0, S.H2, S.W3b, S.b3p, ctx->C, \
                                                   ctx->Cpad, S.k, S.min_mass, S.prop, S.mass, \
                                                   S.fb, S.fb_list, S.counters, zo)
      if (km == 8)
        IVX_L3(8);
      else if (km == 20)
        IVX_L3(20);
      else
        IVX_L3(32);
#undef IVX_L3
    }
    if (h1_out && hipMemcpyAsync(h1_out + r0 * S.H1, S.h1b, sizeof(uint16_t) * rows * S.H1,
                                 hipMemcpyDeviceToDevice, s) != hipSuccess)
      return false;
    if (h2_out && hipMemcpyAsync(h2_out + r0 * S.H2, S.h2b, sizeof(uint16_t) * rows * S.H2,
                                 hipMemcpyDeviceToDevice, s) != hipSuccess)
      return false;
  }
  return true;
}

// Exact FP64 scores of the proposals within the margin of each frame's best
// filter score, bucketed by component and scored by k_exact_sorted (the
// sort buffers of the filter pass are reused).
static void exact_kept(ivx_ctx* ctx, const float* X, int64_t F, int k, const int* prop, const int* fb,
                const float* score, float margin, float* thr, int* hist, int* coff, int2* ent,
                double* lscore, hipStream_t s) {
  k_sel_thr<<<(unsigned)((F + 255) / 256), 256, 0, s>>>(F, k, score, margin, thr);
  const int nb = (int)((F + HBS - 1) / HBS);
  const size_t ldsc = sizeof(int) * ctx->C;
  k_kept_hist<<<nb, 256, ldsc, s>>>(F, k, ctx->C, prop, fb, score, thr, hist);
  launch_hist_scan(nb, ctx->C, hist, coff, s);
  k_kept_scatter<<<nb, 256, ldsc, s>>>(F, k, ctx->C, prop, fb, score, thr, hist, ent);
  launch_exact_sorted(ctx, ent, coff, k, X, lscore, s);
}

void launch_select_learned(ivx_ctx* ctx, const float* X, int64_t F, int prec, int* post_idx,
                           float* post_val, double* frame_ll, hipStream_t s) {
  if (F <= 0) return;
  Selector& S = *ctx->sel;
  (void)launch_selector_mlp(ctx, X, F, nullptr, nullptr, nullptr, s);  // no copies asked for
  {
    ProfScope ps(ctx, PK_SEL_SCORE, s);
    const int nb = (int)((F + HBS - 1) / HBS);
    const size_t ldsc = sizeof(int) * ctx->C;
    k_sel_hist<<<nb, 256, ldsc, s>>>(F, S.k, ctx->C, S.prop, S.fb, S.hist);
    launch_hist_scan(nb, ctx->C, S.hist, S.coff, s);
    k_sel_scatter<<<nb, 256, ldsc, s>>>(F, S.k, ctx->C, S.prop, S.fb, S.hist, S.ent);
    const int64_t cap = F * S.k;
    k_sel_score<<<(unsigned)((cap + 255) / 256), 256, 0, s>>>(
        X, ctx->D, S.k, S.coff, ctx->C, S.ent, cap, ctx->mu, ctx->linv32r, ctx->cst, S.score);
    exact_kept(ctx, X, F, S.k, S.prop, S.fb, S.score, S.margin, S.thr, S.hist, S.coff, S.ent,
               S.lscore, s);
    k_sel_finalize<<<(unsigned)((F + 3) / 4), 256, 0, s>>>(
        X, F, ctx->D, ctx->C, S.k, S.prop, S.fb, S.score, S.lscore, S.margin, 0.0f, post_idx,
        post_val, frame_ll, ctx->dev_err);
  }
  // fallback frames: all components, results written at their own rows
  k_gather_rows<<<2048, 256, 0, s>>>(X, ctx->D, S.fb_list, S.counters, F, S.xfb);
  launch_frame_select(ctx, S.xfb, F, prec, s, S.counters);
  launch_rescore(ctx, S.xfb, F, prec, post_idx, post_val, frame_ll, s, S.counters, S.fb_list);
}

// Pruned alignment (Sec. 4.2) for frames [0, F): diagonal-UBM top-k,
// full-covariance scores of the k (FP32 filter, FP64 within the margin),
// posteriors over them, entries below `prune` dropped, the rest renormalised.
void launch_select_pruned(ivx_ctx* ctx, const float* X, int64_t F, int* post_idx, float* post_val,
                          double* frame_ll, hipStream_t s) {
  if (F <= 0) return;
  Presel& P = *ctx->presel;
  {
    ProfScope ps(ctx, PK_SEL_MLP, s);
    k_diag_prepare<<<(ctx->Cpad + 255) / 256, 256, 0, s>>>(ctx->w, ctx->mu, ctx->cov, ctx->shift,
                                                           ctx->C, ctx->Cpad, ctx->D, P.Kd8, P.Wd);
    const int km = l3_km(P.k);
    const unsigned nb = (unsigned)((F + 127) / 128);
    const size_t lds = diag_lds_bytes(ctx->D, P.Kd8, km);
#define IVX_DIAG(KMV)                                                                          \
  k_diag_topk<KMV><<<nb, 256, lds, s>>>(X, F, ctx->D, ctx->shift, P.Wd, ctx->C, ctx->Cpad,      \
                                        P.Kd8, P.pairs, P.k, P.prop)
    if (km == 8)
      IVX_DIAG(8);
    else if (km == 20)
      IVX_DIAG(20);
    else
      IVX_DIAG(32);
#undef IVX_DIAG
  }
  ProfScope ps(ctx, PK_SEL_SCORE, s);
  const int nb = (int)((F + HBS - 1) / HBS);
  const size_t ldsc = sizeof(int) * ctx->C;
  k_sel_hist<<<nb, 256, ldsc, s>>>(F, P.k, ctx->C, P.prop, nullptr, P.hist);
  launch_hist_scan(nb, ctx->C, P.hist, P.coff, s);
  k_sel_scatter<<<nb, 256, ldsc, s>>>(F, P.k, ctx->C, P.prop, nullptr, P.hist, P.ent);
  const int64_t cap = F * P.k;
  k_sel_score<<<(unsigned)((cap + 255) / 256), 256, 0, s>>>(
      X, ctx->D, P.k, P.coff, ctx->C, P.ent, cap, ctx->mu, ctx->linv32r, ctx->cst, P.score);
  exact_kept(ctx, X, F, P.k, P.prop, nullptr, P.score, P.margin, P.thr, P.hist, P.coff, P.ent,
             P.lscore, s);
  k_sel_finalize<<<(unsigned)((F + 3) / 4), 256, 0, s>>>(
      X, F, ctx->D, ctx->C, P.k, P.prop, nullptr, P.score, P.lscore, P.margin, P.prune, post_idx,
      post_val, frame_ll, ctx->dev_err);
}

// Gradients of the soft-target cross-entropy over a batch of B frames into
// S.grad (flat, the parameter layout), and the mean loss into loss[0].
bool launch_selector_grad(ivx_ctx* ctx, const float* X, int64_t F, const int64_t* fidx, int B,
                          const int* post_idx, const float* post_val, double* loss,
                          hipStream_t s) {
  Selector& S = *ctx->sel;
  const int D = ctx->D, C = ctx->C, H1 = S.H1, H2 = S.H2;
  float* P = S.param;
  float* G = S.grad;
  ProfScope ps(ctx, PK_SEL_TRAIN, s);
  auto colsum = [&](const float* d, int N, float* out) {
    k_colsum_part<<<dim3((N + 255) / 256, CS_PARTS), 256, 0, s>>>(d, B, N, S.colpart);
    k_colsum_final<<<(N + 255) / 256, 256, 0, s>>>(S.colpart, N, out);
  };
  k_train_gather<<<256, 256, 0, s>>>(X, D, fidx, B, F, S.mean, S.istd, S.xs, ctx->dev_err);
  bool ok = true;
  auto gemm = [&](const float* A, int64_t lda, bool ta, const float* Bm, int64_t ldb, bool tb,
                  float* Cm, int64_t ldc, int M, int N, int K) {
    GemmArgs g;
    g.A = A;
    g.B = Bm;
    g.C = Cm;
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.K = K;
    ok = ok && gemm_f32(g, ta, tb, GEMM_STORE, 1, s);
  };
  // forward: a1 = xs W1^T + b1, h1 = relu(a1), ...
  gemm(S.xs, D, false, P + S.oW1, D, true, S.a1, H1, B, H1, D);
  k_bias_act<<<512, 256, 0, s>>>(S.a1, B, H1, P + S.ob1, 1, S.h1);
  gemm(S.h1, H1, false, P + S.oW2, H1, true, S.a2, H2, B, H2, H1);
  k_bias_act<<<512, 256, 0, s>>>(S.a2, B, H2, P + S.ob2, 1, S.h2);
  gemm(S.h2, H2, false, P + S.oW3, H2, true, S.z, C, B, C, H2);
  k_bias_act<<<1024, 256, 0, s>>>(S.z, B, C, P + S.ob3, 0, nullptr);
  k_softmax_xent<<<(B + 3) / 4, 256, 0, s>>>(S.z, B, C, F, fidx, post_idx, post_val, S.dz,
                                             S.loss_part);
  // backward
  gemm(S.dz, C, true, S.h2, H2, false, G + S.oW3, H2, C, H2, B);        // dW3 = dz^T h2
  colsum(S.dz, C, G + S.ob3);
  gemm(S.dz, C, false, P + S.oW3, H2, false, S.dh2, H2, B, H2, C);      // dh2 = dz W3
  k_relu_grad<<<512, 256, 0, s>>>(S.dh2, S.a2, (int64_t)B * H2);
  gemm(S.dh2, H2, true, S.h1, H1, false, G + S.oW2, H1, H2, H1, B);     // dW2 = da2^T h1
  colsum(S.dh2, H2, G + S.ob2);
  gemm(S.dh2, H2, false, P + S.oW2, H1, false, S.dh1, H1, B, H1, H2);   // dh1 = da2 W2
  k_relu_grad<<<512, 256, 0, s>>>(S.dh1, S.a1, (int64_t)B * H1);
  gemm(S.dh1, H1, true, S.xs, D, false, G + S.oW1, D, H1, D, B);        // dW1 = da1^T xs
  colsum(S.dh1, H1, G + S.ob1);
  if (loss) {
    k_zero_f64<<<1, 64, 0, s>>>(loss);
    launch_sum_f64(ctx, S.loss_part, B, loss, s);
  }
  return ok;
}

void launch_selector_adam(ivx_ctx* ctx, float lr, hipStream_t s) {
  Selector& S = *ctx->sel;
  S.step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)S.step), c2 = 1.0f - powf(b2, (float)S.step);
  k_adam<<<1024, 256, 0, s>>>(S.param, S.grad, S.adam_m, S.adam_v, S.P, lr, b1, b2, 1e-8f, c1, c2);
  launch_selector_pack(ctx, s);
}

}  // namespace ivx
