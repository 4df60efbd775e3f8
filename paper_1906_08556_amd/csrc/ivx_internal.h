// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ivx.h"

namespace ivx {

// Posterior list capacity per frame (entries of post_idx / post_val).
constexpr int KP = 16;
constexpr int CSPLIT = 16;  // row chunks of the accumulator column sums
// Candidate margin in nats: components whose log-likelihood is more than
// margin(C) = ln C + 16.64 + 2 below the frame's best are dropped.  Their
// total posterior mass is then below C e^-margin = 2^-24 e^-2, under the FP32
// rounding of the kept posteriors; the extra 2 nats absorb the error of the
// FP32 expanded-form filter (<= 0.4 nats measured on the workload).
inline float candidate_margin(int C) { return logf((float)C) + 18.64f; }
// The BF16 split-form filter is off by up to ~3 nats on the workload
// (measured against FP64); its margin carries 16 nats of allowance instead of 2.
inline float candidate_margin_bf16(int C) { return logf((float)C) + 16.64f + 16.0f; }
// Largest posterior mass a frame may lose when more than KP components lie
// within the margin (the top KP by exact score are kept); beyond it the frame
// raises IVX_ECAPACITY.
constexpr double kMaxDroppedMass = 1e-6;
// Largest number of proposals per frame of the learned selection.
constexpr int kMaxProposals = 32;
// Margin of the learned selection's FP32 shifted-form filter: the proposals
// more than ln k + 16.64 + 2 nats below the frame's best carry less than
// 2^-24 e^-2 of its mass; the filter itself is off by far less than 2 nats.
inline float selection_margin(int k) { return logf((float)k) + 18.64f; }
// Tile size of the tile-packed symmetric layout.
constexpr int TB = 16;

// Kernel groups timed by the opt-in event profiler (ivx_profile_*).
enum ProfKernel {
  PK_FRAME_SELECT = 0,  // expanded-feature MFMA GEMM + running max + candidates
  PK_RESCORE,           // FP64 candidate rescoring and posteriors
  PK_STATS_NF,          // n, f
  PK_STATS_S,           // second-order statistics
  PK_TV_PREP,           // V_c, U_c
  PK_ESTEP_GEMM,        // precision assembly + linear term GEMMs
  PK_ESTEP_CHOL,        // per-utterance Cholesky, solve, inverse
  PK_ACCUM,             // M-step accumulator GEMMs and sums
  PK_MSTEP,             // FP64 M-step solve and objective
  PK_MINDIV,            // minimum divergence
  PK_UBM,               // UBM preparation / realignment
  PK_SEL_MLP,           // learned selection: network forward and top-k
  PK_SEL_SCORE,         // learned selection: pair sort, filter and exact scores
  PK_SEL_TRAIN,         // learned selection: training gradients
  PK_COUNT
};

inline int64_t tp_size(int R) {
  int64_t nb = (R + TB - 1) / TB;
  return nb * (nb + 1) / 2 * TB * TB;
}

// State of the learned Gaussian selection: parameters (flat FP32 master
// vector W1 [H1][D], b1 [H1], W2 [H2][H1], b2 [H2], W3 [C][H2], b3 [C]), Adam
// moments, BF16 inference copies and workspace.  Owned by the context.
struct Selector {
  int H1 = 0, H2 = 0, k = 0, Bmax = 0;
  float min_mass = 0.99f;
  float margin = 0.0f;
  int64_t P = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  int64_t chunk = 0;  // frames per network pass
  int step = 0;       // Adam steps taken
  float* param = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* mean = nullptr;  // [D]
  float* stdv = nullptr;  // [D]
  float* istd = nullptr;  // [D]
  __bf16* W1b = nullptr;  // [H1][64], features padded with zeros
  __bf16* W2b = nullptr;  // [H2][H1]
  __bf16* W3b = nullptr;  // [Cpad][H2], padding components zero
  float* b3p = nullptr;   // [Cpad]
  __bf16* h1b = nullptr;  // [chunk][H1]
  __bf16* h2b = nullptr;  // [chunk][H2]
  int* prop = nullptr;    // [maxF][k] proposals, largest logit first
  float* mass = nullptr;  // [maxF] the network's softmax mass on its proposals
  int* fb = nullptr;      // [maxF] 1 = all-component fallback
  int* fb_list = nullptr; // [maxF]
  int* counters = nullptr;  // [4]: fallback frames, kept (frame, proposal) pairs
  float* score = nullptr;   // [maxF][k] FP32 filter scores
  float* thr = nullptr;     // [maxF] the frame's best filter score minus the margin
  double* lscore = nullptr; // [maxF][k] exact FP64 scores of the kept proposals
  int* hist = nullptr;      // [maxF / 8192 + 1][C]
  int* coff = nullptr;      // [C + 1]
  int2* ent = nullptr;      // [maxF * k] (frame * k + slot, component), by component
  float* xfb = nullptr;     // [maxF][D] fallback frames, gathered
  // training, batch <= Bmax
  float* xs = nullptr;      // [Bmax][D]
  float* a1 = nullptr;      // [Bmax][H1]
  float* h1 = nullptr;
  float* a2 = nullptr;      // [Bmax][H2]
  float* h2 = nullptr;
  float* z = nullptr;       // [Bmax][C]
  float* dz = nullptr;
  float* dh1 = nullptr;     // [Bmax][H1]
  float* dh2 = nullptr;     // [Bmax][H2]
  double* loss_part = nullptr;  // [Bmax]
  float* colpart = nullptr;     // [32][max(C, H1, H2)] column-sum partials
};

// State of the pruned alignment (Sec. 4.2): diagonal-UBM coefficients and
// the scoring workspace.  Owned by the context.
struct Presel {
  int k = 20;
  float prune = 0.025f;
  float margin = 0.0f;
  int Kd8 = 0;              // 1 + 2D features rounded up to 8
  float* Wd = nullptr;      // [Kd8/8][Cpad][8] diagonal coefficients, chunk-major
  uint16_t* pairs = nullptr;  // [Kd8] feature index pairs (1, x_d, x_d^2)
  int* prop = nullptr;      // [maxF][k]
  float* score = nullptr;   // [maxF][k]
  float* thr = nullptr;     // [maxF] the frame's best filter score minus the margin
  double* lscore = nullptr; // [maxF][k] exact FP64 scores of the kept proposals
  int* hist = nullptr;      // [maxF / 8192 + 1][C]
  int* coff = nullptr;      // [C + 1]
  int2* ent = nullptr;      // [maxF * k]
};

// Records a message for ivx_last_error() (printf-style).
void set_error(const char* fmt, ...);

// Device-side error state ctx->dev_err[4]: [0] first error code, [1] smallest
// failing index reported with it (component / utterance), [2] the kernel group
// (ProfKernel) that raised the first error, [3] count of raising events.
__device__ inline void raise_error(int* err, int code, int source, int index = -1) {
  if (!err) return;
  if (atomicCAS(err, 0, code) == 0) err[2] = source;
  if (index >= 0) atomicMin(err + 1, index);
  atomicAdd(err + 3, 1);
}

}  // namespace ivx

struct ivx_ctx {
  int device = 0;
  int ncu = 0;     // compute units of the device (persistent grids)
  int C = 0, D = 0, R = 0;
  int maxU = 0;
  int64_t maxF = 0;
  int K = 0;       // expanded features (D+1)(D+2)/2
  int Kpad = 0;    // K rounded up to a multiple of 16
  int Cpad = 0;    // C rounded up to a multiple of 256 (frame GEMM tile)
  int Dp = 0;      // D(D+1)/2
  int64_t TP = 0;  // tile-packed size for R
  float margin = 0.0f;       // candidate margin (nats), FP32 filter
  float margin_bf16 = 0.0f;  // candidate margin (nats), BF16 split-form filter
  bool ubm_set = false;
  bool tv_set = false;

  // UBM, FP64 master copy
  double* w = nullptr;      // [C]
  double* mu = nullptr;     // [C][D]
  double* cov = nullptr;    // [C][D][D]
  // UBM-derived
  float* shift = nullptr;     // [D] global mean shift applied before expansion
  float* Wexp = nullptr;      // [Kpad/8][Cpad][8] expanded quadratic-form coefficients
  __bf16* W16 = nullptr;      // [Kpad/16][Cpad][32] the same as BF16 (16 hi, 16 lo per chunk)
  double* linv = nullptr;     // [C][Dp] L_c^{-1}, lower triangle column by column
  float* linv32r = nullptr;   // [C][Dp] L_c^{-1} in FP32, lower triangle row by row
  double* ldense = nullptr;   // [C][64][64] L_c^{-1} dense, column-major, zero-padded
  double* cst = nullptr;      // [C] log w_c - D/2 log 2pi - sum_i log L_c[i,i]
  uint16_t* pairs = nullptr;  // [Kpad] expanded-feature index pairs (a | b << 8)

  // TV model, FP64 master copy
  double* T = nullptr;      // [C][D][R]
  double* Sigma = nullptr;  // [C][D][D]
  double* p = nullptr;      // [R]
  // standard formulation (Sec. 2.1): bias m_c, statistics centred on it
  bool standard = false;
  double* bias = nullptr;   // [C][D]
  float* bias32 = nullptr;  // [C][D] FP32 copy for the first-order centring

  // frame-stage workspace
  int2* cand = nullptr;       // [maxF][KP] candidate (component, FP32 score bits)
  float* cM = nullptr;        // [maxF] running maximum of the FP32 scores
  int* cflag = nullptr;       // [maxF] candidate-list overflow
  int* post_idx = nullptr;    // [maxF][KP]
  float* post_val = nullptr;  // [maxF][KP]
  double* frame_ll = nullptr; // [maxF]
  double* lscore = nullptr;   // [maxF][KP] exact FP64 scores of the kept candidates
  int* hist = nullptr;        // [nhist][C]
  int* coff = nullptr;        // [C+1]
  int2* ent = nullptr;        // [maxF*KP] component-sorted (frame, gamma bits)
  double* partial = nullptr;  // [1024] reduction partials
  int nhist = 0;

  // TV-derived quantities (recomputed when the TV model changes)
  bool tv_dirty = true;
  float* Y32 = nullptr;       // [C][D][R] L_c^{-1} T_c
  float* V32 = nullptr;       // [C][D][R] Sigma_c^{-1} T_c
  float* Utp = nullptr;       // [C][TP]   T_c^T Sigma_c^{-1} T_c, tile-packed
  double* Psig = nullptr;     // [C][D][D] Sigma_c^{-1}
  double* sig_logdet = nullptr;  // [C]   log|Sigma_c|

  // utterance-batch workspace
  int nsplit_max = 64;
  float* Lbuf = nullptr;      // [maxU][TP] L(u) -> G -> Phi(u)
  float* Wbuf = nullptr;      // [maxU][TP] G^{-1}
  double* Psi64 = nullptr;    // [maxU][TP] Psi(u) = Phi(u) + phi phi^T (accumulate call)
  float* bpart = nullptr;     // [nsplit_max][maxU][R]
  double* colpart = nullptr;  // [CSPLIT][C + R + TP] column-sum partials
  float* bvec = nullptr;      // [maxU][R]
  double* llu = nullptr;      // [maxU]
  float* n_ws = nullptr;      // [maxU][C]   (extract_ivectors)
  unsigned long long* nf_acc = nullptr;  // [maxU][C][D+1] fixed-point n/f sums, kept at zero
  int* umap = nullptr;        // [maxF] frame -> utterance of the current batch
  float* f_ws = nullptr;      // [maxU][C][D]

  // M-step / minimum-divergence workspace
  double* Tnew = nullptr;     // [C][D][R]
  double* obj_part = nullptr; // [C]
  double* Gmat = nullptr;     // [R][R]
  double* Mmat = nullptr;     // [R][R]
  double* Winv = nullptr;     // [C][nb * 256] inverses of the diagonal Cholesky tiles (FP64 solves)
  // BF16 precision assembly: U^tp transposed and split hi / lo, [TP][Ck];
  // N split hi / lo, [maxU][Ck] (Ck = C rounded up to a multiple of 8)
  __bf16* Ut16hi = nullptr;
  __bf16* Ut16lo = nullptr;
  __bf16* n16hi = nullptr;
  __bf16* n16lo = nullptr;
  bool utp16_valid = false;
  double* mvec = nullptr;     // [4][R]
  int* mstat = nullptr;       // [C]

  int* dev_err = nullptr;     // [4]: see raise_error

  // launch shapes picked by the autotuner (ivx_autotune); defaults below
  ivx_tuning tune = {8, 8, 0, 0, 0, 0, 0};

  // learned Gaussian selection (ivx_selector_set), null until set
  ivx::Selector* sel = nullptr;
  // pruned alignment (ivx_pruned_set), null until set
  ivx::Presel* presel = nullptr;

  // event profiler (off unless ivx_profile_enable)
  bool prof_on = false;
  int prof_cap = 0, prof_used = 0;
  hipEvent_t* prof_ev = nullptr;  // [2 * prof_cap]
  int* prof_kind = nullptr;       // [prof_cap]
};

namespace ivx {
// Records a start event for kernel group k on stream s; returns a slot or -1.
int prof_begin(ivx_ctx* ctx, int k, hipStream_t s);
void prof_end(ivx_ctx* ctx, int slot, hipStream_t s);
struct ProfScope {
  ivx_ctx* ctx;
  hipStream_t s;
  int slot;
  ProfScope(ivx_ctx* c, int k, hipStream_t st) : ctx(c), s(st), slot(prof_begin(c, k, st)) {}
  ~ProfScope() { prof_end(ctx, slot, s); }
};
}  // namespace ivx

namespace ivx {

// ---- k_ubm.hip
void launch_ubm_prepare(ivx_ctx* ctx, hipStream_t s);
void launch_init_tv(ivx_ctx* ctx, const double* T_rand, double p0, hipStream_t s);
void launch_init_tv_standard(ivx_ctx* ctx, const double* T_rand, hipStream_t s);
void launch_bias32(ivx_ctx* ctx, hipStream_t s);
void launch_update_means(ivx_ctx* ctx, hipStream_t s);

// Target of the zeroth- and first-order statistics accumulated beside the
// posteriors: frame -> utterance map (k_frame_utt), utterance count, FP32
// bias of the standard formulation (or null) and the fixed-point sums
// [U][C][D+1] (k_nf.h).
struct NfTarget {
  const int* umap;
  int64_t U;
  const float* mb;
  unsigned long long* acc;
};

// ---- k_frame.hip
bool frame_set_attributes(const ivx_ctx* ctx);
bool mstep_set_attributes();
bool estep_rr_setup();
// Fdev (optional): device frame count, at most F, read by the kernels (the
// grid is sized for F).  fmap (optional): output row of compact frame i.
void launch_frame_select(ivx_ctx* ctx, const float* X, int64_t F, int prec, hipStream_t s,
                         const int* Fdev = nullptr);
// nf (optional): n/f of every frame's kept posteriors are added to nf->acc.
void launch_rescore(ivx_ctx* ctx, const float* X, int64_t F, int prec, int* post_idx,
                    float* post_val, double* frame_ll, hipStream_t s, const int* Fdev = nullptr,
                    const int* fmap = nullptr, const NfTarget* nf = nullptr);
void launch_dense_gamma(ivx_ctx* ctx, int64_t F, const int* post_idx, const float* post_val,
                        float* gamma, hipStream_t s);

// ---- k_stats.hip
// Frame -> utterance map of the batch in ctx->umap (offsets checked; bad
// ones raise IVX_EINVAL); returns the n/f target of the batch.
NfTarget launch_frame_utt(ivx_ctx* ctx, const int64_t* utt_off, int64_t U, int64_t F,
                          hipStream_t s);
// n/f sums of the posterior lists (paths whose posteriors are not produced
// by launch_rescore)
void launch_nf_accum(ivx_ctx* ctx, const float* X, int64_t F, const int* post_idx,
                     const float* post_val, const NfTarget& nf, hipStream_t s);
// n [U][C], f [U][C][D] from the sums, which are reset
void launch_nf_finish(ivx_ctx* ctx, int64_t U, float* n, float* f, hipStream_t s);
void launch_stats_S(ivx_ctx* ctx, const float* X, int64_t F, double* S_acc, hipStream_t s);
void launch_sum_f64(ivx_ctx* ctx, const double* x, int64_t n, double* acc, hipStream_t s);
// lscore[slot] = exact FP64 log w_c N(x_g; mu_c, Sigma_c) for the slots of
// ent[0, coff[C]) sorted by component (slot = g * kpf + index, c = .y)
void launch_exact_sorted(ivx_ctx* ctx, const int2* ent, const int* coff, int kpf, const float* X,
                         double* lscore, hipStream_t s);
void launch_hist_scan(int nb, int C, int* hist, int* coff, hipStream_t s);

// ---- ivx_api_tv.hip
ivx_status launch_linear_term(ivx_ctx* ctx, const float* f, int64_t U, int ns, hipStream_t s);
ivx_status ensure_tv_ready(ivx_ctx* ctx, hipStream_t s);

// ---- ivx_static.hip
// Resolves the device address of the static workspace of
// ubm_posteriors_static on `device` (which must be current); idempotent.
hipError_t static_scratch_init(int device);

// ---- ivx_api_sel.hip
void selector_free(ivx_ctx* ctx);
void presel_free(ivx_ctx* ctx);
// nf (optional): also accumulate n/f of the posteriors (launch_frame_utt)
void launch_posteriors(ivx_ctx* ctx, const float* X, int64_t F, int prec, int sel, int* post_idx,
                       float* post_val, double* frame_ll, hipStream_t s,
                       const NfTarget* nf = nullptr);

// ---- k_select.hip
bool select_set_attributes();
void launch_selector_pack(ivx_ctx* ctx, hipStream_t s);
void launch_feature_stats(ivx_ctx* ctx, const float* X, int64_t F, float* mean, float* stdv,
                          hipStream_t s);
void launch_selector_inv_std(ivx_ctx* ctx, hipStream_t s);
bool launch_selector_mlp(ivx_ctx* ctx, const float* X, int64_t F, uint16_t* h1_out,
                         uint16_t* h2_out, float* z_out, hipStream_t s);
void launch_select_learned(ivx_ctx* ctx, const float* X, int64_t F, int prec, int* post_idx,
                           float* post_val, double* frame_ll, hipStream_t s);
void launch_select_pruned(ivx_ctx* ctx, const float* X, int64_t F, int* post_idx, float* post_val,
                          double* frame_ll, hipStream_t s);
bool launch_selector_grad(ivx_ctx* ctx, const float* X, int64_t F, const int64_t* fidx, int B,
                          const int* post_idx, const float* post_val, double* loss,
                          hipStream_t s);
void launch_selector_adam(ivx_ctx* ctx, float lr, hipStream_t s);

}  // namespace ivx
