/*
 * ivx.h -- C ABI of the MI355X (gfx950) TV-model EM hot path.
 *
 * The operations follow Vestman, Lee, Kinnunen, Koshinaka, "Unleashing the
 * Unused Potential of I-Vectors Enabled by GPU Acceleration" (Interspeech
 * 2019), augmented formulation (Sec. 2.2): frame posteriors against a
 * full-covariance UBM, Baum-Welch statistics (Sec. 2), the E-step of
 * eqs. (3)-(4), the M-step of the factor-analysis EM cited in Sec. 2.1 and
 * Sec. 3.2 step 3, minimum-divergence re-estimation of eqs. (6)-(12), and the
 * UBM-mean realignment of Sec. 3.2.
 *
 * Conventions (every call):
 *  - Pointers named as device pointers must point to memory on the context's
 *    device; pointers named as host pointers to host memory.  The caller owns
 *    every pointer argument and keeps it valid until the work queued on
 *    `stream` has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Hot-path calls are asynchronous on `stream`: they never synchronise and
 *    never allocate, so they can be captured in a HIP graph.
 *  - Arrays are row-major, C-contiguous.  Sizes are in elements.
 *  - "packed" symmetric R x R storage is the upper triangle row by row:
 *    element (i, j), i <= j, at i*R - i*(i-1)/2 + (j - i); R(R+1)/2 entries.
 *  - "tile-packed" symmetric R x R storage (ivx_tp_size(R) entries) splits
 *    the matrix into 16 x 16 tiles (R padded up to a multiple of 16 with
 *    zeros) and stores the tiles (bi, bj) with bi >= bj in the order
 *    bi = 0..nb-1, bj = 0..bi, each tile as 16 x 16 row-major (rows of block
 *    row bi, columns of block column bj).  Diagonal tiles are stored in full.
 *  - The latent dimension R includes the prior-offset dimension, which is
 *    index 0 (the paper's element 1).
 *  - Argument errors are detected on the host before anything is queued and
 *    return IVX_EINVAL (nothing is launched).  Problems found by kernels
 *    (non-positive-definite matrices, non-finite values, malformed utterance
 *    offsets, candidate-list overflow) set a flag in the context that
 *    ivx_sync_status() reports; ivx_last_error() gives a message.
 *  - One host thread at a time per context.  Separate contexts are
 *    independent.
 */
#ifndef IVX_H
#define IVX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ivx_ctx ivx_ctx;

typedef enum {
  IVX_OK = 0,
  IVX_EINVAL = -1,     /* bad argument or dimension */
  IVX_ENOMEM = -2,     /* device allocation failed (only in ivx_create) */
  IVX_ENOTPD = -3,     /* a covariance / precision matrix is not positive definite */
  IVX_EDEVICE = -4,    /* HIP runtime error */
  IVX_ENUMERIC = -5,   /* non-finite value met by a kernel */
  IVX_ECAPACITY = -6   /* a frame's posterior does not fit the 16-entry list (see ubm_posteriors) */
} ivx_status;

typedef enum { IVX_FP32 = 0, IVX_BF16 = 1 } ivx_precision;
/* Which components a frame's posterior is computed over.
 *   IVX_SEL_ALL      every component (Sec. 4.2 posteriors, exact).
 *   IVX_SEL_LEARNED  the k proposals of the learned selector (ivx_selector_set),
 *                    scored exactly and renormalised over the proposals; a
 *                    frame whose proposals carry less than min_mass of the
 *                    network's softmax falls back to IVX_SEL_ALL.  This stands
 *                    where the paper's diagonal-UBM preselection of 20
 *                    components stands (Sec. 4.2); the network is not from the
 *                    paper.
 *   IVX_SEL_PRUNED   the paper's pruned alignment (Sec. 4.2, ivx_pruned_set):
 *                    the k best components of a diagonal-covariance UBM (the
 *                    diagonal of the full one) are scored with the full
 *                    covariances, posteriors are computed over them, those
 *                    below `prune` are dropped and the rest renormalised.
 *                    The precision argument does not apply (FP32 diagonal
 *                    scores and filter, FP64 exact scores). */
typedef enum { IVX_SEL_ALL = 0, IVX_SEL_LEARNED = 1, IVX_SEL_PRUNED = 2 } ivx_selection;

/* Problem dimensions, fixed for the life of a context.
 *   C  UBM components (>= 1), D feature dimension (1..63), R latent
 *   dimension including the offset dimension (2..480).
 *   max_batch_utts    largest U accepted by the utterance-batch calls.
 *   max_batch_frames  largest F accepted by the frame-batch calls, at most
 *                     2^31 / 32 - 1 = 67,108,863 (per-frame candidate and
 *                     proposal slots are numbered in 32-bit ints); ivx_create
 *                     returns IVX_EINVAL above it. */
typedef struct {
  int32_t C, D, R;
  int32_t max_batch_utts;
  int64_t max_batch_frames;
} ivx_dims;

/* M-step accumulators (all device pointers, FP64, caller-allocated and
 * caller-zeroed; tv_mstep_accumulate adds to them).
 *   A     [C][ivx_tp_size(R)]  A_c = sum_u n_c(u) (Phi(u) + phi(u) phi(u)^T), tile-packed
 *   Cc    [C][D][R]            Cc_c = sum_u f_c(u) phi(u)^T
 *   N     [C]                  N_c = sum_u n_c(u)
 *   h     [R]                  sum_u phi(u)                (U * eq. (6))
 *   H     [ivx_tp_size(R)]     sum_u Phi(u) + phi(u) phi(u)^T (U * eq. (7)), tile-packed
 *   count [1]                  number of utterances accumulated (double) */
typedef struct {
  double* A;
  double* Cc;
  double* N;
  double* h;
  double* H;
  double* count;
} ivx_accum;

/* ---------------------------------------------------------------- lifecycle */

/* Creates a context on HIP device `device` and allocates all model storage
 * and workspace for `dims` (the only call besides ivx_set_* that allocates).
 * Returns IVX_EINVAL for bad dims, IVX_ENOMEM if allocation fails. */
ivx_status ivx_create(const ivx_dims* dims, int device, ivx_ctx** out);

/* Frees everything the context owns.  NULL is ignored. */
void ivx_destroy(ivx_ctx* ctx);

/* Message for the last error on the calling thread ("" if none). */
const char* ivx_last_error(void);

/* Synchronises `stream`, then returns and clears the first error recorded by
 * a kernel since the last call (IVX_OK if none). */
ivx_status ivx_sync_status(ivx_ctx* ctx, void* stream);

/* Number of doubles/floats in a tile-packed symmetric R x R matrix. */
int64_t ivx_tp_size(int32_t R);

/* ------------------------------------------------------------------- model */

/* Loads the full-covariance UBM (Sec. 4.1): weights w [C], means mu [C][D],
 * covariances cov [C][D][D] (device pointers, FP64) and derives the per-
 * component Cholesky factors, log-determinants and the expanded
 * quadratic-form coefficients used for the frame log-likelihoods.
 * Synchronises `stream`; returns IVX_ENOTPD if a covariance is not positive
 * definite. */
ivx_status ivx_set_ubm(ivx_ctx* ctx, const double* w, const double* mu, const double* cov,
                       void* stream);

/* Augmented initialisation (Sec. 2.1-2.2): T_c <- T_rand_c (device, FP64
 * [C][D][R], N(0,1) draws supplied by the caller) with column 0 replaced by
 * mu_c / p0, Sigma_c <- UBM covariance, p <- p0 e_1.  Requires ivx_set_ubm. */
ivx_status ivx_init_tv(ivx_ctx* ctx, const double* T_rand, double p0, void* stream);

/* Standard initialisation (Sec. 2.1): T_c <- T_rand_c (device, FP64
 * [C][D][R], N(0,1) draws supplied by the caller), Sigma_c <- UBM covariance,
 * p <- 0 and the bias m_c <- UBM mean mu_c.  Puts the context in the standard
 * formulation: from then on bw_stats and extract_ivectors centre their
 * statistics on m (Sec. 2), tv_mindiv whitens only (Sec. 3.1) and
 * ubm_update_means is refused.  ivx_init_tv returns it to the augmented one.
 * Requires ivx_set_ubm. */
ivx_status ivx_init_tv_standard(ivx_ctx* ctx, const double* T_rand, void* stream);

/* Sets the bias m [C][D] (device, FP64; copied) and puts the context in the
 * standard formulation; m = NULL returns it to the augmented formulation.
 * The prior offset p is not changed: the standard formulation needs p = 0
 * (ivx_set_tv). */
ivx_status ivx_set_bias(ivx_ctx* ctx, const double* m, void* stream);

/* Reads the bias m [C][D] (device, FP64).  IVX_EINVAL in the augmented
 * formulation. */
ivx_status ivx_get_bias(ivx_ctx* ctx, double* m, void* stream);

/* Sets / reads the TV model: T [C][D][R], Sigma [C][D][D], p [R] (device,
 * FP64).  ivx_get_tv also returns the current UBM means mu [C][D]; any output
 * pointer may be NULL. */
ivx_status ivx_set_tv(ivx_ctx* ctx, const double* T, const double* Sigma, const double* p,
                      void* stream);
ivx_status ivx_get_tv(ivx_ctx* ctx, double* T, double* Sigma, double* p, double* mu,
                      void* stream);

/* ---------------------------------------------------------------- hot path */

/* Frame posteriors gamma_tc = w_c N(x_t; mu_c, cov_c) / sum_c' (...)
 * (frame alignment, Sec. 3.2 step 1 and Sec. 4.2) over ALL C components.
 *   X         [F][D] FP32 device frames.
 *   gamma     [F][C] FP32 dense posteriors, or NULL.
 *   post_idx  [F][K] int32 / post_val [F][K] FP32: the components within the
 *             candidate margin of each frame's best one and their posteriors
 *             (unused slots: index -1, value 0), or NULL.  K must be 16.
 *   frame_ll  [F] FP64 log sum_c w_c N(x_t; ...), or NULL.
 * Components more than ln C + 18.64 nats below the frame's best carry a
 * total mass below 2^-24 e^-2 and are reported as 0.  If more than 16
 * components lie within that margin, the 16 with the highest exact scores
 * are kept, and IVX_ECAPACITY is recorded when the others carry more than
 * 1e-6 of the frame's mass (very flat posteriors, e.g. small D). */
ivx_status ubm_posteriors(ivx_ctx* ctx, const float* X, int64_t F, ivx_precision prec,
                          ivx_selection sel, float* gamma, int32_t* post_idx, float* post_val,
                          int32_t K, double* frame_ll, void* stream);

/* ubm_posteriors with IVX_SEL_ALL for callers that cannot allocate device
 * memory or hold a batch-sized workspace (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the frame-stage workspace
 * (candidate lists, maxima, overflow flags, exact scores, the component-
 * sorted slot list) lives in one fixed device array of the library, 64 MiB
 * per device (ivx_static_bytes), resolved by ivx_create on each device it
 * creates a context on.  The call allocates nothing; F is bounded by that
 * array, not by the context's max_batch_frames: it needs about
 * 392 + C/2048 bytes per frame (about 170,000 frames at C = 2048) and
 * returns IVX_EINVAL, before any launch, for a larger F.
 *   post_idx [F][K] int32 / post_val [F][K] FP32 (K = 16) are required;
 *   frame_ll [F] FP64 or NULL; prec as in ubm_posteriors.
 * Results equal ubm_posteriors(..., IVX_SEL_ALL, ...) on the same inputs.
 * Every call on a device shares that device's array and overwrites all of
 * it that it reads: calls that overlap on one device (two streams or host
 * threads, whatever the context) race and must be serialised by the
 * caller. */
ivx_status ubm_posteriors_static(ivx_ctx* ctx, const float* X, int64_t F, ivx_precision prec,
                                 int32_t* post_idx, float* post_val, int32_t K, double* frame_ll,
                                 void* stream);

/* Size in bytes of ubm_posteriors_static's per-device array. */
int64_t ivx_static_bytes(void);

/* Baum-Welch statistics of U utterances (Sec. 2), uncentred in the augmented
 * formulation; in the standard formulation every term is centred on the bias
 * first: f~_c(u) = sum_t gamma_tc (x_t - m_c), S~_c = sum_t gamma_tc
 * (x_t - m_c)(x_t - m_c)^T (n and ll_acc are the same in both).
 *   X        [F][D] FP32 device frames, utterances concatenated.
 *   utt_off  [U+1] int64 device offsets: utt_off[0] = 0, non-decreasing,
 *            utt_off[U] = F (checked by a kernel).
 *   n        [U][C] FP32  n_c(u) = sum_t gamma_tc
 *   f        [U][C][D] FP32  f_c(u) = sum_t gamma_tc x_t
 *   S_acc    [C][D(D+1)/2] FP64, packed: S_c += sum_t gamma_tc x_t x_t^T, or NULL
 *   ll_acc   [1] FP64: += sum_t log p(x_t | UBM), or NULL */
ivx_status bw_stats(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U, int64_t F,
                    ivx_precision prec, ivx_selection sel, float* n, float* f, double* S_acc,
                    double* ll_acc, void* stream);

/* E-step, eqs. (3)-(4), for U utterances (U <= max_batch_utts):
 *   L(u) = I + sum_c n_c(u) T_c^T Sigma_c^{-1} T_c,  b(u) = p + sum_c T_c^T Sigma_c^{-1} f_c(u)
 *   phi  [U][R] FP32  phi(u) = L(u)^{-1} b(u)
 *   Phi  [U][R(R+1)/2] FP32 packed Phi(u) = L(u)^{-1}, or NULL
 *   ll_acc [1] FP64 += sum_u (-1/2 log|L(u)| + 1/2 b(u)^T phi(u) - 1/2 p^T p), or NULL
 *   info [U] int32: 0, or k > 0 if the Cholesky factorisation of L(u) met a
 *        non-positive pivot at row k-1 (that utterance's outputs are then
 *        undefined), or NULL.
 * n, f are the device arrays produced by bw_stats. */
ivx_status tv_estep(ivx_ctx* ctx, const float* n, const float* f, int64_t U,
                    ivx_precision prec, float* phi, float* Phi, double* ll_acc, int32_t* info,
                    void* stream);

/* Adds the M-step sufficient statistics of U utterances to `acc` (see
 * ivx_accum): n [U][C], f [U][C][D], phi [U][R], Phi [U][R(R+1)/2] packed
 * (device, FP32, as produced by bw_stats / tv_estep).  `acc` itself is a
 * host struct of device pointers. */
ivx_status tv_mstep_accumulate(ivx_ctx* ctx, const float* n, const float* f, const float* phi,
                               const float* Phi, int64_t U, const ivx_accum* acc, void* stream);

/* i-vector extraction (Sec. 3.2, last paragraph): posteriors against the
 * current (possibly realigned) UBM, n and f (centred on the bias in the
 * standard formulation), then eq. (4).
 *   phi [U][R] FP32.  X, utt_off as in bw_stats. */
ivx_status extract_ivectors(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                            int64_t F, ivx_precision prec, ivx_selection sel, float* phi,
                            void* stream);

/* ------------------------------------------------------ iteration finalise */

/* M-step (Sec. 3.2 step 3), FP64: for every component with N_c >= 0.5,
 *   T_c <- Cc_c A_c^{-1};  if update_sigma: Sigma_c <- sym((S_c - T_c Cc_c^T) / N_c)
 * S [C][D(D+1)/2] FP64 packed (from bw_stats).  acc->A is overwritten by the
 * Cholesky factors of A_c.  A new Sigma_c that is not positive definite is
 * rejected (old one kept) and flagged in `status`.
 *   objective [1] FP64 or NULL: receives the EM objective at the incoming
 *     parameters, sum_c N_c(-D/2 log 2pi - 1/2 log|Sigma_c|)
 *     - 1/2 sum_c tr(Sigma_c^{-1} S_c) + ll_sum, where ll_sum is read from
 *     ll_sum_dev [1] (the tv_estep ll_acc of the same pass).
 *   status [C] int32 or NULL: 0 updated, 1 skipped (N_c < 0.5), 2 Sigma not PD
 *     (T updated, Sigma kept), 3 A_c not PD (nothing updated). */
ivx_status tv_mstep_solve(ivx_ctx* ctx, const ivx_accum* acc, const double* S, int update_sigma,
                          const double* ll_sum_dev, double* objective, int32_t* status,
                          void* stream);

/* Minimum-divergence re-estimation, augmented formulation (eqs. (6)-(12)),
 * from acc->h, acc->H, acc->count: G = H/U - (h/U)(h/U)^T, P1 = L_G^{-1}
 * (Cholesky whitening, method 0; other methods return IVX_EINVAL),
 * Householder P2, T_c <- T_c P1^{-1} P2^{-1}, p <- P2 P1 h.  In the standard
 * formulation: T_c <- T_c P1^{-1} only (see tv_mindiv_standard). */
ivx_status tv_mindiv(ivx_ctx* ctx, const ivx_accum* acc, int method, void* stream);

/* Standard-formulation minimum divergence (Sec. 3.1), from acc->h, acc->H,
 * acc->count: G = H/U - (h/U)(h/U)^T = L_G L_G^T (method 0, Cholesky; other
 * methods return IVX_EINVAL) and T_c <- T_c L_G (= T_c P1^{-1}).  With
 * update_mean != 0 the bias first absorbs the i-vector mean (Sec. 5):
 * m_c <- m_c + T_c h/U with the incoming T_c.  If G is not positive definite
 * nothing changes and IVX_ENOTPD is recorded.  IVX_EINVAL in the augmented
 * formulation.  tv_mindiv on a standard context equals update_mean = 0. */
ivx_status tv_mindiv_standard(ivx_ctx* ctx, const ivx_accum* acc, int method, int update_mean,
                              void* stream);

/* Realignment (Sec. 3.2 step 5): mu_c <- p[0] * T_c[:, 0], then re-derives
 * the UBM quantities used by ubm_posteriors.  Augmented formulation only
 * (IVX_EINVAL in the standard one). */
ivx_status ubm_update_means(ivx_ctx* ctx, void* stream);

/* -------------------------------------------------------- iteration graphs */

typedef struct ivx_graph ivx_graph;

/* Records one full EM iteration (Sec. 3.2, steps 1-5) into a HIP graph:
 * clears S, the accumulators and the two log-likelihood sums (fill kernels),
 * then bw_stats, tv_estep (with the TV precompute), tv_mstep_accumulate,
 * tv_mstep_solve (objective at the incoming parameters into objective[0]),
 * tv_mindiv (Cholesky whitening) and, if realign != 0, ubm_update_means.
 * The formulation (augmented or standard) is the one the context holds at
 * capture time; realign != 0 needs the augmented one.
 * Every pointer is caller-owned device memory with the layout of the
 * corresponding call; it is bound at capture time and must stay valid for
 * the life of the graph.  Capture runs on a private stream and executes
 * nothing; each ivx_graph_launch runs one iteration on `stream`. */
ivx_status ivx_graph_create_em(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                               int64_t F, ivx_precision prec, float* n, float* f, double* S,
                               float* phi, float* Phi, const ivx_accum* acc, double* ll_frames,
                               double* ll_utts, double* objective, int update_sigma, int realign,
                               ivx_graph** out);
ivx_status ivx_graph_launch(ivx_graph* g, void* stream);
void ivx_graph_destroy(ivx_graph* g);

/* ------------------------------------------------------- learned selection */

/* The selector network: z = W3 relu(W2 relu(W1 x_hat + b1) + b2) + b3 over
 * the standardised features x_hat = (x - mean) / std, softmax over the C
 * components.  Inference runs on BF16 MFMA (weights and activations rounded to
 * BF16, FP32 accumulation); training keeps an FP32 master copy.
 *   H1, H2           hidden sizes, multiples of 128 in [128, 4096]
 *   k                proposals per frame, 1..min(32, C)
 *   min_mass         fallback threshold on the proposals' softmax mass
 *   max_train_batch  largest training batch (0: inference only) */
typedef struct {
  int32_t H1, H2, k;
  float min_mass;
  int32_t max_train_batch;
} ivx_selector_dims;

/* Global mean and standard deviation of F frames X [F][D] (FP64 sums) into
 * mean [D], std [D] (device FP32). */
ivx_status ivx_feature_stats(ivx_ctx* ctx, const float* X, int64_t F, float* mean, float* std,
                             void* stream);

/* Installs a selector (replacing any previous one; synchronises `stream`,
 * allocates its workspace: about maxF * (12 k + 4 D + 16) bytes plus the
 * weights).  params: device FP32, flat, in the order W1 [H1][D], b1 [H1],
 * W2 [H2][H1], b2 [H2], W3 [C][H2], b3 [C] (ivx_selector_param_count values).
 * mean, std: [D] device FP32 (std > 0, else IVX_EINVAL from ivx_sync_status).
 * Adam moments start at zero. */
ivx_status ivx_selector_set(ivx_ctx* ctx, const ivx_selector_dims* dims, const float* params,
                            const float* mean, const float* std, void* stream);
int64_t ivx_selector_param_count(const ivx_ctx* ctx);
/* Copies the FP32 master parameters (layout of ivx_selector_set) to params. */
ivx_status ivx_selector_get(ivx_ctx* ctx, float* params, void* stream);

/* Runs the network over X [F][D] and returns, each optional (NULL):
 *   h1 [F][H1], h2 [F][H2]  BF16 activations (raw 16-bit patterns)
 *   z  [F][C]  FP32 logits
 *   prop [F][k] int32: the k largest logits, largest first, ties to the lower
 *        component index
 *   mass [F] FP32 sum of softmax(z) over the proposals
 *   fallback [F] int32: 1 where mass < min_mass */
ivx_status ivx_selector_forward(ivx_ctx* ctx, const float* X, int64_t F, uint16_t* h1,
                                uint16_t* h2, float* z, int32_t* prop, float* mass,
                                int32_t* fallback, void* stream);

/* Soft-target cross-entropy -1/B sum_b sum_c gamma_bc log softmax(z_b)_c over
 * the B frames X[frame_idx[b]] (FP32 forward and backward on MFMA, FP32
 * master weights), with targets gamma from the posterior lists post_idx /
 * post_val [F][16] (the layout of ubm_posteriors, indexed by frame).
 *   ivx_selector_grad writes the gradient (parameter layout) to grad (device
 *   FP32, or NULL) and the loss to loss[0] (device FP64, or NULL); the
 *   parameters are unchanged.
 *   ivx_selector_train_step also applies one Adam step (beta 0.9 / 0.999,
 *   eps 1e-8) with learning rate lr and refreshes the BF16 copies.
 * A frame index outside [0, F) records IVX_EINVAL (ivx_sync_status). */
ivx_status ivx_selector_grad(ivx_ctx* ctx, const float* X, int64_t F, const int64_t* frame_idx,
                             int32_t B, const int32_t* post_idx, const float* post_val,
                             float* grad, double* loss, void* stream);
ivx_status ivx_selector_train_step(ivx_ctx* ctx, const float* X, int64_t F,
                                   const int64_t* frame_idx, int32_t B, const int32_t* post_idx,
                                   const float* post_val, float lr, double* loss, void* stream);

/* Sets up the pruned alignment (IVX_SEL_PRUNED): k (1..min(32, C)) best
 * diagonal-UBM components per frame, pruning threshold in [0, 0.5) (the paper
 * uses k = 20 and 0.025).  Synchronises `stream`; allocates about
 * maxF * 20 k bytes of workspace.  The diagonal coefficients follow the
 * current UBM (recomputed by every pruned pass).  If more than 16 of a
 * frame's posteriors reach the threshold, IVX_ECAPACITY is recorded. */
ivx_status ivx_pruned_set(ivx_ctx* ctx, int32_t k, float prune, void* stream);

/* Counters of the last learned-selection pass (synchronises `stream`):
 * frames that fell back to all components, and the (frame, proposal) pairs
 * that were scored. */
ivx_status ivx_selector_counts(ivx_ctx* ctx, int64_t* fallback_frames, int64_t* kept_pairs,
                               void* stream);

/* -------------------------------------------------------------- autotuner */

/* Launch shapes of the hot-path kernels.  Every choice computes the same
 * result (up to FP32 summation order in the split GEMM).
 *   frame_ncb       launch shape of the FP32 frame GEMM: 8 (256 components
 *                   per launch, one 32-frame block per wave), 4 (128
 *                   components) or 2 (128 components, two frame blocks per
 *                   wave)
 *   frame_ncb_bf16  the same for the BF16 split form
 *   b_split         K-splits of the linear-term GEMM b = p + F V (0: chosen
 *                   from the grid size; else 1..max)
 *   frame_direct    FP32 frame GEMM with one 32-frame block per wave: 1 reads
 *                   the coefficients straight into registers (no LDS staging,
 *                   no barrier in the k loop), 0 stages them through LDS
 *   mstep_left      M-step Cholesky of A_c: 1 left-looking (each block column
 *                   formed in LDS from the finished ones and written once),
 *                   0 right-looking (trailing tiles updated in place)
 *   estep_global    per-utterance E-step factorisation: 0 holds the whole
 *                   precision matrix in the registers of one workgroup
 *                   (R <= 400; larger R always use the other form), 1 works
 *                   on the matrix in device memory tile by tile
 *   mstep_global    M-step solve: 0 keeps the right-hand sides in registers
 *                   and runs the forward solve inside a left-looking Cholesky
 *                   (R <= 400), 1 the form chosen by mstep_left, with the
 *                   right-hand sides in device memory */
typedef struct {
  int32_t frame_ncb, frame_ncb_bf16, b_split, frame_direct, mstep_left, estep_global,
      mstep_global;
} ivx_tuning;

/* Times the candidate launch shapes on the given workload (X, utt_off as in
 * bw_stats; needs the UBM and the TV model) with HIP events on `stream`,
 * keeps the fastest in the context and returns them in *out (or NULL).
 * Synchronises; allocates nothing; overwrites the context's workspace. */
ivx_status ivx_autotune(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                        int64_t F, ivx_tuning* out, void* stream);
ivx_status ivx_tuning_get(const ivx_ctx* ctx, ivx_tuning* out);
/* Sets the launch shapes (e.g. a saved tuning); IVX_EINVAL for values
 * outside the lists above. */
ivx_status ivx_tuning_set(ivx_ctx* ctx, const ivx_tuning* t);

/* ----------------------------------------------------------------- tracing */

/* Opt-in kernel timing with HIP events recorded on the stream each kernel
 * group is launched on.  ivx_profile_enable(ctx, capacity) creates
 * `capacity` event pairs (capacity 0 disables and frees them; it
 * synchronises the device).  ivx_profile_read() synchronises the device, adds
 * the elapsed milliseconds of every completed pair to ms[k] and its count to
 * calls[k] for the kernel groups k = 0..n-1 (host arrays of length n, n <= the
 * number of groups), then resets the pairs.  Groups: 0 frame-select GEMM,
 * 1 rescoring, 2 n/f statistics, 3 second-order statistics, 4 TV precompute,
 * 5 E-step GEMMs, 6 E-step Cholesky/solve/inverse, 7 accumulators, 8 M-step
 * solve, 9 minimum divergence, 10 UBM preparation.  Pairs beyond the capacity
 * are not recorded. */
ivx_status ivx_profile_enable(ivx_ctx* ctx, int32_t capacity);
ivx_status ivx_profile_read(ivx_ctx* ctx, double* ms, int64_t* calls, int32_t n);

/* ------------------------------------------------ streaming host pipeline */

/* Data loaders and fixed-size batches of Sec. 4.2 (Fig. 1): utterances held
 * in host memory (or produced on demand by a frame source) are cut into runs
 * of consecutive utterances, copied by loader threads into pinned host slots,
 * uploaded on a copy stream into one of two device buffers and processed on
 * the caller's stream while the next batch is in flight.  Device memory is
 * set by the batch limits, not by the corpus size. */

/* Greedy batch plan (host only, no GPU needed): consecutive utterances are
 * added to a batch until one more would exceed max_utts utterances or
 * max_frames frames.  utt_off [U+1] host, utt_off[0] = 0, non-decreasing.
 * starts [cap] receives the first utterance of each batch followed by U;
 * *nbatches receives the number of batches (also when cap is too small, which
 * returns IVX_EINVAL).  IVX_EINVAL if an utterance is longer than max_frames. */
ivx_status ivx_plan_batches(const int64_t* utt_off, int64_t U, int32_t max_utts,
                            int64_t max_frames, int64_t* starts, int64_t cap, int64_t* nbatches);

typedef struct ivx_stream ivx_stream;

/* max_batch_utts / max_batch_frames: batch limits, at most the context's
 * max_batch_utts / max_batch_frames; loaders: host threads (1-64) filling
 * slots; slots: pinned host buffers of one batch each (2-16). */
typedef struct {
  int32_t max_batch_utts;
  int64_t max_batch_frames;
  int32_t loaders;
  int32_t slots;
} ivx_stream_config;

/* A frame source writes the frames of utterances [u0, u1) (host offsets
 * utt_off as given to the pass) into X_dst, [utt_off[u1] - utt_off[u0]][D]
 * FP32, and returns 0 (anything else stops the pass with IVX_EINVAL).  It is
 * called from the loader threads, several at a time. */
typedef int32_t (*ivx_frame_source)(void* user, int64_t u0, int64_t u1, const int64_t* utt_off,
                                    float* X_dst);

/* Allocates the pinned slots, the two device frame buffers and the per-batch
 * n, f, phi, Phi workspace for `ctx` (which must outlive the stream object).
 * IVX_EINVAL for limits outside the context's, IVX_ENOMEM if allocation fails. */
ivx_status ivx_stream_create(ivx_ctx* ctx, const ivx_stream_config* cfg, ivx_stream** out);
void ivx_stream_destroy(ivx_stream* st);

/* Statistics, E-step and accumulation of one EM pass over host-resident
 * utterances: per batch bw_stats (adding to S_acc and ll_frames), tv_estep
 * (adding to ll_utts) and tv_mstep_accumulate (adding to acc), exactly the
 * calls a caller would make, on `stream`.  The frames come from X [F][D] FP32
 * host memory (F = utt_off[U]) or from `src` (exactly one of the two).
 * phi_out [U][R] FP32 device receives every utterance's i-vector, or NULL.
 * S_acc, ll_frames, ll_utts may be NULL as in the calls above.  Returns once
 * every batch has been uploaded and issued (X is no longer read); results are
 * complete when `stream` completes.  Follows the context's formulation and
 * any selection set up on it.  Passes on one stream object are ordered among
 * themselves on the GPU whatever streams they are issued on: a pass waits for
 * the previous pass's batches before it reuses their device buffers. */
ivx_status ivx_stream_em_pass(ivx_stream* st, const float* X, ivx_frame_source src,
                              void* src_user, const int64_t* utt_off, int64_t U,
                              ivx_precision prec, ivx_selection sel, double* S_acc,
                              double* ll_frames, double* ll_utts, const ivx_accum* acc,
                              float* phi_out, void* stream);

/* i-vector extraction of host-resident utterances in batches (as
 * extract_ivectors per batch): phi [U][R] FP32 device. */
ivx_status ivx_stream_extract(ivx_stream* st, const float* X, ivx_frame_source src,
                              void* src_user, const int64_t* utt_off, int64_t U,
                              ivx_precision prec, ivx_selection sel, float* phi, void* stream);

/* ------------------------------------------------------- scoring back-end */

/* The back-end of Sec. 4.1 (after extraction): i-vectors are centred,
 * whitened when minimum divergence was not used, length-normalised, reduced
 * by LDA (400 -> 200 in the paper) and scored by a Gaussian PLDA; accuracy is
 * the equal error rate.  The paper gives no formulas for these steps; this
 * library takes: whitening W = Lambda^{-1/2} Q^T of the covariance
 * Q Lambda Q^T (divisor N); LDA from Sb v = lambda Sw v (between- and
 * within-class scatter, divisor N) with V^T Sw V = I and decreasing
 * eigenvalues; the two-covariance PLDA y = mu + s + e, s ~ N(0, B),
 * e ~ N(0, W), with B = Sb and W = Sw of its training vectors, scored by the
 * log-likelihood ratio of "same speaker" against "different speakers"; EER =
 * the crossing of P_miss = P_fa on the operating points (P_miss(t), P_fa(t))
 * of every threshold t among the scores and above them, joined by straight
 * segments, misses being targets below t and false alarms non-targets at or
 * above t.
 * Symmetric eigenproblems are solved on the GPU by a one-workgroup Jacobi
 * method in FP64.  Vectors are FP32 [n][dim] rows, matrices FP64 row-major,
 * all on the device unless stated. */
typedef struct ivx_backend ivx_backend;

/* Workspace for up to max_n vectors of dimension <= max_dim (2..512) and up
 * to max_classes classes.  IVX_ENOMEM if allocation fails. */
ivx_status ivx_backend_create(int32_t max_dim, int64_t max_n, int32_t max_classes, int device,
                              ivx_backend** out);
void ivx_backend_destroy(ivx_backend* be);

/* mean [dim] and whitening matrix W [dim][dim] of the rows of X [n][dim];
 * synchronises `stream`.  IVX_ENOTPD if the covariance is singular
 * (an eigenvalue below 1e-13 of the largest). */
ivx_status ivx_backend_whitening(ivx_backend* be, const float* X, int64_t n, int32_t dim,
                                 double* mean, double* W, void* stream);

/* Y = W (X - mean) scaled to unit length per row; mean and W may be NULL
 * (no centring / no whitening).  X, Y [n][dim]; asynchronous. */
ivx_status ivx_backend_lnorm(ivx_backend* be, const float* X, int64_t n, int32_t dim,
                             const double* mean, const double* W, float* Y, void* stream);

/* LDA of X [n][dim] with labels [n] in [0, K): V [dim][out_dim] and its
 * eigenvalues eigval [out_dim] (or NULL); synchronises `stream`.
 * IVX_EINVAL for labels outside [0, K), IVX_ENOTPD if Sw is singular. */
ivx_status ivx_backend_lda(ivx_backend* be, const float* X, int64_t n, int32_t dim,
                           const int32_t* labels, int32_t K, int32_t out_dim, double* V,
                           double* eigval, void* stream);

/* Y [n][out_dim] = X [n][dim] V [dim][out_dim] (FP64 sums); asynchronous. */
ivx_status ivx_backend_project(ivx_backend* be, const float* X, int64_t n, int32_t dim,
                               const double* V, int32_t out_dim, float* Y, void* stream);

/* Two-covariance PLDA of Y [n][d] with labels [n] in [0, K): mu [d] and the
 * simultaneous diagonaliser A [d][d] (A^T W A = I, A^T B A = diag(psi)) with
 * psi [d]; synchronises `stream`.  Errors as ivx_backend_lda. */
ivx_status ivx_backend_plda_fit(ivx_backend* be, const float* Y, int64_t n, int32_t d,
                                const int32_t* labels, int32_t K, double* mu, double* A,
                                double* psi, void* stream);

/* scores [T] FP32: the PLDA log-likelihood ratio of every trial
 * (Y1[trials[2t]], Y2[trials[2t+1]]), trials [T][2] int32; Y1 [n1][d],
 * Y2 [n2][d] (Y2 may equal Y1); asynchronous.  A trial index outside its set
 * gives NaN and is reported by ivx_backend_status. */
ivx_status ivx_backend_plda_score(ivx_backend* be, const double* mu, const double* A,
                                  const double* psi, int32_t d, const float* Y1, int64_t n1,
                                  const float* Y2, int64_t n2, const int32_t* trials, int64_t T,
                                  float* scores, void* stream);

/* Synchronises `stream`; IVX_EINVAL if a scored trial index was out of range. */
ivx_status ivx_backend_status(ivx_backend* be, void* stream);

/* Equal error rate of host scores [n] with host flags is_target [n] (0 / 1),
 * as defined above.  Host only. */
ivx_status ivx_eer(const float* scores, const uint8_t* is_target, int64_t n, double* eer);

#ifdef __cplusplus
}
#endif

#endif /* IVX_H */
