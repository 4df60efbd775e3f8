// C ABI entry points of the E-step, the M-step and extraction.
#include <cstdio>

#include "ivx_internal.h"
#include "ivx_tv.h"
#include "k_gemm.h"

using namespace ivx;

#define IVX_CHECK(cond, ...)  \
  do {                        \
    if (!(cond)) {            \
      set_error(__VA_ARGS__); \
      return IVX_EINVAL;      \
    }                         \
  } while (0)

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

ivx_status after_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

ivx_status gemm(const GemmArgs& g, bool ta, bool tb, int epi, int batches, hipStream_t s,
                const char* what) {
  if (!gemm_f32(g, ta, tb, epi, batches, s)) {
    set_error("%s: GEMM variant not available", what);
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

// Recomputes V_c, U_c (and Sigma_c^{-1}, log|Sigma_c|) after the TV model changed.
ivx_status ensure_tv(ivx_ctx* ctx, hipStream_t s) {
  if (!ctx->tv_dirty) return IVX_OK;
  ProfScope ps(ctx, PK_TV_PREP, s);
  launch_tv_prep(ctx, s);
  GemmArgs g;
  g.A = ctx->Y32;
  g.B = ctx->Y32;
  g.C = ctx->Utp;
  g.lda = ctx->R;
  g.ldb = ctx->R;
  g.ldc = 0;
  g.M = ctx->R;
  g.N = ctx->R;
  g.K = ctx->D;
  g.sA = (int64_t)ctx->D * ctx->R;
  g.sB = g.sA;
  g.sC = ctx->TP;
  ivx_status st = gemm(g, true, false, GEMM_STORE_TP, ctx->C, s, "tv precompute");
  if (st != IVX_OK) return st;
  ctx->tv_dirty = false;
  ctx->utp16_valid = false;
  return IVX_OK;
}

}  // namespace

namespace ivx {

// b(u) = p + sum_c V_c^T f_c(u) into ctx->bvec: the FP32 GEMM F V split over
// K = C D into ns partial products (ns <= 0: enough splits for ~1024
// workgroups), then a reduction that adds p.
ivx_status launch_linear_term(ivx_ctx* ctx, const float* f, int64_t U, int ns_req, hipStream_t s) {
  const int C = ctx->C, D = ctx->D, R = ctx->R;
  const int64_t K = (int64_t)C * D;
  int64_t ns = ns_req;
  if (ns <= 0) {
    const int64_t tiles = ((U + 127) / 128) * ((R + 127) / 128);
    ns = (1024 + tiles - 1) / tiles;
  }
  if (ns > ctx->nsplit_max) ns = ctx->nsplit_max;
  if (ns < 1) ns = 1;
  int64_t kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + 15) / 16 * 16;
  ns = (K + kchunk - 1) / kchunk;
  GemmArgs gb;
  gb.A = f;
  gb.lda = K;
  gb.B = ctx->V32;
  gb.ldb = R;
  gb.C = ctx->bpart;
  gb.ldc = R;
  gb.sS = U * R;
  gb.M = (int)U;
  gb.N = R;
  gb.K = (int)K;
  gb.ksplit = (int)ns;
  gb.kchunk = (int)kchunk;
  if (!gemm_f32(gb, false, false, GEMM_STORE, 1, s)) {
    set_error("tv_estep: GEMM variant not instantiated");
    return IVX_EINVAL;
  }
  launch_reduce_b(ctx, ctx->bpart, (int)ns, U * R, U, ctx->bvec, s);
  return IVX_OK;
}

ivx_status ensure_tv_ready(ivx_ctx* ctx, hipStream_t s) { return ensure_tv(ctx, s); }

}  // namespace ivx

namespace {

ivx_status estep_impl(ivx_ctx* ctx, const float* n, const float* f, int64_t U, int prec,
                      float* phi, float* Phi, double* ll_acc, int32_t* info, hipStream_t s) {
  ivx_status st = ensure_tv(ctx, s);
  if (st != IVX_OK) return st;
  const int C = ctx->C, D = ctx->D, R = ctx->R;
  int slot = prof_begin(ctx, PK_ESTEP_GEMM, s);
  // L(u) = I + sum_c n_c(u) U_c
  GemmArgs gl;
  gl.A = n;
  gl.lda = C;
  gl.B = ctx->Utp;
  gl.ldb = ctx->TP;
  gl.C = ctx->Lbuf;
  gl.ldc = ctx->TP;
  gl.M = (int)U;
  gl.N = (int)ctx->TP;
  gl.K = C;
  if (prec == IVX_BF16) {
    // operands split into BF16 high / low parts, K (= C) contiguous and
    // padded to a multiple of 8: U^tp once per model, N per call
    const int64_t Ck = (C + 7) / 8 * 8;
    if (!ctx->utp16_valid) {
      split_bf16_transposed(ctx->Utp, C, ctx->TP, Ck, ctx->Ut16hi, ctx->Ut16lo, s);
      ctx->utp16_valid = true;
    }
    split_bf16(n, U, C, Ck, ctx->n16hi, ctx->n16lo, s);
    gemm_bf16x3_nt(ctx->n16hi, ctx->n16lo, Ck, ctx->Ut16hi, ctx->Ut16lo, Ck, ctx->Lbuf, ctx->TP,
                   (int)U, (int)ctx->TP, (int)Ck, s);
  } else if ((st = gemm(gl, false, false, GEMM_STORE, 1, s, "tv_estep")) != IVX_OK) {
    return st;
  }
  launch_add_identity(ctx, ctx->Lbuf, U, s);
  // b(u) = p + sum_c V_c^T f_c(u), split over K = C*D
  if ((st = launch_linear_term(ctx, f, U, ctx->tune.b_split, s)) != IVX_OK) return st;
  prof_end(ctx, slot, s);
  {
    ProfScope ps(ctx, PK_ESTEP_CHOL, s);
    launch_estep_chol(ctx, U, ctx->Lbuf, ctx->Wbuf, ctx->bvec, phi, ctx->llu, info, Phi, s);
  }
  if (ll_acc) launch_sum_f64(ctx, ctx->llu, U, ll_acc, s);
  return after_launch("tv_estep");
}

}  // namespace

extern "C" {

ivx_status tv_estep(ivx_ctx* ctx, const float* n, const float* f, int64_t U, ivx_precision prec,
                    float* phi, float* Phi, double* ll_acc, int32_t* info, void* stream) {
  IVX_CHECK(ctx, "tv_estep: null context");
  IVX_CHECK(ctx->tv_set, "tv_estep: no TV model (ivx_init_tv / ivx_set_tv)");
  IVX_CHECK(U >= 0 && U <= ctx->maxU, "tv_estep: U=%lld outside [0, max_batch_utts=%d]",
            (long long)U, ctx->maxU);
  IVX_CHECK(U == 0 || (n && f && phi), "tv_estep: null n / f / phi");
  IVX_CHECK(prec == IVX_FP32 || prec == IVX_BF16, "tv_estep: unknown precision %d", (int)prec);
  if (U == 0) return IVX_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("tv_estep: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  return estep_impl(ctx, n, f, U, prec, phi, Phi, ll_acc, info, as_stream(stream));
}

ivx_status tv_mstep_accumulate(ivx_ctx* ctx, const float* n, const float* f, const float* phi,
                               const float* Phi, int64_t U, const ivx_accum* acc, void* stream) {
  IVX_CHECK(ctx && acc, "tv_mstep_accumulate: null argument");
  IVX_CHECK(U >= 0 && U <= ctx->maxU, "tv_mstep_accumulate: U=%lld outside [0, %d]",
            (long long)U, ctx->maxU);
  IVX_CHECK(U == 0 || (n && f && phi && Phi), "tv_mstep_accumulate: null input");
  IVX_CHECK(acc->A && acc->Cc && acc->N && acc->h && acc->H && acc->count,
            "tv_mstep_accumulate: null accumulator");
  if (U == 0) return IVX_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("tv_mstep_accumulate: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  hipStream_t s = as_stream(stream);
  const int C = ctx->C, D = ctx->D, R = ctx->R;
  ProfScope ps(ctx, PK_ACCUM, s);
  launch_packed_to_psi(ctx, Phi, phi, U, ctx->Psi64, s);
  // A_c += sum_u n_c(u) Psi(u), Cc_c += sum_u f_c(u) phi(u)^T: FP64 products and sums
  gemm64_tn(n, C, ctx->Psi64, true, ctx->TP, acc->A, ctx->TP, C, (int)ctx->TP, (int)U, s);
  gemm64_tn(f, (int64_t)C * D, phi, false, R, acc->Cc, R, C * D, R, (int)U, s);
  launch_colsums(ctx, n, phi, ctx->Psi64, U, acc, s);
  return after_launch("tv_mstep_accumulate");
}

ivx_status extract_ivectors(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                            int64_t F, ivx_precision prec, ivx_selection sel, float* phi,
                            void* stream) {
  IVX_CHECK(ctx, "extract_ivectors: null context");
  IVX_CHECK(ctx->ubm_set && ctx->tv_set, "extract_ivectors: UBM and TV model required");
  IVX_CHECK(U >= 1 && U <= ctx->maxU, "extract_ivectors: U=%lld outside [1, %d]", (long long)U,
            ctx->maxU);
  IVX_CHECK(F >= 0 && F <= ctx->maxF, "extract_ivectors: F=%lld outside [0, %lld]", (long long)F,
            (long long)ctx->maxF);
  IVX_CHECK(utt_off && phi && (F == 0 || X), "extract_ivectors: null argument");
  IVX_CHECK(prec == IVX_FP32 || prec == IVX_BF16, "extract_ivectors: unknown precision");
  IVX_CHECK(sel == IVX_SEL_ALL || (sel == IVX_SEL_LEARNED && ctx->sel) ||
                (sel == IVX_SEL_PRUNED && ctx->presel),
            "extract_ivectors: unknown selection, or a selection that was not set up");
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("extract_ivectors: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  hipStream_t s = as_stream(stream);
  const NfTarget nf = launch_frame_utt(ctx, utt_off, U, F, s);
  launch_posteriors(ctx, X, F, prec, sel, ctx->post_idx, ctx->post_val, ctx->frame_ll, s, &nf);
  {
    ProfScope ps(ctx, PK_STATS_NF, s);
    launch_nf_finish(ctx, U, ctx->n_ws, ctx->f_ws, s);
  }
  ivx_status st = after_launch("extract_ivectors");
  if (st != IVX_OK) return st;
  return estep_impl(ctx, ctx->n_ws, ctx->f_ws, U, prec, phi, nullptr, nullptr, nullptr, s);
}

ivx_status tv_mstep_solve(ivx_ctx* ctx, const ivx_accum* acc, const double* S, int update_sigma,
                          const double* ll_sum_dev, double* objective, int32_t* status,
                          void* stream) {
  IVX_CHECK(ctx && acc && S, "tv_mstep_solve: null argument");
  IVX_CHECK(ctx->tv_set, "tv_mstep_solve: no TV model");
  IVX_CHECK(acc->A && acc->Cc && acc->N, "tv_mstep_solve: null accumulator");
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("tv_mstep_solve: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  hipStream_t s = as_stream(stream);
  ivx_status st = ensure_tv(ctx, s);
  if (st != IVX_OK) return st;
  {
    ProfScope ps(ctx, PK_MSTEP, s);
    if (objective) launch_objective(ctx, acc->N, S, ll_sum_dev, objective, s);
    launch_mstep_solve(ctx, acc, S, update_sigma, status ? status : ctx->mstat, s);
  }
  ctx->tv_dirty = true;
  return after_launch("tv_mstep_solve");
}

ivx_status tv_mindiv(ivx_ctx* ctx, const ivx_accum* acc, int method, void* stream) {
  IVX_CHECK(ctx && acc, "tv_mindiv: null argument");
  IVX_CHECK(ctx->tv_set, "tv_mindiv: no TV model");
  IVX_CHECK(acc->h && acc->H && acc->count, "tv_mindiv: null accumulator");
  IVX_CHECK(method == 0, "tv_mindiv: method %d not available (0 = Cholesky whitening)", method);
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("tv_mindiv: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  ivx_status st;
  {
    ProfScope ps(ctx, PK_MINDIV, as_stream(stream));
    st = launch_mindiv(ctx, acc, ctx->standard, false, as_stream(stream));
  }
  ctx->tv_dirty = true;
  if (st != IVX_OK) return st;
  return after_launch("tv_mindiv");
}

ivx_status tv_mindiv_standard(ivx_ctx* ctx, const ivx_accum* acc, int method, int update_mean,
                              void* stream) {
  IVX_CHECK(ctx && acc, "tv_mindiv_standard: null argument");
  IVX_CHECK(ctx->tv_set, "tv_mindiv_standard: no TV model");
  IVX_CHECK(ctx->standard, "tv_mindiv_standard: the context holds the augmented formulation");
  IVX_CHECK(acc->h && acc->H && acc->count, "tv_mindiv_standard: null accumulator");
  IVX_CHECK(method == 0, "tv_mindiv_standard: method %d not available (0 = Cholesky whitening)",
            method);
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("tv_mindiv_standard: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  ivx_status st;
  {
    ProfScope ps(ctx, PK_MINDIV, as_stream(stream));
    st = launch_mindiv(ctx, acc, true, update_mean != 0, as_stream(stream));
  }
  ctx->tv_dirty = true;
  if (st != IVX_OK) return st;
  return after_launch("tv_mindiv_standard");
}

}  // extern "C"
