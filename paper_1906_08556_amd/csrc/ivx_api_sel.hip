// C-ABI of the learned Gaussian selection: set-up, training steps, network
// inspection and counters.  The selection itself runs inside ubm_posteriors,
// bw_stats and extract_ivectors when they are called with IVX_SEL_LEARNED.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ivx_internal.h"

using namespace ivx;

namespace ivx {

void selector_free(ivx_ctx* ctx) {
  if (!ctx || !ctx->sel) return;
  Selector* S = ctx->sel;
  void* ptrs[] = {S->param, S->grad, S->adam_m, S->adam_v, S->mean, S->stdv, S->istd, S->W1b,
                  S->W2b, S->W3b, S->b3p, S->h1b, S->h2b, S->prop, S->mass, S->fb, S->fb_list,
                  S->counters, S->score, S->thr, S->lscore, S->hist, S->coff, S->ent, S->xfb,
                  S->xs, S->a1, S->h1,
                  S->a2, S->h2, S->z, S->dz, S->dh1, S->dh2, S->loss_part, S->colpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);  // teardown
  delete S;
  ctx->sel = nullptr;
}

void presel_free(ivx_ctx* ctx) {
  if (!ctx || !ctx->presel) return;
  Presel* P = ctx->presel;
  void* ptrs[] = {P->Wd, P->pairs, P->prop, P->score, P->thr, P->lscore, P->hist, P->coff,
                  P->ent};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);  // teardown
  delete P;
  ctx->presel = nullptr;
}

// Posterior lists for frames [0, F): every component, the learned selection
// with the all-component fallback, or the pruned alignment.
void launch_posteriors(ivx_ctx* ctx, const float* X, int64_t F, int prec, int sel, int* post_idx,
                       float* post_val, double* frame_ll, hipStream_t s, const NfTarget* nf) {
  if (sel == IVX_SEL_PRUNED || sel == IVX_SEL_LEARNED) {
    if (sel == IVX_SEL_PRUNED)
      launch_select_pruned(ctx, X, F, post_idx, post_val, frame_ll, s);
    else
      launch_select_learned(ctx, X, F, prec, post_idx, post_val, frame_ll, s);
    if (nf) {
      ProfScope ps(ctx, PK_STATS_NF, s);
      launch_nf_accum(ctx, X, F, post_idx, post_val, *nf, s);
    }
    return;
  }
  launch_frame_select(ctx, X, F, prec, s);
  ProfScope ps(ctx, PK_RESCORE, s);
  launch_rescore(ctx, X, F, prec, post_idx, post_val, frame_ll, s, nullptr, nullptr, nf);
}

}  // namespace ivx

namespace {

#define SEL_CHECK(cond, ...)       \
  do {                             \
    if (!(cond)) {                 \
      set_error(__VA_ARGS__);      \
      return IVX_EINVAL;           \
    }                              \
  } while (0)

template <typename T>
bool salloc(T** p, int64_t n) {
  if (n <= 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), (size_t)n * sizeof(T)) == hipSuccess;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

ivx_status after_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

ivx_status set_device(ivx_ctx* ctx) {
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("hipSetDevice(%d) failed", ctx->device);
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

}  // namespace

extern "C" {

ivx_status ivx_feature_stats(ivx_ctx* ctx, const float* X, int64_t F, float* mean, float* stdv,
                             void* stream) {
  SEL_CHECK(ctx && X && mean && stdv, "ivx_feature_stats: null argument");
  SEL_CHECK(F >= 1 && F <= ctx->maxF, "ivx_feature_stats: F=%lld outside [1, %lld]",
            (long long)F, (long long)ctx->maxF);
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  launch_feature_stats(ctx, X, F, mean, stdv, as_stream(stream));
  return after_launch("ivx_feature_stats");
}

ivx_status ivx_selector_set(ivx_ctx* ctx, const ivx_selector_dims* sd, const float* params,
                            const float* mean, const float* stdv, void* stream) {
  SEL_CHECK(ctx && sd && params && mean && stdv, "ivx_selector_set: null argument");
  SEL_CHECK(sd->H1 >= 128 && sd->H1 <= 4096 && sd->H1 % 128 == 0 && sd->H2 >= 128 &&
                sd->H2 <= 4096 && sd->H2 % 128 == 0,
            "ivx_selector_set: hidden sizes must be multiples of 128 in [128, 4096]");
  SEL_CHECK(sd->k >= 1 && sd->k <= kMaxProposals && sd->k <= ctx->C,
            "ivx_selector_set: k=%d outside [1, min(%d, C)]", sd->k, kMaxProposals);
  SEL_CHECK(sd->min_mass >= 0.0f && sd->min_mass <= 1.0f,
            "ivx_selector_set: min_mass outside [0, 1]");
  SEL_CHECK(sd->max_train_batch >= 0 && sd->max_train_batch <= (1 << 20),
            "ivx_selector_set: max_train_batch outside [0, 2^20]");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("ivx_selector_set: stream synchronisation failed");
    return IVX_EDEVICE;
  }
  selector_free(ctx);
  Selector* S = new Selector();
  ctx->sel = S;
  const int64_t D = ctx->D, C = ctx->C, Cpad = ctx->Cpad, H1 = sd->H1, H2 = sd->H2;
  const int64_t maxF = ctx->maxF, k = sd->k, B = sd->max_train_batch;
  S->H1 = (int)H1;
  S->H2 = (int)H2;
  S->k = (int)k;
  S->Bmax = (int)B;
  S->min_mass = sd->min_mass;
  S->margin = selection_margin((int)k);
  S->oW1 = 0;
  S->ob1 = S->oW1 + H1 * D;
  S->oW2 = S->ob1 + H1;
  S->ob2 = S->oW2 + H2 * H1;
  S->oW3 = S->ob2 + H2;
  S->ob3 = S->oW3 + C * H2;
  S->P = S->ob3 + C;
  S->chunk = std::min<int64_t>(maxF, (int64_t)1 << 20);
  const int64_t nbh = maxF / 8192 + 1;
  bool ok = true;
  auto A = [&](bool r) { ok = ok && r; };
  A(salloc(&S->param, S->P));
  A(salloc(&S->grad, S->P));
  A(salloc(&S->adam_m, S->P));
  A(salloc(&S->adam_v, S->P));
  A(salloc(&S->mean, D));
  A(salloc(&S->stdv, D));
  A(salloc(&S->istd, D));
  A(salloc(&S->W1b, H1 * 64));
  A(salloc(&S->W2b, H2 * H1));
  A(salloc(&S->W3b, Cpad * H2));
  A(salloc(&S->b3p, Cpad));
  A(salloc(&S->h1b, S->chunk * H1));
  A(salloc(&S->h2b, S->chunk * H2));
  A(salloc(&S->prop, maxF * k));
  A(salloc(&S->mass, maxF));
  A(salloc(&S->fb, maxF));
  A(salloc(&S->fb_list, maxF));
  A(salloc(&S->counters, 4));
  A(salloc(&S->score, maxF * k));
  A(salloc(&S->thr, maxF));
  A(salloc(&S->lscore, maxF * k));
  A(salloc(&S->hist, nbh * C));
  A(salloc(&S->coff, C + 1));
  A(salloc(&S->ent, maxF * k));
  A(salloc(&S->xfb, maxF * D));
  if (B > 0) {
    A(salloc(&S->xs, B * D));
    A(salloc(&S->a1, B * H1));
    A(salloc(&S->h1, B * H1));
    A(salloc(&S->a2, B * H2));
    A(salloc(&S->h2, B * H2));
    A(salloc(&S->z, B * C));
    A(salloc(&S->dz, B * C));
    A(salloc(&S->dh1, B * H1));
    A(salloc(&S->dh2, B * H2));
    A(salloc(&S->loss_part, B));
    A(salloc(&S->colpart, 32 * std::max<int64_t>(C, std::max(H1, H2))));
  }
  if (!ok) {
    selector_free(ctx);
    (void)hipGetLastError();
    set_error("ivx_selector_set: device allocation failed");
    return IVX_ENOMEM;
  }
  ok = hipMemcpyAsync(S->param, params, sizeof(float) * S->P, hipMemcpyDeviceToDevice, s) ==
           hipSuccess &&
       hipMemcpyAsync(S->mean, mean, sizeof(float) * D, hipMemcpyDeviceToDevice, s) == hipSuccess &&
       hipMemcpyAsync(S->stdv, stdv, sizeof(float) * D, hipMemcpyDeviceToDevice, s) == hipSuccess &&
       hipMemsetAsync(S->adam_m, 0, sizeof(float) * S->P, s) == hipSuccess &&
       hipMemsetAsync(S->adam_v, 0, sizeof(float) * S->P, s) == hipSuccess &&
       hipMemsetAsync(S->counters, 0, sizeof(int) * 4, s) == hipSuccess;
  if (!ok) {
    selector_free(ctx);
    set_error("ivx_selector_set: upload failed");
    return IVX_EDEVICE;
  }
  launch_selector_inv_std(ctx, s);
  launch_selector_pack(ctx, s);
  return after_launch("ivx_selector_set");
}

ivx_status ivx_pruned_set(ivx_ctx* ctx, int32_t k, float prune, void* stream) {
  SEL_CHECK(ctx, "ivx_pruned_set: null context");
  SEL_CHECK(k >= 1 && k <= kMaxProposals && k <= ctx->C,
            "ivx_pruned_set: k=%d outside [1, min(%d, C)]", k, kMaxProposals);
  SEL_CHECK(prune >= 0.0f && prune < 0.5f, "ivx_pruned_set: prune outside [0, 0.5)");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) {
    set_error("ivx_pruned_set: stream synchronisation failed");
    return IVX_EDEVICE;
  }
  presel_free(ctx);
  Presel* P = new Presel();
  ctx->presel = P;
  const int64_t D = ctx->D, C = ctx->C, Cpad = ctx->Cpad, maxF = ctx->maxF;
  P->k = k;
  P->prune = prune;
  P->margin = selection_margin(k);
  P->Kd8 = (int)((1 + 2 * D + 7) / 8 * 8);
  bool ok = true;
  auto A = [&](bool r) { ok = ok && r; };
  A(salloc(&P->Wd, (int64_t)P->Kd8 * Cpad));
  A(salloc(&P->pairs, P->Kd8));
  A(salloc(&P->prop, maxF * k));
  A(salloc(&P->score, maxF * k));
  A(salloc(&P->thr, maxF));
  A(salloc(&P->lscore, maxF * k));
  A(salloc(&P->hist, (maxF / 8192 + 1) * C));
  A(salloc(&P->coff, C + 1));
  A(salloc(&P->ent, maxF * k));
  if (!ok) {
    presel_free(ctx);
    (void)hipGetLastError();
    set_error("ivx_pruned_set: device allocation failed");
    return IVX_ENOMEM;
  }
  // feature pairs (a | b << 8) over x~ = [1, x']: (0,0), (0,d), (d,d)
  std::vector<uint16_t> pr(P->Kd8, 0);
  for (int d = 1; d <= D; ++d) {
    pr[d] = (uint16_t)(0 | (d << 8));
    pr[D + d] = (uint16_t)(d | (d << 8));
  }
  if (hipMemcpy(P->pairs, pr.data(), sizeof(uint16_t) * P->Kd8, hipMemcpyHostToDevice) !=
      hipSuccess) {
    presel_free(ctx);
    set_error("ivx_pruned_set: upload failed");
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

ivx_status ivx_selector_get(ivx_ctx* ctx, float* params, void* stream) {
  SEL_CHECK(ctx && params, "ivx_selector_get: null argument");
  SEL_CHECK(ctx->sel, "ivx_selector_get: no selector set");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  if (hipMemcpyAsync(params, ctx->sel->param, sizeof(float) * ctx->sel->P,
                     hipMemcpyDeviceToDevice, as_stream(stream)) != hipSuccess) {
    set_error("ivx_selector_get: copy failed");
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

int64_t ivx_selector_param_count(const ivx_ctx* ctx) { return (ctx && ctx->sel) ? ctx->sel->P : 0; }

ivx_status ivx_selector_forward(ivx_ctx* ctx, const float* X, int64_t F, uint16_t* h1,
                                uint16_t* h2, float* z, int32_t* prop, float* mass,
                                int32_t* fallback, void* stream) {
  SEL_CHECK(ctx && (F == 0 || X), "ivx_selector_forward: null argument");
  SEL_CHECK(ctx->sel, "ivx_selector_forward: no selector set");
  SEL_CHECK(F >= 0 && F <= ctx->maxF, "ivx_selector_forward: F=%lld outside [0, %lld]",
            (long long)F, (long long)ctx->maxF);
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  if (F == 0) return IVX_OK;
  hipStream_t s = as_stream(stream);
  Selector& S = *ctx->sel;
  bool ok = launch_selector_mlp(ctx, X, F, h1, h2, z, s);
  if (prop)
    ok = ok && hipMemcpyAsync(prop, S.prop, sizeof(int) * F * S.k, hipMemcpyDeviceToDevice, s) ==
                   hipSuccess;
  if (mass)
    ok = ok && hipMemcpyAsync(mass, S.mass, sizeof(float) * F, hipMemcpyDeviceToDevice, s) ==
                   hipSuccess;
  if (fallback)
    ok = ok && hipMemcpyAsync(fallback, S.fb, sizeof(int) * F, hipMemcpyDeviceToDevice, s) ==
                   hipSuccess;
  if (!ok) {
    set_error("ivx_selector_forward: copy failed");
    return IVX_EDEVICE;
  }
  return after_launch("ivx_selector_forward");
}

static ivx_status check_train(ivx_ctx* ctx, const char* fn, const float* X, int64_t F,
                              const int64_t* fidx, int32_t B, const int32_t* post_idx,
                              const float* post_val) {
  SEL_CHECK(ctx && X && fidx && post_idx && post_val, "%s: null argument", fn);
  SEL_CHECK(ctx->sel, "%s: no selector set", fn);
  SEL_CHECK(B >= 1 && B <= ctx->sel->Bmax, "%s: batch %d outside [1, max_train_batch=%d]", fn,
            (int)B, ctx->sel->Bmax);
  SEL_CHECK(F >= 1 && F <= ((int64_t)1 << 40), "%s: F=%lld must be >= 1", fn, (long long)F);
  return IVX_OK;
}

ivx_status ivx_selector_grad(ivx_ctx* ctx, const float* X, int64_t F, const int64_t* frame_idx,
                             int32_t B, const int32_t* post_idx, const float* post_val,
                             float* grad, double* loss, void* stream) {
  ivx_status st = check_train(ctx, "ivx_selector_grad", X, F, frame_idx, B, post_idx, post_val);
  if (st != IVX_OK) return st;
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  if (!launch_selector_grad(ctx, X, F, frame_idx, B, post_idx, post_val, loss, s)) {
    set_error("ivx_selector_grad: GEMM variant not available");
    return IVX_EINVAL;
  }
  if (grad && hipMemcpyAsync(grad, ctx->sel->grad, sizeof(float) * ctx->sel->P,
                             hipMemcpyDeviceToDevice, s) != hipSuccess) {
    set_error("ivx_selector_grad: copy failed");
    return IVX_EDEVICE;
  }
  return after_launch("ivx_selector_grad");
}

ivx_status ivx_selector_train_step(ivx_ctx* ctx, const float* X, int64_t F,
                                   const int64_t* frame_idx, int32_t B, const int32_t* post_idx,
                                   const float* post_val, float lr, double* loss, void* stream) {
  ivx_status st =
      check_train(ctx, "ivx_selector_train_step", X, F, frame_idx, B, post_idx, post_val);
  if (st != IVX_OK) return st;
  SEL_CHECK(lr > 0.0f && std::isfinite(lr), "ivx_selector_train_step: bad learning rate");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  if (!launch_selector_grad(ctx, X, F, frame_idx, B, post_idx, post_val, loss, s)) {
    set_error("ivx_selector_train_step: GEMM variant not available");
    return IVX_EINVAL;
  }
  launch_selector_adam(ctx, lr, s);
  return after_launch("ivx_selector_train_step");
}

ivx_status ivx_selector_counts(ivx_ctx* ctx, int64_t* fallback_frames, int64_t* kept_pairs,
                               void* stream) {
  SEL_CHECK(ctx && fallback_frames && kept_pairs, "ivx_selector_counts: null argument");
  SEL_CHECK(ctx->sel, "ivx_selector_counts: no selector set");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  int c[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize(as_stream(stream)) != hipSuccess ||
      hipMemcpy(c, ctx->sel->counters, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("ivx_selector_counts: copy failed");
    return IVX_EDEVICE;
  }
  *fallback_frames = c[0];
  *kept_pairs = (int64_t)(unsigned)c[1];
  return IVX_OK;
}

}  // extern "C"
