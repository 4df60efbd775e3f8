// C ABI entry points: argument validation, context lifecycle, launch order.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ivx_internal.h"

namespace ivx {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int prof_begin(ivx_ctx* ctx, int k, hipStream_t s) {
  if (!ctx || !ctx->prof_on || ctx->prof_used >= ctx->prof_cap) return -1;
  const int slot = ctx->prof_used++;
  ctx->prof_kind[slot] = k;
  if (hipEventRecord(ctx->prof_ev[2 * slot], s) != hipSuccess) {
    --ctx->prof_used;  // slot not started: the group goes untimed
    return -1;
  }
  return slot;
}

void prof_end(ivx_ctx* ctx, int slot, hipStream_t s) {
  if (slot < 0) return;
  // a failed record leaves this slot out of the totals (no elapsed time)
  (void)hipEventRecord(ctx->prof_ev[2 * slot + 1], s);
}

static void prof_free(ivx_ctx* ctx) {
  if (ctx->prof_ev) {
    for (int i = 0; i < 2 * ctx->prof_cap; ++i) (void)hipEventDestroy(ctx->prof_ev[i]);
    delete[] ctx->prof_ev;
    delete[] ctx->prof_kind;
  }
  ctx->prof_ev = nullptr;
  ctx->prof_kind = nullptr;
  ctx->prof_cap = ctx->prof_used = 0;
  ctx->prof_on = false;
}

}  // namespace ivx

using namespace ivx;

#define IVX_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return IVX_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define IVX_CHECK(cond, ...)       \
  do {                             \
    if (!(cond)) {                 \
      set_error(__VA_ARGS__);      \
      return IVX_EINVAL;           \
    }                              \
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

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

// Expanded-feature index pairs (a, b), a <= b over x~ = [1, x_0..x_{D-1}],
// row by row; padding entries are (0, 0) with zero coefficients.
std::vector<uint16_t> make_pairs(int D, int Kpad) {
  std::vector<uint16_t> v;
  v.reserve(Kpad);
  for (int a = 0; a <= D; ++a)
    for (int b = a; b <= D; ++b) v.push_back((uint16_t)(a | (b << 8)));
  while ((int)v.size() < Kpad) v.push_back(0);
  return v;
}

ivx_status set_device(ivx_ctx* ctx) {
  IVX_HIP(hipSetDevice(ctx->device));
  return IVX_OK;
}

}  // namespace

extern "C" {

const char* ivx_last_error(void) { return g_err; }

int64_t ivx_tp_size(int32_t R) { return R > 0 ? tp_size(R) : 0; }

void ivx_destroy(ivx_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->prof_ev) {
    (void)hipDeviceSynchronize();
    prof_free(ctx);
  }
  selector_free(ctx);
  presel_free(ctx);
  void* ptrs[] = {ctx->w, ctx->mu, ctx->cov, ctx->shift, ctx->Wexp, ctx->W16, ctx->linv,
                  ctx->linv32r, ctx->ldense, ctx->cst,
                  ctx->pairs, ctx->T, ctx->Sigma, ctx->p, ctx->bias, ctx->bias32, ctx->cand, ctx->cM, ctx->cflag, ctx->post_idx,
                  ctx->post_val, ctx->frame_ll, ctx->lscore, ctx->hist, ctx->coff, ctx->ent, ctx->partial,
                  ctx->Y32, ctx->V32, ctx->Utp, ctx->Psig, ctx->sig_logdet, ctx->Lbuf, ctx->Wbuf, ctx->Psi64,
                  ctx->bpart, ctx->colpart, ctx->bvec, ctx->llu, ctx->n_ws, ctx->f_ws, ctx->Tnew, ctx->obj_part,
                  ctx->Gmat, ctx->Mmat, ctx->Winv, ctx->Ut16hi, ctx->Ut16lo, ctx->n16hi,
                  ctx->n16lo, ctx->mvec, ctx->mstat, ctx->dev_err, ctx->nf_acc, ctx->umap};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete ctx;
}

ivx_status ivx_create(const ivx_dims* dims, int device, ivx_ctx** out) {
  IVX_CHECK(dims && out, "ivx_create: null argument");
  *out = nullptr;
  IVX_CHECK(dims->C >= 1 && dims->C <= (1 << 20), "ivx_create: C=%d out of range", dims->C);
  IVX_CHECK(dims->D >= 1 && dims->D <= 63, "ivx_create: D=%d out of range [1, 63]", dims->D);
  IVX_CHECK(dims->R >= 2 && dims->R <= 480, "ivx_create: R=%d out of range [2, 480]", dims->R);
  IVX_CHECK(dims->max_batch_utts >= 1, "ivx_create: max_batch_utts must be >= 1");
  // candidate, posterior and proposal slots are addressed as frame * slots
  // in 32-bit ints (slots <= max(KP, kMaxProposals)), so every slot id of a
  // batch must stay below 2^31
  const int64_t max_frames = int64_t(INT32_MAX) / (KP > kMaxProposals ? KP : kMaxProposals);
  IVX_CHECK(dims->max_batch_frames >= 1 && dims->max_batch_frames <= max_frames,
            "ivx_create: max_batch_frames=%lld out of range [1, %lld]",
            (long long)dims->max_batch_frames, (long long)max_frames);
  int ndev = 0;
  IVX_HIP(hipGetDeviceCount(&ndev));
  IVX_CHECK(device >= 0 && device < ndev, "ivx_create: device %d not present (%d visible)", device,
            ndev);
  IVX_HIP(hipSetDevice(device));
  IVX_HIP(static_scratch_init(device));

  int ncu = 0;
  IVX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
  IVX_CHECK(ncu >= 1, "ivx_create: device %d reports %d compute units", device, ncu);

  ivx_ctx* c = new ivx_ctx();
  c->device = device;
  c->ncu = ncu;
  c->C = dims->C;
  c->D = dims->D;
  c->R = dims->R;
  c->maxU = dims->max_batch_utts;
  c->maxF = dims->max_batch_frames;
  c->K = (c->D + 1) * (c->D + 2) / 2;
  c->Kpad = (c->K + 15) / 16 * 16;
  c->Cpad = (c->C + 255) / 256 * 256;  // multiple of the frame GEMM component tile
  c->Dp = c->D * (c->D + 1) / 2;
  c->TP = tp_size(c->R);
  c->margin = candidate_margin(c->C);
  c->margin_bf16 = candidate_margin_bf16(c->C);
  c->nhist = (int)((c->maxF + 8191) / 8192);

  const size_t C = c->C, D = c->D, R = c->R, F = c->maxF;
  bool ok = true;
  auto A = [&](hipError_t e) { ok = ok && (e == hipSuccess); };
  A(dalloc(&c->w, C));
  A(dalloc(&c->mu, C * D));
  A(dalloc(&c->cov, C * D * D));
  A(dalloc(&c->shift, D));
  A(dalloc(&c->Wexp, (size_t)c->Cpad * c->Kpad));
  A(dalloc(&c->W16, (size_t)c->Cpad * c->Kpad * 2));
  A(dalloc(&c->linv, C * c->Dp));
  A(dalloc(&c->linv32r, C * c->Dp));
  A(dalloc(&c->ldense, C * 4096));
  A(dalloc(&c->cst, C));
  A(dalloc(&c->pairs, (size_t)c->Kpad));
  A(dalloc(&c->T, C * D * R));
  A(dalloc(&c->Sigma, C * D * D));
  A(dalloc(&c->p, R));
  A(dalloc(&c->bias, C * D));
  A(dalloc(&c->bias32, C * D));
  A(dalloc(&c->cand, F * KP));
  A(dalloc(&c->cM, F));
  A(dalloc(&c->cflag, F));
  A(dalloc(&c->post_idx, F * KP));
  A(dalloc(&c->post_val, F * KP));
  A(dalloc(&c->frame_ll, F));
  A(dalloc(&c->lscore, F * KP));
  A(dalloc(&c->hist, (size_t)c->nhist * C));
  A(dalloc(&c->coff, C + 1));
  A(dalloc(&c->ent, F * KP));
  A(dalloc(&c->partial, 1024));
  const size_t U = c->maxU, TP = c->TP;
  A(dalloc(&c->Y32, C * D * R));
  A(dalloc(&c->V32, C * D * R));
  A(dalloc(&c->Utp, C * TP));
  A(dalloc(&c->Psig, C * D * D));
  A(dalloc(&c->sig_logdet, C));
  A(dalloc(&c->Lbuf, U * TP));
  A(dalloc(&c->Wbuf, U * TP));
  A(dalloc(&c->Psi64, U * TP));
  A(dalloc(&c->bpart, (size_t)c->nsplit_max * U * R));
  A(dalloc(&c->colpart, (size_t)CSPLIT * (C + R + TP)));
  A(dalloc(&c->bvec, U * R));
  A(dalloc(&c->llu, U));
  A(dalloc(&c->n_ws, U * C));
  A(dalloc(&c->nf_acc, U * C * (D + 1)));
  A(dalloc(&c->umap, F));
  A(dalloc(&c->f_ws, U * C * D));
  A(dalloc(&c->Tnew, C * D * R));
  A(dalloc(&c->obj_part, C));
  A(dalloc(&c->Gmat, R * R));
  A(dalloc(&c->Mmat, R * R));
  A(dalloc(&c->Winv, (size_t)C * ((R + 15) / 16) * 256));
  {
    const size_t Ck = ((size_t)C + 7) / 8 * 8;
    A(dalloc(&c->Ut16hi, (size_t)TP * Ck));
    A(dalloc(&c->Ut16lo, (size_t)TP * Ck));
    A(dalloc(&c->n16hi, (size_t)U * Ck));
    A(dalloc(&c->n16lo, (size_t)U * Ck));
  }
  A(dalloc(&c->mvec, 4 * R));
  A(dalloc(&c->mstat, C));
  A(dalloc(&c->dev_err, 4));
  if (!ok) {
    ivx_destroy(c);
    (void)hipGetLastError();
    set_error("ivx_create: device allocation failed");
    return IVX_ENOMEM;
  }
  // the tile-packed U_c keeps zero padding (its GEMM never writes it)
  // the fixed-point n/f sums start (and are kept) at zero
  if (hipMemset(c->Utp, 0, sizeof(float) * C * TP) != hipSuccess ||
      hipMemset(c->nf_acc, 0, sizeof(unsigned long long) * U * C * (D + 1)) != hipSuccess) {
    ivx_destroy(c);
    set_error("ivx_create: memset failed");
    return IVX_EDEVICE;
  }
  std::vector<uint16_t> pairs = make_pairs(c->D, c->Kpad);
  int init_err[4] = {0, 0x7fffffff, -1, 0};
  if (hipMemcpy(c->pairs, pairs.data(), pairs.size() * sizeof(uint16_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(c->dev_err, init_err, sizeof(init_err), hipMemcpyHostToDevice) != hipSuccess) {
    ivx_destroy(c);
    set_error("ivx_create: upload failed");
    return IVX_EDEVICE;
  }
  if (!frame_set_attributes(c) || !select_set_attributes() || !mstep_set_attributes() ||
      !estep_rr_setup()) {
    ivx_destroy(c);
    set_error("ivx_create: hipFuncSetAttribute failed for a large-LDS kernel");
    return IVX_EDEVICE;
  }
  *out = c;
  return IVX_OK;
}

ivx_status ivx_sync_status(ivx_ctx* ctx, void* stream) {
  IVX_CHECK(ctx, "ivx_sync_status: null context");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  IVX_HIP(hipStreamSynchronize(as_stream(stream)));
  int e[4];
  IVX_HIP(hipMemcpy(e, ctx->dev_err, sizeof(e), hipMemcpyDeviceToHost));
  const int reset[4] = {0, 0x7fffffff, -1, 0};
  IVX_HIP(hipMemcpy(ctx->dev_err, reset, sizeof(reset), hipMemcpyHostToDevice));
  static const char* kSrc[PK_COUNT] = {"frame select", "rescoring", "n/f statistics",
                                       "second-order statistics", "TV precompute (Sigma_c)",
                                       "E-step GEMMs", "E-step Cholesky of L(u)",
                                       "accumulators", "M-step (A_c)", "minimum divergence (G)",
                                       "UBM preparation (covariance)",
                                       "learned selection (network)",
                                       "learned selection (scoring)",
                                       "learned selection (training batch)"};
  const char* src = (e[2] >= 0 && e[2] < PK_COUNT) ? kSrc[e[2]] : "?";
  const int idx = e[1] == 0x7fffffff ? -1 : e[1];
  switch (e[0]) {
    case 0:
      return IVX_OK;
    case IVX_ENOTPD:
      set_error("device: matrix not positive definite in %s (first index %d, %d events)", src, idx,
                e[3]);
      break;
    case IVX_EINVAL:
      set_error("device: malformed utterance offsets (utterance %d)", idx);
      break;
    case IVX_ENUMERIC:
      set_error("device: non-finite value in %s (index %d, %d events)", src, idx, e[3]);
      break;
    case IVX_ECAPACITY:
      set_error("device: frame %d has more than %d components within the posterior margin and "
                "the components beyond them carry more than %g of its mass (%d frames)",
                idx, KP, kMaxDroppedMass, e[3]);
      break;
    default:
      set_error("device: error %d in %s", e[0], src);
  }
  return (ivx_status)e[0];
}

ivx_status ivx_set_ubm(ivx_ctx* ctx, const double* w, const double* mu, const double* cov,
                       void* stream) {
  IVX_CHECK(ctx && w && mu && cov, "ivx_set_ubm: null argument");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  IVX_HIP(hipMemcpyAsync(ctx->w, w, sizeof(double) * ctx->C, hipMemcpyDeviceToDevice, s));
  IVX_HIP(hipMemcpyAsync(ctx->mu, mu, sizeof(double) * ctx->C * ctx->D, hipMemcpyDeviceToDevice, s));
  IVX_HIP(hipMemcpyAsync(ctx->cov, cov, sizeof(double) * ctx->C * ctx->D * ctx->D,
                         hipMemcpyDeviceToDevice, s));
  launch_ubm_prepare(ctx, s);
  ivx_status st = after_launch("ivx_set_ubm");
  if (st != IVX_OK) return st;
  st = ivx_sync_status(ctx, stream);
  if (st == IVX_ENOTPD) {
    char msg[512];
    snprintf(msg, sizeof(msg), "ivx_set_ubm: UBM covariance not positive definite (%s)",
             ivx_last_error());
    set_error("%s", msg);
  }
  if (st == IVX_OK) ctx->ubm_set = true;
  return st;
}

ivx_status ivx_init_tv(ivx_ctx* ctx, const double* T_rand, double p0, void* stream) {
  IVX_CHECK(ctx && T_rand, "ivx_init_tv: null argument");
  IVX_CHECK(ctx->ubm_set, "ivx_init_tv: call ivx_set_ubm first");
  IVX_CHECK(p0 > 0.0, "ivx_init_tv: p0 must be > 0");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  launch_init_tv(ctx, T_rand, p0, as_stream(stream));
  ctx->tv_set = true;
  ctx->tv_dirty = true;
  ctx->standard = false;
  return after_launch("ivx_init_tv");
}

ivx_status ivx_init_tv_standard(ivx_ctx* ctx, const double* T_rand, void* stream) {
  IVX_CHECK(ctx && T_rand, "ivx_init_tv_standard: null argument");
  IVX_CHECK(ctx->ubm_set, "ivx_init_tv_standard: call ivx_set_ubm first");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  launch_init_tv_standard(ctx, T_rand, as_stream(stream));
  ctx->tv_set = true;
  ctx->tv_dirty = true;
  ctx->standard = true;
  return after_launch("ivx_init_tv_standard");
}

ivx_status ivx_set_bias(ivx_ctx* ctx, const double* m, void* stream) {
  IVX_CHECK(ctx, "ivx_set_bias: null context");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  if (!m) {
    ctx->standard = false;
    return IVX_OK;
  }
  hipStream_t s = as_stream(stream);
  IVX_HIP(hipMemcpyAsync(ctx->bias, m, sizeof(double) * ctx->C * ctx->D, hipMemcpyDeviceToDevice,
                         s));
  launch_bias32(ctx, s);
  ctx->standard = true;
  return after_launch("ivx_set_bias");
}

ivx_status ivx_get_bias(ivx_ctx* ctx, double* m, void* stream) {
  IVX_CHECK(ctx && m, "ivx_get_bias: null argument");
  IVX_CHECK(ctx->standard, "ivx_get_bias: the context holds the augmented formulation (no bias)");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  IVX_HIP(hipMemcpyAsync(m, ctx->bias, sizeof(double) * ctx->C * ctx->D, hipMemcpyDeviceToDevice,
                         as_stream(stream)));
  return IVX_OK;
}

ivx_status ivx_set_tv(ivx_ctx* ctx, const double* T, const double* Sigma, const double* p,
                      void* stream) {
  IVX_CHECK(ctx && T && Sigma && p, "ivx_set_tv: null argument");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  const size_t C = ctx->C, D = ctx->D, R = ctx->R;
  IVX_HIP(hipMemcpyAsync(ctx->T, T, sizeof(double) * C * D * R, hipMemcpyDeviceToDevice, s));
  IVX_HIP(hipMemcpyAsync(ctx->Sigma, Sigma, sizeof(double) * C * D * D, hipMemcpyDeviceToDevice, s));
  IVX_HIP(hipMemcpyAsync(ctx->p, p, sizeof(double) * R, hipMemcpyDeviceToDevice, s));
  ctx->tv_set = true;
  ctx->tv_dirty = true;
  return IVX_OK;
}

ivx_status ivx_get_tv(ivx_ctx* ctx, double* T, double* Sigma, double* p, double* mu,
                      void* stream) {
  IVX_CHECK(ctx, "ivx_get_tv: null context");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  const size_t C = ctx->C, D = ctx->D, R = ctx->R;
  if (T) IVX_HIP(hipMemcpyAsync(T, ctx->T, sizeof(double) * C * D * R, hipMemcpyDeviceToDevice, s));
  if (Sigma)
    IVX_HIP(hipMemcpyAsync(Sigma, ctx->Sigma, sizeof(double) * C * D * D, hipMemcpyDeviceToDevice, s));
  if (p) IVX_HIP(hipMemcpyAsync(p, ctx->p, sizeof(double) * R, hipMemcpyDeviceToDevice, s));
  if (mu) IVX_HIP(hipMemcpyAsync(mu, ctx->mu, sizeof(double) * C * D, hipMemcpyDeviceToDevice, s));
  return IVX_OK;
}

static ivx_status check_frame_args(ivx_ctx* ctx, const char* fn, const float* X, int64_t F,
                                   ivx_precision prec, ivx_selection sel) {
  IVX_CHECK(ctx, "%s: null context", fn);
  IVX_CHECK(ctx->ubm_set, "%s: no UBM loaded (ivx_set_ubm)", fn);
  IVX_CHECK(F >= 0 && F <= ctx->maxF, "%s: F=%lld outside [0, max_batch_frames=%lld]", fn,
            (long long)F, (long long)ctx->maxF);
  IVX_CHECK(F == 0 || X, "%s: null X", fn);
  IVX_CHECK(prec == IVX_FP32 || prec == IVX_BF16, "%s: unknown precision %d", fn, (int)prec);
  IVX_CHECK(sel == IVX_SEL_ALL || sel == IVX_SEL_LEARNED || sel == IVX_SEL_PRUNED,
            "%s: unknown selection %d", fn, (int)sel);
  IVX_CHECK(sel != IVX_SEL_LEARNED || ctx->sel, "%s: IVX_SEL_LEARNED needs ivx_selector_set", fn);
  IVX_CHECK(sel != IVX_SEL_PRUNED || ctx->presel, "%s: IVX_SEL_PRUNED needs ivx_pruned_set", fn);
  return IVX_OK;
}

ivx_status ubm_posteriors(ivx_ctx* ctx, const float* X, int64_t F, ivx_precision prec,
                          ivx_selection sel, float* gamma, int32_t* post_idx, float* post_val,
                          int32_t K, double* frame_ll, void* stream) {
  ivx_status st = check_frame_args(ctx, "ubm_posteriors", X, F, prec, sel);
  if (st != IVX_OK) return st;
  IVX_CHECK(K == KP || (!post_idx && !post_val), "ubm_posteriors: K must be %d", KP);
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  int* pi = post_idx ? post_idx : ctx->post_idx;
  float* pv = post_val ? post_val : ctx->post_val;
  launch_posteriors(ctx, X, F, prec, sel, pi, pv, frame_ll, s);
  if (gamma) launch_dense_gamma(ctx, F, pi, pv, gamma, s);
  return after_launch("ubm_posteriors");
}

ivx_status bw_stats(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U, int64_t F,
                    ivx_precision prec, ivx_selection sel, float* n, float* f, double* S_acc,
                    double* ll_acc, void* stream) {
  ivx_status st = check_frame_args(ctx, "bw_stats", X, F, prec, sel);
  if (st != IVX_OK) return st;
  IVX_CHECK(U >= 1 && U <= ctx->maxU, "bw_stats: U=%lld outside [1, max_batch_utts=%d]",
            (long long)U, ctx->maxU);
  IVX_CHECK(utt_off && n && f, "bw_stats: null utt_off / n / f");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  hipStream_t s = as_stream(stream);
  // n/f are accumulated beside the posteriors (in the rescoring pass of the
  // all-component form) and converted once all frames are in
  const NfTarget nf = launch_frame_utt(ctx, utt_off, U, F, s);
  launch_posteriors(ctx, X, F, prec, sel, ctx->post_idx, ctx->post_val, ctx->frame_ll, s, &nf);
  {
    ProfScope ps(ctx, PK_STATS_NF, s);
    launch_nf_finish(ctx, U, n, f, s);
  }
  if (S_acc) {
    ProfScope ps(ctx, PK_STATS_S, s);
    launch_stats_S(ctx, X, F, S_acc, s);
  }
  if (ll_acc) launch_sum_f64(ctx, ctx->frame_ll, F, ll_acc, s);
  return after_launch("bw_stats");
}

ivx_status ivx_profile_enable(ivx_ctx* ctx, int32_t capacity) {
  IVX_CHECK(ctx, "ivx_profile_enable: null context");
  IVX_CHECK(capacity >= 0 && capacity <= (1 << 20), "ivx_profile_enable: bad capacity");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  IVX_HIP(hipDeviceSynchronize());
  prof_free(ctx);
  if (capacity == 0) return IVX_OK;
  ctx->prof_ev = new hipEvent_t[2 * capacity];
  ctx->prof_kind = new int[capacity];
  for (int i = 0; i < 2 * capacity; ++i) {
    if (hipEventCreate(&ctx->prof_ev[i]) != hipSuccess) {
      ctx->prof_cap = i / 2;
      prof_free(ctx);
      set_error("ivx_profile_enable: hipEventCreate failed");
      return IVX_EDEVICE;
    }
  }
  ctx->prof_cap = capacity;
  ctx->prof_used = 0;
  ctx->prof_on = true;
  return IVX_OK;
}

ivx_status ivx_profile_read(ivx_ctx* ctx, double* ms, int64_t* calls, int32_t n) {
  IVX_CHECK(ctx && ms && calls, "ivx_profile_read: null argument");
  IVX_CHECK(n >= 0 && n <= PK_COUNT, "ivx_profile_read: n=%d > %d groups", n, (int)PK_COUNT);
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  IVX_HIP(hipDeviceSynchronize());
  for (int i = 0; i < ctx->prof_used; ++i) {
    const int k = ctx->prof_kind[i];
    float t = 0.0f;
    if (k < n && hipEventElapsedTime(&t, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]) == hipSuccess) {
      ms[k] += t;
      calls[k] += 1;
    }
  }
  ctx->prof_used = 0;
  return IVX_OK;
}

ivx_status ubm_update_means(ivx_ctx* ctx, void* stream) {
  IVX_CHECK(ctx, "ubm_update_means: null context");
  IVX_CHECK(ctx->ubm_set && ctx->tv_set, "ubm_update_means: UBM and TV model required");
  IVX_CHECK(!ctx->standard,
            "ubm_update_means: realignment reads the augmented model (first columns of T_c)");
  if (set_device(ctx) != IVX_OK) return IVX_EDEVICE;
  {
    ProfScope ps(ctx, PK_UBM, as_stream(stream));
    launch_update_means(ctx, as_stream(stream));
  }
  return after_launch("ubm_update_means");
}

}  // extern "C"
