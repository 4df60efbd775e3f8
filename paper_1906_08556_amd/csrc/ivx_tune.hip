// Autotuner: times the candidate launch shapes of the hot-path kernels on the
// caller's workload with HIP events and keeps the fastest in the context.
//   frame GEMM (FP32 and BF16 forms): 256 components per launch, or 128
//   with one or two 32-frame blocks per wave
//   n/f statistics: 128 or 256 components per workgroup
//   linear-term GEMM b = p + F V: number of K splits
#include <cmath>

#include "ivx_internal.h"

using namespace ivx;

namespace {

#define TUNE_CHECK(cond, ...)      \
  do {                             \
    if (!(cond)) {                 \
      set_error(__VA_ARGS__);      \
      return IVX_EINVAL;           \
    }                              \
  } while (0)

bool valid_tuning(const ivx_tuning& t) {
  auto ncb_ok = [](int v) { return v == 2 || v == 4 || v == 8; };
  return ncb_ok(t.frame_ncb) && ncb_ok(t.frame_ncb_bf16) &&
         t.b_split >= 0 && t.b_split <= 1024 && (t.frame_direct == 0 || t.frame_direct == 1) &&
         (t.mstep_left == 0 || t.mstep_left == 1) && (t.estep_global == 0 || t.estep_global == 1) &&
         (t.mstep_global == 0 || t.mstep_global == 1);
}

struct Timer {
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = false;
  explicit Timer(hipStream_t st) : s(st) {
    ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  }
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  // best of `reps` timed runs after one untimed run; ms, or INFINITY on error
  template <typename Fn>
  float best(Fn fn, int reps = 3) {
    fn();
    float b = INFINITY;
    for (int r = 0; r < reps; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) return INFINITY;
      fn();
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return INFINITY;
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return INFINITY;
      b = std::fmin(b, ms);
    }
    return b;
  }
};

}  // namespace

extern "C" {

ivx_status ivx_tuning_get(const ivx_ctx* ctx, ivx_tuning* out) {
  TUNE_CHECK(ctx && out, "ivx_tuning_get: null argument");
  *out = ctx->tune;
  return IVX_OK;
}

ivx_status ivx_tuning_set(ivx_ctx* ctx, const ivx_tuning* t) {
  TUNE_CHECK(ctx && t, "ivx_tuning_set: null argument");
  TUNE_CHECK(valid_tuning(*t), "ivx_tuning_set: value outside the candidate lists");
  ctx->tune = *t;
  return IVX_OK;
}

ivx_status ivx_autotune(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                        int64_t F, ivx_tuning* out, void* stream) {
  TUNE_CHECK(ctx && X && utt_off, "ivx_autotune: null argument");
  TUNE_CHECK(ctx->ubm_set && ctx->tv_set, "ivx_autotune: UBM and TV model required");
  TUNE_CHECK(U >= 1 && U <= ctx->maxU, "ivx_autotune: U=%lld outside [1, %d]", (long long)U,
             ctx->maxU);
  TUNE_CHECK(F >= 1 && F <= ctx->maxF, "ivx_autotune: F=%lld outside [1, %lld]", (long long)F,
             (long long)ctx->maxF);
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("ivx_autotune: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Timer tm(s);
  if (!tm.ok) {
    set_error("ivx_autotune: hipEventCreate failed");
    return IVX_EDEVICE;
  }
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  ivx_tuning best = ctx->tune;
  // frame GEMM, both forms; the FP32 one staged through LDS or direct
  for (int prec = 0; prec < 2; ++prec) {
    float tb = INFINITY;
    for (int v = 0; v < (prec == IVX_BF16 ? 3 : 5); ++v) {
      const int ncb = v < 3 ? (v == 0 ? 8 : v == 1 ? 4 : 2) : (v == 3 ? 8 : 4);
      const int direct = v >= 3 ? 1 : 0;
      if (prec == IVX_BF16) {
        ctx->tune.frame_ncb_bf16 = ncb;
      } else {
        ctx->tune.frame_ncb = ncb;
        ctx->tune.frame_direct = direct;
      }
      const float t = tm.best([&] { launch_frame_select(ctx, X, F, prec, s); });
      // the first candidate (256 components, staged) is kept unless another
      // is clearly faster
      if (t < 0.99f * tb) {
        tb = t;
        if (prec == IVX_BF16) {
          best.frame_ncb_bf16 = ncb;
        } else {
          best.frame_ncb = ncb;
          best.frame_direct = direct;
        }
      }
    }
  }
  ctx->tune = best;
  // statistics of the workload: the first-order ones are the linear term's input
  {
    const NfTarget nf = launch_frame_utt(ctx, utt_off, U, F, s);
    launch_frame_select(ctx, X, F, IVX_FP32, s);
    launch_rescore(ctx, X, F, IVX_FP32, ctx->post_idx, ctx->post_val, ctx->frame_ll, s, nullptr,
                   nullptr, &nf);
    launch_nf_finish(ctx, U, ctx->n_ws, ctx->f_ws, s);
  }
  ivx_status st = ensure_tv_ready(ctx, s);
  if (st == IVX_OK) {
    float tb = INFINITY;
    for (int ns : {1, 2, 4, 8, 16, 32, 64}) {
      if (ns > ctx->nsplit_max) break;
      const float t = tm.best([&] { st = launch_linear_term(ctx, ctx->f_ws, U, ns, s); });
      if (st != IVX_OK) break;
      if (t < tb) {
        tb = t;
        best.b_split = ns;
      }
    }
  }
  ctx->tune = best;
  ctx->prof_on = prof;
  if (st != IVX_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
    set_error("ivx_autotune: a timed launch failed");
    return IVX_EDEVICE;
  }
  if (out) *out = best;
  return IVX_OK;
}

}  // extern "C"
