// Streaming host pipeline (Sec. 4.2, Fig. 1): fixed-size batches of
// utterances read from host memory (or produced by a caller's source) by
// loader threads into pinned slots, uploaded on a copy stream into one of two
// device buffers, and processed on the caller's stream while the next batch
// is in flight.  Device memory is bounded by the batch limits, not by the
// size of the corpus.  Host code only; the per-batch work is the ordinary
// hot-path calls.
#include <cstring>
#include <thread>
#include <vector>

#include "ivx_internal.h"
#include "ivx_stream_engine.h"

using namespace ivx;

struct ivx_stream {
  ivx_ctx* ctx = nullptr;
  ivx_stream_config cfg{};
  int D = 0, R = 0, C = 0;
  // pinned host slots
  std::vector<float*> hX;
  std::vector<int64_t*> hoff;
  std::vector<int64_t> hU, hF;  // utterances / frames held by each slot
  // device double buffer and per-batch workspace
  float* dX[2] = {nullptr, nullptr};
  int64_t* doff[2] = {nullptr, nullptr};
  float* n = nullptr;    // [max_utts][C]
  float* f = nullptr;    // [max_utts][C][D]
  float* phi = nullptr;  // [max_utts][R]
  float* Phi = nullptr;  // [max_utts][R(R+1)/2]
  hipStream_t copy = nullptr;
  std::vector<hipEvent_t> copied;  // per slot: its upload has finished
  hipEvent_t computed[2] = {nullptr, nullptr};  // per device buffer: last use done
  // per device buffer: computed[] holds a recorded use.  Kept across passes:
  // a pass returns before the GPU has finished its last batches, so the next
  // pass's first uploads must wait for them too.
  bool used[2] = {false, false};
};

namespace {

#define ST_CHECK(cond, ...)   \
  do {                        \
    if (!(cond)) {            \
      set_error(__VA_ARGS__); \
      return IVX_EINVAL;      \
    }                         \
  } while (0)

#define ST_HIP(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));                  \
      return IVX_EDEVICE;                                                        \
    }                                                                            \
  } while (0)

void stream_free(ivx_stream* st) {
  for (float* p : st->hX)
    if (p) (void)hipHostFree(p);
  for (int64_t* p : st->hoff)
    if (p) (void)hipHostFree(p);
  for (int i = 0; i < 2; ++i) {
    if (st->dX[i]) (void)hipFree(st->dX[i]);
    if (st->doff[i]) (void)hipFree(st->doff[i]);
    if (st->computed[i]) (void)hipEventDestroy(st->computed[i]);
  }
  for (hipEvent_t e : st->copied)
    if (e) (void)hipEventDestroy(e);
  void* ptrs[] = {st->n, st->f, st->phi, st->Phi};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (st->copy) (void)hipStreamDestroy(st->copy);
  delete st;
}

// Checks host offsets and plans the batches.
ivx_status plan(const ivx_stream* st, const int64_t* utt_off, int64_t U, const char* fn,
                std::vector<int64_t>& starts) {
  ST_CHECK(utt_off && U >= 0, "%s: null utt_off or negative U", fn);
  ST_CHECK(utt_off[0] == 0, "%s: utt_off[0] must be 0", fn);
  const int64_t nb = plan_batches(utt_off, U, st->cfg.max_batch_utts, st->cfg.max_batch_frames,
                                  starts);
  ST_CHECK(nb >= 0, "%s: utterance %lld is longer than max_batch_frames=%lld or has a negative "
                    "length", fn, (long long)(-1 - nb), (long long)st->cfg.max_batch_frames);
  return IVX_OK;
}

// Runs one pass: loaders fill slots from X (or src), the calling thread
// uploads each batch and hands it to work(b, u0, Ub, Fb, dX, doff).
template <class Work>
ivx_status run_pass(ivx_stream* st, const float* X, ivx_frame_source src, void* user,
                    const int64_t* utt_off, const std::vector<int64_t>& starts, hipStream_t s,
                    Work work) {
  const int64_t nb = (int64_t)starts.size() - 1;
  if (nb <= 0) return IVX_OK;
  const int D = st->D;
  const int nslots = st->cfg.slots;
  BatchRing ring(nslots, nb);
  auto fill = [&](int64_t b, int slot) -> bool {
    const int64_t u0 = starts[b], u1 = starts[b + 1];
    const int64_t t0 = utt_off[u0], Fb = utt_off[u1] - t0;
    int64_t* off = st->hoff[slot];
    for (int64_t u = u0; u <= u1; ++u) off[u - u0] = utt_off[u] - t0;
    st->hU[slot] = u1 - u0;
    st->hF[slot] = Fb;
    if (src) return src(user, u0, u1, utt_off, st->hX[slot]) == 0;
    if (Fb > 0) std::memcpy(st->hX[slot], X + t0 * D, sizeof(float) * (size_t)Fb * D);
    return true;
  };
  const int nl = (int)std::min<int64_t>(st->cfg.loaders, nb);
  std::vector<std::thread> loaders;
  loaders.reserve(nl);
  for (int i = 0; i < nl; ++i) loaders.emplace_back([&] { ring.loader_loop(fill); });

  ivx_status status = IVX_OK;
  bool* used = st->used;
  int64_t issued = 0;
  // the per-batch workspace (n, f, phi, Phi) is reused by this pass on `s`;
  // the previous pass may have run on another stream
  for (int i = 0; i < 2 && status == IVX_OK; ++i)
    if (used[i] && hipStreamWaitEvent(s, st->computed[i], 0) != hipSuccess) {
      set_error("ivx_stream: stream wait failed");
      status = IVX_EDEVICE;
    }
  for (int64_t b = 0; b < nb && status == IVX_OK; ++b) {
    if (!ring.wait_ready(b)) break;
    const int slot = ring.slot_of(b);
    const int db = (int)(b & 1);
    hipError_t e = hipSuccess;
    // the device buffer's previous batch must be done before it is overwritten
    if (used[db]) e = hipStreamWaitEvent(st->copy, st->computed[db], 0);
    const int64_t Ub = st->hU[slot], Fb = st->hF[slot];
    if (e == hipSuccess && Fb > 0)
      e = hipMemcpyAsync(st->dX[db], st->hX[slot], sizeof(float) * (size_t)Fb * D,
                         hipMemcpyHostToDevice, st->copy);
    if (e == hipSuccess)
      e = hipMemcpyAsync(st->doff[db], st->hoff[slot], sizeof(int64_t) * (size_t)(Ub + 1),
                         hipMemcpyHostToDevice, st->copy);
    if (e == hipSuccess) e = hipEventRecord(st->copied[slot], st->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, st->copied[slot], 0);
    if (e != hipSuccess) {
      set_error("ivx_stream: upload of batch %lld failed: %s", (long long)b, hipGetErrorString(e));
      status = IVX_EDEVICE;
      break;
    }
    issued = b + 1;
    status = work(b, starts[b], Ub, Fb, st->dX[db], st->doff[db]);
    // recorded even after a failed call, so that later uploads still wait for
    // whatever it managed to enqueue
    if (hipEventRecord(st->computed[db], s) != hipSuccess && status == IVX_OK) {
      set_error("ivx_stream: event record failed");
      status = IVX_EDEVICE;
    }
    used[db] = true;
    if (status != IVX_OK) break;
    if (b >= 1) {  // batch b - 1 has been uploaded once its event completes
      if (hipEventSynchronize(st->copied[ring.slot_of(b - 1)]) != hipSuccess) {
        set_error("ivx_stream: upload wait failed");
        status = IVX_EDEVICE;
        break;
      }
      ring.release(b - 1);
    }
  }
  ring.stop();
  for (auto& t : loaders) t.join();
  // no slot may be rewritten while an upload still reads it
  if (issued > 0 && hipStreamSynchronize(st->copy) != hipSuccess && status == IVX_OK) {
    set_error("ivx_stream: copy stream failed");
    status = IVX_EDEVICE;
  }
  if (status == IVX_OK && issued < nb) {
    set_error(ring.failed() ? "ivx_stream: the frame source reported an error"
                            : "ivx_stream: pass stopped early");
    status = IVX_EINVAL;
  }
  return status;
}

}  // namespace

extern "C" {

ivx_status ivx_plan_batches(const int64_t* utt_off, int64_t U, int32_t max_utts,
                            int64_t max_frames, int64_t* starts, int64_t cap, int64_t* nbatches) {
  ST_CHECK(utt_off && nbatches && U >= 0, "ivx_plan_batches: null argument or negative U");
  ST_CHECK(max_utts >= 1 && max_frames >= 1, "ivx_plan_batches: limits must be >= 1");
  ST_CHECK(utt_off[0] == 0, "ivx_plan_batches: utt_off[0] must be 0");
  std::vector<int64_t> st;
  const int64_t nb = plan_batches(utt_off, U, max_utts, max_frames, st);
  ST_CHECK(nb >= 0, "ivx_plan_batches: utterance %lld is longer than max_frames or has a "
                    "negative length", (long long)(-1 - nb));
  *nbatches = nb;
  ST_CHECK(starts && cap >= nb + 1, "ivx_plan_batches: starts needs %lld entries",
           (long long)(nb + 1));
  std::memcpy(starts, st.data(), sizeof(int64_t) * (size_t)(nb + 1));
  return IVX_OK;
}

ivx_status ivx_stream_create(ivx_ctx* ctx, const ivx_stream_config* cfg, ivx_stream** out) {
  ST_CHECK(ctx && cfg && out, "ivx_stream_create: null argument");
  *out = nullptr;
  ST_CHECK(cfg->max_batch_utts >= 1 && cfg->max_batch_utts <= ctx->maxU,
           "ivx_stream_create: max_batch_utts=%d outside [1, %d] (the context's limit)",
           cfg->max_batch_utts, ctx->maxU);
  ST_CHECK(cfg->max_batch_frames >= 1 && cfg->max_batch_frames <= ctx->maxF,
           "ivx_stream_create: max_batch_frames=%lld outside [1, %lld] (the context's limit)",
           (long long)cfg->max_batch_frames, (long long)ctx->maxF);
  ST_CHECK(cfg->loaders >= 1 && cfg->loaders <= 64, "ivx_stream_create: loaders must be 1..64");
  ST_CHECK(cfg->slots >= 2 && cfg->slots <= 16, "ivx_stream_create: slots must be 2..16");
  ST_HIP(hipSetDevice(ctx->device));
  ivx_stream* st = new ivx_stream();
  st->ctx = ctx;
  st->cfg = *cfg;
  st->D = ctx->D;
  st->R = ctx->R;
  st->C = ctx->C;
  const size_t U = cfg->max_batch_utts, F = (size_t)cfg->max_batch_frames;
  const size_t C = ctx->C, D = ctx->D, R = ctx->R;
  bool ok = true;
  st->hX.assign(cfg->slots, nullptr);
  st->hoff.assign(cfg->slots, nullptr);
  st->hU.assign(cfg->slots, 0);
  st->hF.assign(cfg->slots, 0);
  st->copied.assign(cfg->slots, nullptr);
  for (int i = 0; i < cfg->slots && ok; ++i) {
    ok = hipHostMalloc(reinterpret_cast<void**>(&st->hX[i]), sizeof(float) * F * D,
                       hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&st->hoff[i]), sizeof(int64_t) * (U + 1),
                       hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&st->copied[i], hipEventDisableTiming) == hipSuccess;
  }
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipMalloc(reinterpret_cast<void**>(&st->dX[i]), sizeof(float) * F * D) == hipSuccess &&
         hipMalloc(reinterpret_cast<void**>(&st->doff[i]), sizeof(int64_t) * (U + 1)) ==
             hipSuccess &&
         hipEventCreateWithFlags(&st->computed[i], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipMalloc(reinterpret_cast<void**>(&st->n), sizeof(float) * U * C) == hipSuccess &&
       hipMalloc(reinterpret_cast<void**>(&st->f), sizeof(float) * U * C * D) == hipSuccess &&
       hipMalloc(reinterpret_cast<void**>(&st->phi), sizeof(float) * U * R) == hipSuccess &&
       hipMalloc(reinterpret_cast<void**>(&st->Phi), sizeof(float) * U * (R * (R + 1) / 2)) ==
           hipSuccess &&
       hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    stream_free(st);
    set_error("ivx_stream_create: allocation failed");
    return IVX_ENOMEM;
  }
  *out = st;
  return IVX_OK;
}

void ivx_stream_destroy(ivx_stream* st) {
  if (!st) return;
  (void)hipSetDevice(st->ctx->device);
  if (st->copy) (void)hipStreamSynchronize(st->copy);
  for (int i = 0; i < 2; ++i)  // the last batches may still be computing
    if (st->used[i]) (void)hipEventSynchronize(st->computed[i]);
  stream_free(st);
}

ivx_status ivx_stream_em_pass(ivx_stream* st, const float* X, ivx_frame_source src,
                              void* src_user, const int64_t* utt_off, int64_t U,
                              ivx_precision prec, ivx_selection sel, double* S_acc,
                              double* ll_frames, double* ll_utts, const ivx_accum* acc,
                              float* phi_out, void* stream) {
  ST_CHECK(st && acc, "ivx_stream_em_pass: null stream or accumulators");
  ST_CHECK((X != nullptr) != (src != nullptr),
           "ivx_stream_em_pass: give exactly one of X and a frame source");
  std::vector<int64_t> starts;
  ivx_status r = plan(st, utt_off, U, "ivx_stream_em_pass", starts);
  if (r != IVX_OK) return r;
  ST_HIP(hipSetDevice(st->ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int R = st->R;
  auto work = [&](int64_t, int64_t u0, int64_t Ub, int64_t Fb, const float* dX,
                  const int64_t* doff) -> ivx_status {
    float* phi = phi_out ? phi_out + (size_t)u0 * R : st->phi;
    ivx_status e = bw_stats(st->ctx, dX, doff, Ub, Fb, prec, sel, st->n, st->f, S_acc, ll_frames,
                            stream);
    if (e == IVX_OK)
      e = tv_estep(st->ctx, st->n, st->f, Ub, prec, phi, st->Phi, ll_utts, nullptr, stream);
    if (e == IVX_OK) e = tv_mstep_accumulate(st->ctx, st->n, st->f, phi, st->Phi, Ub, acc, stream);
    return e;
  };
  return run_pass(st, X, src, src_user, utt_off, starts, s, work);
}

ivx_status ivx_stream_extract(ivx_stream* st, const float* X, ivx_frame_source src,
                              void* src_user, const int64_t* utt_off, int64_t U,
                              ivx_precision prec, ivx_selection sel, float* phi, void* stream) {
  ST_CHECK(st && phi, "ivx_stream_extract: null stream or phi");
  ST_CHECK((X != nullptr) != (src != nullptr),
           "ivx_stream_extract: give exactly one of X and a frame source");
  std::vector<int64_t> starts;
  ivx_status r = plan(st, utt_off, U, "ivx_stream_extract", starts);
  if (r != IVX_OK) return r;
  ST_HIP(hipSetDevice(st->ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int R = st->R;
  auto work = [&](int64_t, int64_t u0, int64_t Ub, int64_t Fb, const float* dX,
                  const int64_t* doff) -> ivx_status {
    return extract_ivectors(st->ctx, dX, doff, Ub, Fb, prec, sel, phi + (size_t)u0 * R, stream);
  };
  return run_pass(st, X, src, src_user, utt_off, starts, s, work);
}

}  // extern "C"
