// ubm_posteriors_static: frame posteriors over all C components whose
// frame-stage workspace (candidate lists, running maxima, overflow flags,
// exact scores, the component-sorted slot list and its histograms) lives in
// a fixed device array of this library instead of the context's buffers, so
// the call allocates nothing and needs no workspace sized for the batch.
//
// The array is resolved once per device by ivx_create (with that device
// current) through hipGetSymbolAddress; host code only ever uses the
// resolved address, never the array's own name.  Every call on a device
// shares that device's array: calls that overlap on one device (two streams,
// two host threads) race, and each call overwrites everything it reads, so
// nothing has to be cleared between calls.
#include <mutex>

#include "ivx_internal.h"

namespace {
constexpr size_t kStaticBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Bytes of the workspace for F frames and C components, with each piece
// 256-byte aligned; *off receives the offsets of the seven pieces.
size_t static_layout(int64_t F, int C, size_t off[7]) {
  const size_t f = (size_t)F, kp = ivx::KP;
  const size_t nhist = (size_t)((F + 8191) / 8192);
  const size_t sz[7] = {f * kp * sizeof(int2),   // cand
                        f * sizeof(float),       // cM
                        f * sizeof(int),         // cflag
                        f * kp * sizeof(double), // lscore
                        f * kp * sizeof(int2),   // ent
                        nhist * C * sizeof(int), // hist
                        ((size_t)C + 1) * sizeof(int)};  // coff
  size_t o = 0;
  for (int i = 0; i < 7; ++i) {
    off[i] = o;
    o += align256(sz[i] > 0 ? sz[i] : 1);
  }
  return o;
}
}  // namespace

namespace ivx {

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

}  // namespace ivx

extern "C" {

int64_t ivx_static_bytes(void) { return (int64_t)kStaticBytes; }

ivx_status ubm_posteriors_static(ivx_ctx* ctx, const float* X, int64_t F, ivx_precision prec,
                                 int32_t* post_idx, float* post_val, int32_t K, double* frame_ll,
                                 void* stream) {
  if (!ctx) {
    ivx::set_error("ubm_posteriors_static: null context");
    return IVX_EINVAL;
  }
  if (!ctx->ubm_set) {
    ivx::set_error("ubm_posteriors_static: no UBM loaded (ivx_set_ubm)");
    return IVX_EINVAL;
  }
  if (prec != IVX_FP32 && prec != IVX_BF16) {
    ivx::set_error("ubm_posteriors_static: unknown precision %d", (int)prec);
    return IVX_EINVAL;
  }
  if (K != ivx::KP || !post_idx || !post_val) {
    ivx::set_error("ubm_posteriors_static: post_idx and post_val [F][%d] are required (K=%d)",
                   ivx::KP, (int)K);
    return IVX_EINVAL;
  }
  if (F < 0 || F > (int64_t(1) << 26) || (F > 0 && !X)) {
    ivx::set_error("ubm_posteriors_static: F=%lld out of range or null X", (long long)F);
    return IVX_EINVAL;
  }
  size_t off[7];
  const size_t need = static_layout(F, ctx->C, off);
  if (need > kStaticBytes) {
    ivx::set_error("ubm_posteriors_static: F=%lld frames at C=%d need %zu bytes, more than the "
                   "%zu-byte static workspace (about 392 + C/2048 bytes per frame)",
                   (long long)F, ctx->C, need, kStaticBytes);
    return IVX_EINVAL;
  }
  if (F == 0) return IVX_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ivx::set_error("ubm_posteriors_static: hipSetDevice(%d) failed", ctx->device);
    return IVX_EDEVICE;
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
  }
  if (!base) {
    ivx::set_error("ubm_posteriors_static: static workspace of device %d not resolved",
                   ctx->device);
    return IVX_EDEVICE;
  }
  // the context's model with the workspace pointers moved into the array
  ivx_ctx w = *ctx;
  char* b = static_cast<char*>(base);
  w.cand = reinterpret_cast<int2*>(b + off[0]);
  w.cM = reinterpret_cast<float*>(b + off[1]);
  w.cflag = reinterpret_cast<int*>(b + off[2]);
  w.lscore = reinterpret_cast<double*>(b + off[3]);
  w.ent = reinterpret_cast<int2*>(b + off[4]);
  w.hist = reinterpret_cast<int*>(b + off[5]);
  w.coff = reinterpret_cast<int*>(b + off[6]);
  w.prof_on = false;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ivx::launch_posteriors(&w, X, F, prec, IVX_SEL_ALL, post_idx, post_val, frame_ll, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ivx::set_error("ubm_posteriors_static: kernel launch failed: %s", hipGetErrorString(e));
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

}  // extern "C"
