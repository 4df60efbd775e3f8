// One full EM iteration captured into a HIP graph (the iteration executor).
//
// The hot-path calls never allocate or synchronise and read no host-side
// state that changes between iterations, so their launch sequence can be
// recorded once and replayed.  Accumulators are cleared by a fill kernel
// inside the graph (no memset nodes).
#include "ivx_internal.h"

struct ivx_graph {
  ivx_ctx* ctx = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

__global__ void k_fill_f64(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void zero(double* p, int64_t n, hipStream_t s) {
  if (!p || n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill_f64<<<(unsigned)nb, 256, 0, s>>>(p, n);
}

}  // namespace

using namespace ivx;

extern "C" {

void ivx_graph_destroy(ivx_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
}

ivx_status ivx_graph_create_em(ivx_ctx* ctx, const float* X, const int64_t* utt_off, int64_t U,
                               int64_t F, ivx_precision prec, float* n, float* f, double* S,
                               float* phi, float* Phi, const ivx_accum* acc, double* ll_frames,
                               double* ll_utts, double* objective, int update_sigma, int realign,
                               ivx_graph** out) {
  if (!ctx || !out || !acc || !S || !ll_frames || !ll_utts || !objective || !Phi) {
    set_error("ivx_graph_create_em: null argument");
    return IVX_EINVAL;
  }
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("ivx_graph_create_em: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  ivx_graph* g = new ivx_graph();
  g->ctx = ctx;
  if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    set_error("ivx_graph_create_em: stream creation failed");
    return IVX_EDEVICE;
  }
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;     // no event nodes in the graph
  ctx->tv_dirty = true;     // the TV precompute is part of every iteration
  hipStream_t s = g->cap;
  ivx_status st = IVX_OK;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    ctx->prof_on = prof;
    ivx_graph_destroy(g);
    set_error("ivx_graph_create_em: hipStreamBeginCapture failed");
    return IVX_EDEVICE;
  }
  const int64_t C = ctx->C, D = ctx->D, R = ctx->R;
  zero(S, C * ctx->Dp, s);
  zero(ll_frames, 1, s);
  zero(ll_utts, 1, s);
  zero(acc->A, C * ctx->TP, s);
  zero(acc->Cc, C * D * R, s);
  zero(acc->N, C, s);
  zero(acc->h, R, s);
  zero(acc->H, ctx->TP, s);
  zero(acc->count, 1, s);
  void* sv = reinterpret_cast<void*>(s);
  if (st == IVX_OK)
    st = bw_stats(ctx, X, utt_off, U, F, prec, IVX_SEL_ALL, n, f, S, ll_frames, sv);
  if (st == IVX_OK) st = tv_estep(ctx, n, f, U, prec, phi, Phi, ll_utts, nullptr, sv);
  if (st == IVX_OK) st = tv_mstep_accumulate(ctx, n, f, phi, Phi, U, acc, sv);
  if (st == IVX_OK) st = tv_mstep_solve(ctx, acc, S, update_sigma, ll_utts, objective, nullptr, sv);
  if (st == IVX_OK) st = tv_mindiv(ctx, acc, 0, sv);
  if (st == IVX_OK && realign) st = ubm_update_means(ctx, sv);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  ctx->prof_on = prof;
  ctx->tv_dirty = true;
  if (st != IVX_OK || ec != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    ivx_graph_destroy(g);
    if (st == IVX_OK) {
      set_error("ivx_graph_create_em: stream capture failed: %s", hipGetErrorString(ec));
      st = IVX_EDEVICE;
    }
    return st;
  }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    ivx_graph_destroy(g);
    set_error("ivx_graph_create_em: hipGraphInstantiate failed");
    return IVX_EDEVICE;
  }
  *out = g;
  return IVX_OK;
}

ivx_status ivx_graph_launch(ivx_graph* g, void* stream) {
  if (!g || !g->exec) {
    set_error("ivx_graph_launch: null graph");
    return IVX_EINVAL;
  }
  if (hipSetDevice(g->ctx->device) != hipSuccess) {
    set_error("ivx_graph_launch: hipSetDevice failed");
    return IVX_EDEVICE;
  }
  const hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error("ivx_graph_launch: %s", hipGetErrorString(e));
    return IVX_EDEVICE;
  }
  return IVX_OK;
}

}  // extern "C"
