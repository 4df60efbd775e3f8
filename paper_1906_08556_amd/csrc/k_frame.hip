// Frame posteriors against the full-covariance UBM over all C components.
//
// Stage 1 (k_frame_tile): the log-likelihood of every (frame, component)
// pair is one dot product of the expanded feature vector vech(x~ x~^T),
// x~ = [1, x - s], with the component's coefficient row (see k_ubm.hip).  The
// product runs on MFMA (v_mfma_f32_32x32x2_f32) with components on the M side
// and frames on the N side, so each lane ends a component tile holding 128
// log-likelihoods of one frame.  One persistent launch: each workgroup takes
// 128-frame tiles in turn and sweeps all C components over each, keeping the
// frames' running maximum, candidate count and overflow flag in registers
// and adding the components within the candidate margin to the frame's list
// as they appear; the [F x C] log-likelihood matrix never leaves registers
// and each frame is read once.
//
// Stage 2 (k_exact_sorted, k_rescore): every surviving candidate is rescored
// exactly in FP64 (candidates bucketed by component first, so that each
// L_c^-1 is read once per run of its candidates),
// l = const_c - 1/2 || L_c^{-1} (x - mu_c) ||^2, and the posteriors follow
// from a log-sum-exp over the candidates.  Frames whose candidate list
// overflowed are rescored over all C components and keep the KP best.
#include <algorithm>
#include <cmath>

#include "ivx_internal.h"
#include "k_exact.h"
#include "k_nf.h"

namespace ivx {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int FR = 32;        // frames per wave (one 32-frame MFMA block)
constexpr int NW = 4;         // waves per workgroup
constexpr int FT = FR * NW;   // frames per workgroup
// NCB (template): 32-component MFMA blocks per tile, CT = 32 NCB components
// per launch; 4 or 8 (picked by the autotuner)
constexpr int CAPL = KP / 2;  // candidate slots per lane-half per frame
constexpr int WLD = 12;       // LDS row stride (floats) of a staged [CT][8] W chunk

// Drops the entries of a lane-half's candidate list (global, CAPL slots,
// filled from slot 0) that fell below the running threshold.
__device__ inline int compact_cands(int2* __restrict__ lst, float thr) {
  int w = 0;
  for (int s = 0; s < CAPL; ++s) {
    const int2 e = lst[s];
    if (e.x >= 0 && __int_as_float(e.y) >= thr) lst[w++] = e;
  }
  for (int s = w; s < CAPL; ++s) lst[s] = make_int2(-1, 0);
  return w;
}

// Candidate state of one lane-half of a frame, in registers for the whole
// sweep over the components: running maximum M, number of filled list slots,
// overflow flag.  The list itself (CAPL slots of the lane-half, filled from
// slot 0) is in global memory, written only when a candidate is added.
struct FrameState {
  int64_t g;
  bool valid;
  int2* lst;
  float M;
  int cnt;
  bool ov;
};

__device__ inline void frame_state_init(FrameState& st, int64_t g, int64_t F, int h,
                                        int2* __restrict__ cand) {
  st.g = g;
  st.valid = g < F;
  st.lst = cand + (st.valid ? g : 0) * KP + h * CAPL;
  st.M = -INFINITY;
  st.cnt = 0;
  st.ov = false;
  if (st.valid)
    for (int s = 0; s < CAPL; ++s) st.lst[s] = make_int2(-1, 0);
}

// Epilogue of one 32-frame block: lane holds frame l32 and rows
// 8*(r/4) + 4*h + r%4 of each 32-component block; its partner lane
// (lane ^ 32) holds the other rows.  Two unrolled passes with small bodies
// keep acc[] in registers: count this tile's hits, make room once, store.
template <int NCB>
__device__ inline void frame_epilogue(const floatx16 (&acc)[NCB], FrameState& st, int h, int c0,
                                      int C, float margin, bool last, float* __restrict__ cM,
                                      int* __restrict__ cflag) {
  float vmax = -INFINITY;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) vmax = fmaxf(vmax, acc[cb][r]);
  const float lmax = vmax;
  vmax = fmaxf(vmax, __shfl_xor(vmax, 32));
  st.M = fmaxf(st.M, vmax);
  const float thr = st.M - margin;
  if (st.valid && lmax >= thr) {
    int nh = 0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) nh += (acc[cb][r] >= thr) ? 1 : 0;
    if (st.cnt + nh > CAPL) st.cnt = compact_cands(st.lst, thr);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float v = acc[cb][r];
        const int comp = c0 + cb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (v >= thr && comp < C) {
          if (st.cnt < CAPL) {
            st.lst[st.cnt] = make_int2(comp, __float_as_int(v));
            ++st.cnt;
          } else {
            st.ov = true;
          }
        }
      }
  }
  if (!last) return;
  const int ovi = st.ov ? 1 : 0;
  const int ovp = __shfl_xor(ovi, 32);
  if (st.valid && h == 0) {
    cM[st.g] = st.M;
    cflag[st.g] = ovi | ovp;
  }
}

// Loads the workgroup's frames as x~ = [1, x - shift] rows of DS floats.
__device__ inline void load_frames(float* xs, int nfr, int DS, const float* __restrict__ X,
                                   int64_t f0, int64_t F, int D, const float* __restrict__ shift) {
  for (int i = threadIdx.x; i < nfr * DS; i += 256) {
    const int fr = i / DS, a = i - fr * DS;
    const int64_t g = f0 + fr;
    float v = (a == 0) ? 1.0f : 0.0f;
    if (a > 0 && g < F) v = X[g * D + (a - 1)] - shift[a - 1];
    xs[i] = v;
  }
}

// Persistent: workgroup b takes frame tiles b, b + G, b + 2G, ... (G the
// grid size, a few workgroups per CU), so the workgroups move through the
// frames together.  For each tile it sweeps the component tiles of CT =
// 32 NCB components in order; each wave handles FB blocks of 32 frames (FT FB
// frames per workgroup).  The workgroups of the grid start together and
// spend the same time per component tile, so at any moment they stream
// nearby slices of W, which stay in every XCD's L2.  Chunks of 8 expanded
// features are staged through LDS (double buffered) and shared by the 4
// waves, and each staged coefficient serves the FB frame blocks of a wave.
//
// W layout (k_ubm_prepare): chunk-major, coefficient (c, k) at
// ((k / 8) * Cpad + c) * 8 + k % 8, so a chunk of a component tile is contiguous.
template <int NCB, int FB>
__global__ void __launch_bounds__(256, FB == 1 ? 2 : 1)
k_frame_tile(const float* __restrict__ X, int64_t F, int D, const float* __restrict__ shift,
             const float* __restrict__ W, int C, int Cpad, int Kpad,
             const uint16_t* __restrict__ pairs, float margin, int2* __restrict__ cand,
             float* __restrict__ cM, int* __restrict__ cflag, const int* __restrict__ Fdev) {
  constexpr int CT = 32 * NCB;   // components per component tile
  constexpr int TPC = 256 / CT;  // threads per staged component
  constexpr int NV = 2 / TPC;    // float4 per thread and chunk
  constexpr int FTB = FT * FB;   // frames per workgroup tile
  extern __shared__ float smem[];
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  const int64_t ntile = (F + FTB - 1) / FTB;
  if ((int64_t)blockIdx.x >= ntile) return;  // whole workgroup, before any barrier
  const int DS = D + 1;
  float* Ws = smem;                                              // [2][CT][WLD]
  float* xs = smem + 2 * CT * WLD;                               // [FTB][DS]
  uint32_t* prs = reinterpret_cast<uint32_t*>(xs + FTB * DS);    // [Kpad/2] index pairs
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int nq = Kpad / 8;
  for (int i = tid; i < Kpad / 2; i += 256) prs[i] = reinterpret_cast<const uint32_t*>(pairs)[i];
  // W chunk loader: TPC threads stage the 8 coefficients of one component
  // (named registers, not an array: an array captured by the lambdas ends
  // up in scratch memory)
  const int lc = tid / TPC, part = tid % TPC;
  float4 r0, r1;
  auto gload = [&](int q, int c0) {
    const float4* p =
        reinterpret_cast<const float4*>(W + ((size_t)q * Cpad + c0 + lc) * 8 + part * 4 * NV);
    r0 = p[0];
    if constexpr (NV == 2) r1 = p[1];
  };
  auto sstore = [&](int buf) {
    float* d = Ws + (buf * CT + lc) * WLD + part * 4 * NV;
    *reinterpret_cast<float4*>(d) = r0;
    if constexpr (NV == 2) *reinterpret_cast<float4*>(d + 4) = r1;
  };
  const float* xw = xs + (wave * FB * FR + l32) * DS;

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t f0 = tile * FTB;
    __syncthreads();  // the previous tile's readers of xs and Ws are done
    load_frames(xs, FTB, DS, X, f0, F, D, shift);
    FrameState st[FB];
#pragma unroll
    for (int fb = 0; fb < FB; ++fb)
      frame_state_init(st[fb], f0 + (wave * FB + fb) * FR + l32, F, h, cand);
    for (int c0 = 0; c0 < Cpad; c0 += CT) {
      gload(0, c0);
      sstore(0);
      __syncthreads();
      floatx16 acc[FB][NCB];
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[fb][cb] = floatx16{0};
      for (int q = 0; q < nq; ++q) {
        const int cur = q & 1;
        if (q + 1 < nq) gload(q + 1, c0);
        const float* wb = Ws + (cur * CT + l32) * WLD + 4 * h;
        float4 wv[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) wv[cb] = *reinterpret_cast<const float4*>(wb + cb * 32 * WLD);
        const uint32_t pw0 = prs[4 * q + 2 * h], pw1 = prs[4 * q + 2 * h + 1];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint32_t pr = ((s < 2) ? pw0 : pw1) >> ((s & 1) * 16);
          const int a = pr & 0xff, b = (pr >> 8) & 0xff;
#pragma unroll
          for (int fb = 0; fb < FB; ++fb) {
            const float* xf = xw + fb * FR * DS;
            const float bv = xf[a] * xf[b];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
              const float av = (s == 0) ? wv[cb].x : (s == 1) ? wv[cb].y : (s == 2) ? wv[cb].z : wv[cb].w;
              acc[fb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[fb][cb], 0, 0, 0);
            }
          }
        }
        if (q + 1 < nq) sstore(cur ^ 1);
        __syncthreads();
      }
      const bool last = c0 + CT >= Cpad;
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
        frame_epilogue<NCB>(acc[fb], st[fb], h, c0, C, margin, last, cM, cflag);
    }
  }
}

// The same persistent FP32 kernel with the coefficient operand read by each
// lane straight from the caches into registers (two chunks double
// buffered) instead of being staged through LDS: the waves of a workgroup
// share only the frames, so the k loop has no barrier and every wave runs
// ahead on its own.  Each lane reads the float4 of its component row and
// k-half of every 32-component block (NCB float4 per chunk of 8 features;
// the four waves of a workgroup read the same 8 KB, mostly from L1).
template <int NCB>
__global__ void __launch_bounds__(256, 2)
k_frame_tile_direct(const float* __restrict__ X, int64_t F, int D,
                    const float* __restrict__ shift, const float* __restrict__ W, int C, int Cpad,
                    int Kpad, const uint16_t* __restrict__ pairs, float margin,
                    int2* __restrict__ cand, float* __restrict__ cM, int* __restrict__ cflag,
                    const int* __restrict__ Fdev) {
  constexpr int CT = 32 * NCB;  // components per component tile
  extern __shared__ float smem[];
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  const int64_t ntile = (F + FT - 1) / FT;
  if ((int64_t)blockIdx.x >= ntile) return;  // whole workgroup, before any barrier
  const int DS = D + 1;
  float* xs = smem;                                              // [FT][DS]
  uint32_t* prs = reinterpret_cast<uint32_t*>(xs + FT * DS);     // [Kpad/2] index pairs
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int nq = Kpad / 8;  // even: Kpad is a multiple of 16
  for (int i = tid; i < Kpad / 2; i += 256) prs[i] = reinterpret_cast<const uint32_t*>(pairs)[i];
  const float* xw = xs + (wave * FR + l32) * DS;

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t f0 = tile * FT;
    __syncthreads();  // the previous tile's readers of xs are done
    load_frames(xs, FT, DS, X, f0, F, D, shift);
    FrameState st;
    frame_state_init(st, f0 + wave * FR + l32, F, h, cand);
    __syncthreads();
    for (int c0 = 0; c0 < Cpad; c0 += CT) {
      // lane's coefficients: chunk q, component c0 + 32 cb + l32, features 4h..4h+3
      const float* wl = W + ((size_t)c0 + l32) * 8 + 4 * h;
      const size_t qs = (size_t)Cpad * 8;  // stride between chunks
      float4 wa[NCB], wb[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) wa[cb] = *reinterpret_cast<const float4*>(wl + cb * 256);
      floatx16 acc[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = floatx16{0};
      auto chunk = [&](int q, const float4 (&wv)[NCB]) {
        const uint32_t pw0 = prs[4 * q + 2 * h], pw1 = prs[4 * q + 2 * h + 1];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint32_t pr = ((s < 2) ? pw0 : pw1) >> ((s & 1) * 16);
          const float bv = xw[pr & 0xff] * xw[(pr >> 8) & 0xff];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            const float av = (s == 0) ? wv[cb].x : (s == 1) ? wv[cb].y : (s == 2) ? wv[cb].z : wv[cb].w;
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[cb], 0, 0, 0);
          }
        }
      };
      for (int q = 0; q < nq; q += 2) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          wb[cb] = *reinterpret_cast<const float4*>(wl + (q + 1) * qs + cb * 256);
        chunk(q, wa);
        if (q + 2 < nq) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            wa[cb] = *reinterpret_cast<const float4*>(wl + (q + 2) * qs + cb * 256);
        }
        chunk(q + 1, wb);
      }
      frame_epilogue<NCB>(acc, st, h, c0, C, margin, c0 + CT >= Cpad, cM, cflag);
    }
  }
}

// ---------------------------------------------------------------- BF16 form
// Same tiling as k_frame_tile, with the dot products on
// v_mfma_f32_32x32x16_bf16 and FP32 accumulation.  Both operands are split
// into BF16 high and low parts (v = hi + lo, lo = bf16(v - hi)) and three
// products hi*hi + hi*lo + lo*hi are accumulated: plain BF16 would be off by
// hundreds of nats on this range, the split form by a few nats.  The result
// only selects candidates; every kept component is rescored exactly in FP64.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int WB16 = 40;  // LDS row stride (bf16) of a staged comp: 16 hi, 16 lo, 8 pad

// W16 layout (k_ubm_prepare): [Kpad/16][Cpad][32] bf16, per component 16 hi
// then 16 lo coefficients of the chunk.  Persistent over frame tiles and
// component tiles as k_frame_tile.
template <int NCB, int FB>
__global__ void __launch_bounds__(256, FB == 1 ? 2 : 1)
k_frame_tile_bf16(const float* __restrict__ X, int64_t F, int D, const float* __restrict__ shift,
                  const __bf16* __restrict__ W16, int C, int Cpad, int Kpad,
                  const uint16_t* __restrict__ pairs, float margin, int2* __restrict__ cand,
                  float* __restrict__ cM, int* __restrict__ cflag, const int* __restrict__ Fdev) {
  constexpr int CT = 32 * NCB;   // components per component tile
  constexpr int TPC = 256 / CT;  // threads per staged component
  constexpr int NV = 4 / TPC;    // uint4 (8 bf16) per thread and chunk
  constexpr int FTB = FT * FB;   // frames per workgroup tile
  extern __shared__ float smem[];
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  const int64_t ntile = (F + FTB - 1) / FTB;
  if ((int64_t)blockIdx.x >= ntile) return;  // whole workgroup, before any barrier
  const int DS = D + 1;
  __bf16* Ws = reinterpret_cast<__bf16*>(smem);                  // [2][CT][WB16]
  float* xs = smem + (2 * CT * WB16) / 2;                         // [FTB][DS]
  uint32_t* prs = reinterpret_cast<uint32_t*>(xs + FTB * DS);     // [Kpad/2]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int nq = Kpad / 16;
  for (int i = tid; i < Kpad / 2; i += 256) prs[i] = reinterpret_cast<const uint32_t*>(pairs)[i];
  // chunk loader: TPC threads stage the 32 bf16 (64 B) of one component
  const int lc = tid / TPC, part = tid % TPC;
  uint4 r0, r1, r2, r3;  // named registers (see k_frame_tile)
  auto gload = [&](int q, int c0) {
    const uint4* p =
        reinterpret_cast<const uint4*>(W16 + ((size_t)q * Cpad + c0 + lc) * 32 + part * 8 * NV);
    r0 = p[0];
    r1 = p[1];
    if constexpr (NV == 4) {
      r2 = p[2];
      r3 = p[3];
    }
  };
  auto sstore = [&](int buf) {
    uint4* d = reinterpret_cast<uint4*>(Ws + (buf * CT + lc) * WB16 + part * 8 * NV);
    d[0] = r0;
    d[1] = r1;
    if constexpr (NV == 4) {
      d[2] = r2;
      d[3] = r3;
    }
  };
  const float* xw = xs + (wave * FB * FR + l32) * DS;

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t f0 = tile * FTB;
    __syncthreads();  // the previous tile's readers of xs and Ws are done
    load_frames(xs, FTB, DS, X, f0, F, D, shift);
    FrameState st[FB];
#pragma unroll
    for (int fb = 0; fb < FB; ++fb)
      frame_state_init(st[fb], f0 + (wave * FB + fb) * FR + l32, F, h, cand);
    for (int c0 = 0; c0 < Cpad; c0 += CT) {
      gload(0, c0);
      sstore(0);
      __syncthreads();
      floatx16 acc[FB][NCB];
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[fb][cb] = floatx16{0};
      for (int q = 0; q < nq; ++q) {
        const int cur = q & 1;
        if (q + 1 < nq) gload(q + 1, c0);
        // B operand: products for k = 16 q + 8 h + e, e = 0..7, split hi / lo
        const uint4 pw = *reinterpret_cast<const uint4*>(prs + 8 * q + 4 * h);
        bf16x8 bh[FB], bl[FB];
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) {
          const float* xf = xw + fb * FR * DS;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t w32 = (e < 2) ? pw.x : (e < 4) ? pw.y : (e < 6) ? pw.z : pw.w;
            const uint32_t pr = w32 >> ((e & 1) * 16);
            const float v = xf[pr & 0xff] * xf[(pr >> 8) & 0xff];
            const __bf16 hi = (__bf16)v;
            bh[fb][e] = hi;
            bl[fb][e] = (__bf16)(v - (float)hi);
          }
        }
        const __bf16* wb = Ws + (cur * CT + l32) * WB16 + 8 * h;
        bf16x8 wh[NCB], wl[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          wh[cb] = *reinterpret_cast<const bf16x8*>(wb + cb * 32 * WB16);
          wl[cb] = *reinterpret_cast<const bf16x8*>(wb + cb * 32 * WB16 + 16);
        }
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[fb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[cb], bh[fb], acc[fb][cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[fb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[cb], bl[fb], acc[fb][cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[fb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl[cb], bh[fb], acc[fb][cb], 0, 0, 0);
        }
        if (q + 1 < nq) sstore(cur ^ 1);
        __syncthreads();
      }
      const bool last = c0 + CT >= Cpad;
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
        frame_epilogue<NCB>(acc[fb], st[fb], h, c0, C, margin, last, cM, cflag);
    }
  }
}

// ---- exact FP64 scores of the kept candidates, sorted by component --------
// A candidate slot e = g * KP + s is kept when the frame's list did not
// overflow and its FP32 score lies within the margin of the frame's maximum
// (the test k_rescore applies).  Kept slots are bucketed by component
// (per-block histograms, the shared scan, a scatter); k_exact_sorted then
// walks the sorted slots so that a wave loads each L_c^-1 row once per run
// of slots of one component instead of once per slot.
constexpr int RHB = 8192;  // frames per histogram block

__device__ inline int resc_kept(int64_t e, int C, const int2* __restrict__ cand,
                                const float* __restrict__ cM, float margin,
                                const int* __restrict__ cflag) {
  const int64_t g = e / KP;
  if (cflag[g] != 0) return -1;
  const int2 v = cand[e];
  return (v.x >= 0 && v.x < C && __int_as_float(v.y) >= cM[g] - margin) ? v.x : -1;
}

__global__ void __launch_bounds__(256)
k_resc_hist(int64_t F, int C, const int2* __restrict__ cand, const float* __restrict__ cM,
            float margin, const int* __restrict__ cflag, const int* __restrict__ Fdev,
            int* __restrict__ hist) {
  extern __shared__ int hl[];
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  for (int c = threadIdx.x; c < C; c += 256) hl[c] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * RHB * KP;
  const int64_t e1 = min(F * KP, e0 + (int64_t)RHB * KP);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = resc_kept(e, C, cand, cM, margin, cflag);
    if (c >= 0) atomicAdd(&hl[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) hist[(size_t)blockIdx.x * C + c] = hl[c];
}

__global__ void __launch_bounds__(256)
k_resc_scatter(int64_t F, int C, const int2* __restrict__ cand, const float* __restrict__ cM,
               float margin, const int* __restrict__ cflag, const int* __restrict__ Fdev,
               const int* __restrict__ base, int2* __restrict__ ent) {
  extern __shared__ int cur[];
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  for (int c = threadIdx.x; c < C; c += 256) cur[c] = base[(size_t)blockIdx.x * C + c];
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * RHB * KP;
  const int64_t e1 = min(F * KP, e0 + (int64_t)RHB * KP);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int c = resc_kept(e, C, cand, cM, margin, cflag);
    if (c >= 0) ent[atomicAdd(&cur[c], 1)] = make_int2((int)e, c);
  }
}

constexpr int EXC = 64;  // sorted slots per wave chunk

// lscore[slot] = cst_c - 1/2 ||L_c^-1 (x_g - mu_c)||^2 (FP64) for the sorted
// slots ent[0, coff[C]) (slot = frame * kpf + index), with L_c^-1 read from
// its dense column-major copy
// ldense [C][64][64] (zero outside the lower triangle of the D x D block).
// Lane i holds row i of L_c^-1 and mu_c[i] for the
// current component; (x - mu)_j reaches all lanes as a broadcast LDS read.
// Waves take chunks of EXC slots in a grid-stride loop.
__global__ void __launch_bounds__(256)
k_exact_sorted(const int2* __restrict__ ent, const int* __restrict__ coff, int C, int kpf,
               const float* __restrict__ X, int D, const double* __restrict__ mu,
               const double* __restrict__ ldense, const double* __restrict__ cst,
               double* __restrict__ lscore) {
  __shared__ double dsh[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t total = coff[C];
  const int64_t nw = (int64_t)gridDim.x * 4;
  int cur = -1;
  double Lr[64];
  double mul = 0.0, cc = 0.0;
#pragma unroll
  for (int j = 0; j < 64; ++j) Lr[j] = 0.0;
  for (int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * EXC; e0 < total;
       e0 += nw * EXC) {
    const int64_t e1 = min(total, e0 + EXC);
    for (int64_t e = e0; e < e1; ++e) {
      const int2 v = ent[e];  // wave-uniform
      if (v.y != cur) {
        cur = v.y;
        const double* Lc = ldense + (size_t)cur * 4096 + lane;  // column j at Lc[64 j]
#pragma unroll
        for (int j = 0; j < 64; ++j) Lr[j] = (j < D) ? Lc[64 * j] : 0.0;
        mul = (lane < D) ? mu[(size_t)cur * D + lane] : 0.0;
        cc = cst[cur];
      }
      const int64_t g = v.x / kpf;
      __builtin_amdgcn_wave_barrier();  // previous slot's reads of dsh are done
      dsh[wv][lane] = (lane < D) ? (double)X[g * D + lane] - mul : 0.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double y = 0.0;
#pragma unroll
      for (int j = 0; j < 64; ++j) y += Lr[j] * dsh[wv][j];
      const double q = wave_sum(y * y);
      if (lane == 0) lscore[v.x] = cc - 0.5 * q;
    }
  }
}

__global__ void __launch_bounds__(256)
k_rescore(const float* __restrict__ X, int64_t F, int D, int C, const double* __restrict__ mu,
          const double* __restrict__ linv, const double* __restrict__ cst,
          const int2* __restrict__ cand, const float* __restrict__ cM, float margin,
          const int* __restrict__ cflag, const double* __restrict__ lscore,
          int* __restrict__ post_idx, float* __restrict__ post_val, double* __restrict__ frame_ll,
          int* __restrict__ err, const int* __restrict__ Fdev, const int* __restrict__ fmap,
          const int* __restrict__ umap, int64_t U, const float* __restrict__ mb,
          unsigned long long* __restrict__ nf_acc) {
  __shared__ double dsh[4][64];
  __shared__ double lsh[4][KP];
  __shared__ int ish[4][KP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = (int64_t)blockIdx.x * 4 + wave;
  if (Fdev && (int64_t)Fdev[0] < F) F = Fdev[0];
  if (g >= F) return;  // wave-uniform; no workgroup barriers below
  const int64_t go = fmap ? (int64_t)fmap[g] : g;  // output row
  const int Dp = D * (D + 1) / 2;
  // every input of the frame is requested at once: features, flag, running
  // maximum, candidate slots and their exact scores (k_exact_sorted; slots
  // that were not kept hold stale values and are never read back)
  const double xd = (lane < D) ? (double)X[g * D + lane] : 0.0;
  const int fl = cflag[g];
  const float mg = cM[g];
  int2 e = make_int2(-1, 0);
  double ls = 0.0;
  if (lane < KP) {
    e = cand[g * KP + lane];
    ls = lscore[g * KP + lane];
  }
  int m = 0;
  double full_lse = NAN;  // set when all components were scored
  if (fl == 0) {
    const float thr = mg - margin;
    const int ci = (e.x >= 0 && __int_as_float(e.y) >= thr) ? e.x : -1;
    const int ls_lo = __double2loint(ls), ls_hi = __double2hiint(ls);
    for (int s = 0; s < KP; ++s) {
      const int c = __builtin_amdgcn_readlane(ci, s);
      if (c < 0 || c >= C) continue;
      const double l = __hiloint2double(__builtin_amdgcn_readlane(ls_hi, s),
                                        __builtin_amdgcn_readlane(ls_lo, s));
      if (lane == 0) {
        lsh[wave][m] = l;
        ish[wave][m] = c;
      }
      ++m;
    }
  } else {
    // overflowed candidate list: exact scores over all components; keep the
    // KP best (sorted, lane 0) and the full log-sum-exp
    double run_m = -INFINITY, run_s = 0.0;
    int cnt = 0;
    for (int c = 0; c < C; ++c) {
      const double l = exact_ll(c, xd, lane, D, Dp, mu, linv, cst, dsh[wave]);
      if (l > run_m) {
        run_s = run_s * exp(run_m - l) + 1.0;
        run_m = l;
      } else {
        run_s += exp(l - run_m);
      }
      if (lane == 0 && (cnt < KP || l > lsh[wave][KP - 1])) {
        int pos = cnt < KP ? cnt : KP - 1;
        while (pos > 0 && lsh[wave][pos - 1] < l) {
          lsh[wave][pos] = lsh[wave][pos - 1];
          ish[wave][pos] = ish[wave][pos - 1];
          --pos;
        }
        lsh[wave][pos] = l;
        ish[wave][pos] = c;
      }
      if (cnt < KP) ++cnt;
    }
    __builtin_amdgcn_wave_barrier();
    m = cnt;
    full_lse = run_m + log(run_s);
  }
  __builtin_amdgcn_wave_barrier();
  double mx = -INFINITY;
  for (int s = 0; s < m; ++s) mx = fmax(mx, lsh[wave][s]);
  double se = 0.0;
  for (int s = 0; s < m; ++s) se += exp(lsh[wave][s] - mx);
  const double kept = mx + log(se);
  const double lse = isnan(full_lse) ? kept : full_lse;
  if (!isfinite(lse) && lane == 0) raise_error(err, IVX_ENUMERIC, PK_RESCORE, (int)go);
  if (!isnan(full_lse) && lane == 0 && 1.0 - exp(kept - full_lse) > kMaxDroppedMass)
    raise_error(err, IVX_ECAPACITY, PK_RESCORE, (int)go);
  int id = -1;
  float v = 0.0f;
  if (lane < KP) {
    if (lane < m) {
      id = ish[wave][lane];
      v = (float)exp(lsh[wave][lane] - lse);
    }
    if (post_idx) post_idx[go * KP + lane] = id;
    if (post_val) post_val[go * KP + lane] = v;
  }
  if (lane == 0 && frame_ll) frame_ll[go] = lse;
  // n/f of the frame's utterance from the FP32 posteriors just written (the
  // same values the list-based accumulation reads)
  if (nf_acc) {
    const int u = umap[go];
    if (u < 0 || u >= U) return;  // offsets rejected by k_frame_utt
    const float xv = (lane >= 1 && lane <= D) ? X[g * D + (lane - 1)] : 0.0f;
    for (int sl = 0; sl < m; ++sl)
      nf_add_entry(nf_acc, (int64_t)u * C, D, lane, xv, mb, __shfl(id, sl),
                   (double)__shfl(v, sl), err);
  }
}

__global__ void k_dense_gamma(int64_t F, int C, const int* __restrict__ post_idx,
                              const float* __restrict__ post_val, float* __restrict__ gamma) {
  const int64_t n = F * C;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    gamma[i] = 0.0f;
}

__global__ void k_scatter_gamma(int64_t F, int C, const int* __restrict__ post_idx,
                                const float* __restrict__ post_val, float* __restrict__ gamma) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= F * KP) return;
  const int c = post_idx[i];
  if (c >= 0) gamma[(i / KP) * C + c] = post_val[i];
}

template <int NCB, int FB>
size_t frame_lds_bf16(int D, int Kpad) {
  return sizeof(__bf16) * 2 * (32 * NCB) * WB16 + sizeof(float) * (size_t)FT * FB * (D + 1) +
         sizeof(uint16_t) * Kpad;
}
size_t frame_lds_direct(int D, int Kpad) {
  return sizeof(float) * (size_t)FT * (D + 1) + sizeof(uint16_t) * Kpad;
}
template <int NCB, int FB>
size_t frame_lds_f32(int D, int Kpad) {
  return sizeof(float) * (2 * (32 * NCB) * WLD + (size_t)FT * FB * (D + 1)) +
         sizeof(uint16_t) * Kpad;
}

template <int NCB, int FB>
void frame_launches(ivx_ctx* ctx, const float* X, int64_t F, int prec, hipStream_t s,
                    const int* Fdev) {
  // persistent grid: as many workgroups as fit on the device at once
  const int64_t ntile = (F + FT * FB - 1) / (FT * FB);
  const unsigned nblk =
      (unsigned)std::min<int64_t>(ntile, (int64_t)ctx->ncu * (FB == 1 ? 2 : 1));
  ProfScope ps(ctx, PK_FRAME_SELECT, s);
  if (prec == IVX_BF16) {
    const size_t lds = frame_lds_bf16<NCB, FB>(ctx->D, ctx->Kpad);
    k_frame_tile_bf16<NCB, FB><<<nblk, 256, lds, s>>>(
        X, F, ctx->D, ctx->shift, ctx->W16, ctx->C, ctx->Cpad, ctx->Kpad, ctx->pairs,
        ctx->margin_bf16, ctx->cand, ctx->cM, ctx->cflag, Fdev);
    return;
  }
  if (FB == 1 && ctx->tune.frame_direct) {
    // the 128-component direct kernel fits three workgroups per CU
    const unsigned nd =
        (unsigned)std::min<int64_t>(ntile, (int64_t)ctx->ncu * (NCB == 4 ? 3 : 2));
    k_frame_tile_direct<NCB><<<nd, 256, frame_lds_direct(ctx->D, ctx->Kpad), s>>>(
        X, F, ctx->D, ctx->shift, ctx->Wexp, ctx->C, ctx->Cpad, ctx->Kpad, ctx->pairs,
        ctx->margin, ctx->cand, ctx->cM, ctx->cflag, Fdev);
    return;
  }
  const size_t lds = frame_lds_f32<NCB, FB>(ctx->D, ctx->Kpad);
  k_frame_tile<NCB, FB><<<nblk, 256, lds, s>>>(X, F, ctx->D, ctx->shift, ctx->Wexp, ctx->C,
                                               ctx->Cpad, ctx->Kpad, ctx->pairs, ctx->margin,
                                               ctx->cand, ctx->cM, ctx->cflag, Fdev);
}

}  // namespace

// Kernels using more than 64 KB of LDS (gfx950 has 160 KB per CU); called
// once per context at creation, outside any stream capture.
bool frame_set_attributes(const ivx_ctx* ctx) {
  bool ok = true;
  auto set = [&](const void* fn, size_t bytes) {
    ok = ok && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
                   hipSuccess;
  };
  const int D = ctx->D, Kp = ctx->Kpad;
  set(reinterpret_cast<const void*>(&k_frame_tile_bf16<8, 1>), frame_lds_bf16<8, 1>(D, Kp));
  set(reinterpret_cast<const void*>(&k_frame_tile_bf16<4, 1>), frame_lds_bf16<4, 1>(D, Kp));
  set(reinterpret_cast<const void*>(&k_frame_tile_bf16<4, 2>), frame_lds_bf16<4, 2>(D, Kp));
  set(reinterpret_cast<const void*>(&k_frame_tile<8, 1>), frame_lds_f32<8, 1>(D, Kp));
  set(reinterpret_cast<const void*>(&k_frame_tile<4, 1>), frame_lds_f32<4, 1>(D, Kp));
  set(reinterpret_cast<const void*>(&k_frame_tile<4, 2>), frame_lds_f32<4, 2>(D, Kp));
  return ok;
}

void launch_frame_select(ivx_ctx* ctx, const float* X, int64_t F, int prec, hipStream_t s,
                         const int* Fdev) {
  if (F <= 0) return;
  // frame_ncb: 8 (256 components per launch, one 32-frame block per wave),
  // 4 (128 components), or 2 (128 components, two frame blocks per wave)
  const int ncb = (prec == IVX_BF16) ? ctx->tune.frame_ncb_bf16 : ctx->tune.frame_ncb;
  if (ncb == 4)
    frame_launches<4, 1>(ctx, X, F, prec, s, Fdev);
  else if (ncb == 2)
    frame_launches<4, 2>(ctx, X, F, prec, s, Fdev);
  else
    frame_launches<8, 1>(ctx, X, F, prec, s, Fdev);
}

void launch_rescore(ivx_ctx* ctx, const float* X, int64_t F, int prec, int* post_idx,
                    float* post_val, double* frame_ll, hipStream_t s, const int* Fdev,
                    const int* fmap, const NfTarget* nf) {
  if (F <= 0) return;
  const float margin = prec == IVX_BF16 ? ctx->margin_bf16 : ctx->margin;
  // exact scores of the kept candidates, by component
  const unsigned nb = (unsigned)((F + RHB - 1) / RHB);
  const size_t ldsc = sizeof(int) * ctx->C;
  k_resc_hist<<<nb, 256, ldsc, s>>>(F, ctx->C, ctx->cand, ctx->cM, margin, ctx->cflag, Fdev,
                                    ctx->hist);
  launch_hist_scan((int)nb, ctx->C, ctx->hist, ctx->coff, s);
  k_resc_scatter<<<nb, 256, ldsc, s>>>(F, ctx->C, ctx->cand, ctx->cM, margin, ctx->cflag, Fdev,
                                       ctx->hist, ctx->ent);
  launch_exact_sorted(ctx, ctx->ent, ctx->coff, KP, X, ctx->lscore, s);
  const unsigned nblk = (unsigned)((F + 3) / 4);
  k_rescore<<<nblk, 256, 0, s>>>(X, F, ctx->D, ctx->C, ctx->mu, ctx->linv, ctx->cst, ctx->cand,
                                 ctx->cM, margin, ctx->cflag, ctx->lscore, post_idx, post_val,
                                 frame_ll, ctx->dev_err, Fdev, fmap,
                                 nf ? nf->umap : nullptr, nf ? nf->U : 0,
                                 nf ? nf->mb : nullptr, nf ? nf->acc : nullptr);
}

void launch_exact_sorted(ivx_ctx* ctx, const int2* ent, const int* coff, int kpf, const float* X,
                         double* lscore, hipStream_t s) {
  k_exact_sorted<<<4096, 256, 0, s>>>(ent, coff, ctx->C, kpf, X, ctx->D, ctx->mu, ctx->ldense,
                                      ctx->cst, lscore);
}

void launch_dense_gamma(ivx_ctx* ctx, int64_t F, const int* post_idx, const float* post_val,
                        float* gamma, hipStream_t s) {
  if (F <= 0) return;
  k_dense_gamma<<<2048, 256, 0, s>>>(F, ctx->C, post_idx, post_val, gamma);
  const int64_t n = F * KP;
  k_scatter_gamma<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(F, ctx->C, post_idx, post_val, gamma);
}

}  // namespace ivx
