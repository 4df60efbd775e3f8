// Per-utterance E-step core with the whole matrix held on chip (eqs. (3)-(4)).
//
// One workgroup of 8 waves per utterance.  The lower 16 x 16 tiles of the
// tile-packed precision matrix L(u) (R <= 400: at most 325 tiles, 333 KB in
// FP32; read, not modified) are distributed over the register files of the
// 8 waves: tile t
// (t = bi (bi + 1) / 2 + bj) lives in slot t / 8 of wave t % 8, as the
// accumulator fragment of v_mfma_f32_16x16x4_f32 (lane l holds rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16).  L(u) is read once and
// Phi(u) written once, straight into the packed upper triangle of the
// caller's output; every intermediate stays in registers, and block rows or
// columns that other waves need are exchanged through LDS:
//
//   1. blocked Cholesky L = G G^T, right-looking: the diagonal tile of the
//      next step is updated and factored (with its 16 x 16 inverse) by its
//      owner while the other waves apply the current trailing update;
//      panel tiles are G_ik = C_ik G_kk^{-T}, products on MFMA;
//   2. W = G^{-1}, right-looking over block columns of G:
//      W_kj = G_kk^{-1} B_kj, then B_ij -= G_ik W_kj for i > k;
//   3. Phi = W^T W, one block row of W at a time: Phi_ij += W_ki^T W_kj;
//   4. phi = Phi b (per-tile partial products summed in a fixed order),
//      log|L(u)| from the diagonal of G, the utterance's objective share,
//      and Phi (when wanted) in the packed upper layout.
//
// The tile layout in registers changes between phases: in phase 1 a slot
// holds the fragment of the transposed tile (which lets the panel product
// take it directly as the MFMA B operand), in phase 2 the tile itself, in
// phase 3 the transposed tile again (which gives a float4 store of Phi).
#include <cmath>

#include "ivx_internal.h"
#include "ivx_tv.h"

namespace ivx {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int RR_NW = 8;      // waves per workgroup
constexpr int RR_NT = 41;     // slots per wave: 8 * 41 >= 325 tiles (nb <= 25)
constexpr int RR_MAXNB = 25;  // tiles per side (R <= 400)
constexpr int RR_NPK = (RR_NT + 2) / 3;  // scalar registers of the slot table
constexpr int RR_TILE = 256;
// dynamic LDS, in floats
constexpr int RR_OFF_DINV = 0;                                // [25][256] G_kk^{-1}
constexpr int RR_OFF_BUF = RR_OFF_DINV + RR_MAXNB * RR_TILE;  // [2][25][256] exchange
constexpr int RR_OFF_SCR = RR_OFF_BUF + 2 * RR_MAXNB * RR_TILE;  // [8][16][17] staging
constexpr int RR_OFF_B = RR_OFF_SCR + RR_NW * 272;               // [400] b(u)
constexpr int RR_OFF_RED = RR_OFF_B + RR_MAXNB * 16;             // doubles [64]
constexpr int RR_NRED = 64;
constexpr int RR_OFF_COLM = RR_OFF_RED + 2 * RR_NRED;  // uint64 [8 waves][32] column masks
constexpr size_t RR_LDS_BYTES = (size_t)RR_OFF_COLM * 4 + RR_NW * 32 * sizeof(uint64_t);
constexpr int RR_NG = (RR_NT + 7) / 8;  // groups of eight slots

__device__ inline int64_t tile_off(int bi, int bj) { return (int64_t)(bi * (bi + 1) / 2 + bj) * 256; }

// Position of element (row, col) of a 16 x 16 tile in LDS: row-major with the
// four-column groups of a row permuted by the row, so that the float4 reads
// of "row l % 16, columns 4 (l / 16) .. +3" by a wave spread over the banks.
__device__ __forceinline__ int swz(int row, int col) {
  return row * 16 + ((((col >> 2) ^ (row >> 1)) & 3) << 2) + (col & 3);
}

__device__ __forceinline__ float rl(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ floatx4 ld4(const float* p) { return *reinterpret_cast<const floatx4*>(p); }
__device__ __forceinline__ void st4(float* p, floatx4 v) { *reinterpret_cast<floatx4*>(p) = v; }

__device__ __forceinline__ floatx4 mfma4(floatx4 a, floatx4 b, floatx4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
  return c;
}

// value of lane J of the lane's own 16-lane row (DPP row_newbcast:J)
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xf, 0xf, false));
}
// value of lane src4 / 4
__device__ __forceinline__ float lane_perm(int src4, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(v)));
}

// Factors one symmetric 16 x 16 tile held in scr (16 x 17, row-major, lower
// part used) in the registers of one wave: C = G G^T, writes G^{-1} to dk
// (swizzled row-major), stores sum log G_ii in *ld and returns the first
// non-positive pivot (1-based), 0 if none.  Lane (c, q) = (lane % 16,
// lane / 16) holds rows 4 r + q (r < 4) of column c of the symmetric
// trailing matrix and of X, the right-hand side of G W = I reduced
// alongside.  Step j takes the pivot with a lane read, the column-j entries
// of the lane's own rows with a broadcast inside each 16-lane row, and row j
// (of the trailing matrix and of X) with a permute from the row group that
// holds it; row j of G^{-1} is then final and stored.  Rows above the step
// hold values that are never read again.
__device__ __forceinline__ int rr_factor_diag(const float* scr, float* dk, double* ld) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));  // lane-dependent selects stay inside the call
  const int c = lane & 15, q = lane >> 4;
  float a[4], x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * r + q;
    a[r] = scr[c <= i ? i * 17 + c : c * 17 + i];
    x[r] = i == c ? 1.0f : 0.0f;
  }
  int bad = 0;
  double prod = 1.0;  // product of the pivots G_jj^2 (each in FP32 range: no overflow)
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    float piv = rl(a[j >> 2], 16 * (j & 3) + j);
    if (!(piv > 0.0f) || !isfinite(piv)) {
      if (bad == 0) bad = j + 1;
      piv = 1.0f;
    }
    prod *= (double)piv;
    const float ri = __builtin_amdgcn_rsqf(piv);  // 1 / G_jj
    const float ri2 = ri * ri;
    const int src4 = (16 * (j & 3) + c) * 4;
    const float ajc = lane_perm(src4, a[j >> 2]);
    const float xjc = lane_perm(src4, x[j >> 2]);
    if (q == (j & 3)) dk[swz(j, c)] = x[j >> 2] * ri;
    const float t = c > j ? ajc * ri2 : 0.0f;
    const float u = xjc * ri2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float d;
      switch (j) {  // the DPP control is an immediate
        case 0: d = row_bcast<0>(a[r]); break;
        case 1: d = row_bcast<1>(a[r]); break;
        case 2: d = row_bcast<2>(a[r]); break;
        case 3: d = row_bcast<3>(a[r]); break;
        case 4: d = row_bcast<4>(a[r]); break;
        case 5: d = row_bcast<5>(a[r]); break;
        case 6: d = row_bcast<6>(a[r]); break;
        case 7: d = row_bcast<7>(a[r]); break;
        case 8: d = row_bcast<8>(a[r]); break;
        case 9: d = row_bcast<9>(a[r]); break;
        case 10: d = row_bcast<10>(a[r]); break;
        case 11: d = row_bcast<11>(a[r]); break;
        case 12: d = row_bcast<12>(a[r]); break;
        case 13: d = row_bcast<13>(a[r]); break;
        case 14: d = row_bcast<14>(a[r]); break;
        default: d = row_bcast<15>(a[r]); break;
      }
      a[r] = fmaf(-d, t, a[r]);
      x[r] = fmaf(-d, u, x[r]);
    }
  }
  *ld = 0.5 * log(prod);  // sum log G_jj
  return bad;
}

// Keeps the slot table in scalar registers and opaque to the optimiser, so
// that the per-slot decodes stay next to their use instead of being hoisted
// out of the step loops (82 live scalars would not fit).
#define RR_LAUNDER(pk)                                                        \
  do {                                                                        \
    _Pragma("unroll") for (int n_ = 0; n_ < RR_NPK; ++n_) asm volatile("" : "+s"(pk[n_])); \
  } while (0)
#define RR_TI(pk, s) ((int)((pk[(s) / 3] >> (10 * ((s) % 3) + 5)) & 31u))
#define RR_TJ(pk, s) ((int)((pk[(s) / 3] >> (10 * ((s) % 3))) & 31u))

// Runs the statement block for every slot s whose bit is set in the 64-bit mask M (a
// scalar), with ti, tj its block row and column; groups of eight slots
// without a set bit are skipped with one test.
#define RR_FOR_MASK(M, ...)                                                   \
  do {                                                                        \
    const uint64_t m_ = (M);                                                  \
    RR_LAUNDER(pk);                                                           \
    _Pragma("unroll") for (int g_ = 0; g_ < RR_NG; ++g_) {                    \
      if ((uint32_t)(m_ >> (8 * g_)) & 0xffu) {                               \
        _Pragma("unroll") for (int s = 8 * g_; s < 8 * g_ + 8; ++s) {         \
          if (s < RR_NT && ((m_ >> s) & 1ull)) {                              \
            const int ti = RR_TI(pk, s), tj = RR_TJ(pk, s);                   \
            (void)ti;                                                         \
            (void)tj;                                                         \
            __VA_ARGS__                                                       \
          }                                                                   \
        }                                                                     \
      }                                                                       \
    }                                                                         \
  } while (0)

__device__ __forceinline__ uint64_t lowbits(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// first slot s of wave w whose tile index w + 8 s is >= T
__device__ __forceinline__ int first_slot(int w, int T) {
  const int d = T - w;
  return d <= 0 ? 0 : (d + RR_NW - 1) / RR_NW;
}

__global__ void __launch_bounds__(RR_NW * 64)
k_estep_rr(int R, int nb, int64_t TP, const float* __restrict__ Lb, const float* __restrict__ bvec,
           const double* __restrict__ p, float* __restrict__ phi, double* __restrict__ llu,
           int* __restrict__ info, float* __restrict__ Phi_out, int* __restrict__ err) {
  extern __shared__ float sm[];
  float* dinv = sm + RR_OFF_DINV;
  float* buf = sm + RR_OFF_BUF;
  float* bv = sm + RR_OFF_B;
  double* red = reinterpret_cast<double*>(sm + RR_OFF_RED);
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, q16 = lane >> 4;
  float* scr = sm + RR_OFF_SCR + wave * 272;
  const int64_t u = blockIdx.x;
  const float* L = Lb + u * TP;
  // fragment offsets: "row l16, columns 4 q16 .. 4 q16 + 3" of a swizzled tile
  const int frag = swz(l16, 4 * q16);

  // (block row, block column) of every slot, 10 bits each (bi << 5 | bj),
  // three slots per scalar register; slots past the last tile get bi = 31
  uint32_t pk[RR_NPK];
#pragma unroll
  for (int n = 0; n < RR_NPK; ++n) {
    uint32_t w = 0u;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int t = wave + RR_NW * (3 * n + m);
      int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      i += ((i + 1) * (i + 2) / 2 <= t) ? 1 : 0;
      i -= (i * (i + 1) / 2 > t) ? 1 : 0;
      const int j = t - i * (i + 1) / 2;
      w |= (uint32_t)((i < nb ? i : 31) << 5 | (j & 31)) << (10 * m);
    }
    pk[n] = __builtin_amdgcn_readfirstlane(w);
  }

  // ---- load: slot = fragment of the transposed tile, L_ij[l16][4 q16 + r]
  floatx4 tl[RR_NT];
#pragma unroll
  for (int s = 0; s < RR_NT; ++s) {
    const int ti = RR_TI(pk, s), tj = RR_TJ(pk, s);
    if (ti < nb)
      tl[s] = ld4(L + tile_off(ti, tj) + l16 * 16 + 4 * q16);
    else
      tl[s] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  for (int i = tid; i < nb * 16; i += RR_NW * 64) bv[i] = (i < R) ? bvec[u * R + i] : 0.0f;
  // slot masks: colm[wave][j] = slots of block column j (lane j builds it)
  uint64_t* colm = reinterpret_cast<uint64_t*>(sm + RR_OFF_COLM) + wave * 32;
  if (lane < 32) {
    uint64_t m = 0;
#pragma unroll
    for (int s = 0; s < RR_NT; ++s) {
      const int ti = RR_TI(pk, s), tj = RR_TJ(pk, s);
      if (ti < nb && tj == lane) m |= 1ull << s;
    }
    colm[lane] = m;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  auto col_mask = [&](int j) -> uint64_t {
    const uint64_t v = colm[j];
    // readfirstlane returns a signed int: widen through uint32_t
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
  };
  // slots with block row < i: the first first_slot(wave, i (i + 1) / 2)
  auto rows_below = [&](int i) -> uint64_t { return lowbits(first_slot(wave, i * (i + 1) / 2)); };
  const uint64_t valid = rows_below(nb);

  // ================================================= 1. Cholesky L = G G^T
  // Step k: panel k (G_ik = C_ik G_kk^{-T}), then the diagonal tile k + 1 is
  // updated by its owner, staged in LDS and factored, and the other trailing
  // tiles take the update of panel k.
  float* pan = buf;                       // G_ik, i > k, row-major (tile i - k - 1)
  float* npan = buf + RR_MAXNB * RR_TILE;  // -G_ik
  if (wave == 0) {  // tile (0, 0): slot 0 of wave 0
#pragma unroll
    for (int r = 0; r < 4; ++r) scr[(4 * q16 + r) * 17 + l16] = tl[0][r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    double ld;
    const int b = rr_factor_diag(scr, dinv, &ld);
    if (lane == 0) {
      red[0] = ld;
      if (b) s_bad = b;
    }
  }
  uint64_t done = 0;  // slots of block columns <= k
  for (int k = 0; k < nb; ++k) {
    __syncthreads();  // G_kk^{-1} in dinv[k]; column k up to date
    if (s_bad) break;
    const uint64_t ck = col_mask(k);
    const uint64_t below = ck & ~rows_below(k + 1);  // column k, rows > k
    done |= ck;
    // panel: G_ik^T = G_kk^{-1} C_ik^T (C_ik^T is the slot's fragment)
    const floatx4 gk = ld4(dinv + k * RR_TILE + frag);
    RR_FOR_MASK(below, {
      const floatx4 y = mfma4(gk, tl[s], floatx4{0.0f, 0.0f, 0.0f, 0.0f});
      // y[r] = G_ik[l16][4 q16 + r]
      st4(pan + (ti - k - 1) * RR_TILE + frag, y);
      st4(npan + (ti - k - 1) * RR_TILE + frag, -y);
    });
    __syncthreads();  // panel complete
    // the panel tiles stay in their slots as the fragment of G_ik itself
    RR_FOR_MASK(below, {
      const float* pt = pan + (ti - k - 1) * RR_TILE;
_Pragma("unroll")
      for (int r = 0; r < 4; ++r) tl[s][r] = pt[swz(4 * q16 + r, l16)];
    });
    if (k + 1 < nb) {
      // the next diagonal tile first (its owner only): update and stage it
      const int td = (k + 1) * (k + 2) / 2 + (k + 1);
      const bool own = (td & (RR_NW - 1)) == wave;
      const uint64_t dmask = own ? (1ull << (td >> 3)) : 0ull;
      if (own) {
        const floatx4 a = ld4(npan + frag), b = ld4(pan + frag);
        RR_FOR_MASK(dmask, {
          tl[s] = mfma4(a, b, tl[s]);
_Pragma("unroll")
          for (int r = 0; r < 4; ++r) scr[(4 * q16 + r) * 17 + l16] = tl[s][r];
        });
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        double ld;
        const int bd = rr_factor_diag(scr, dinv + (k + 1) * RR_TILE, &ld);
        if (lane == 0) {
          red[k + 1] = ld;
          if (bd) s_bad = (k + 1) * 16 + bd;
        }
      }
      // trailing tiles (i, j), k < j <= i, except the diagonal one done above:
      // C_ij^T -= G_jk G_ik^T
      RR_FOR_MASK(valid & ~done & ~dmask, {
        tl[s] = mfma4(ld4(npan + (tj - k - 1) * RR_TILE + frag),
                      ld4(pan + (ti - k - 1) * RR_TILE + frag), tl[s]);
      });
    }
  }
  const int bad = s_bad;
  if (bad) {
    if (tid == 0) {
      if (info) info[u] = bad;
      raise_error(err, IVX_ENOTPD, PK_ESTEP_CHOL, (int)u);
      llu[u] = 0.0;
    }
    for (int i = tid; i < R; i += RR_NW * 64) phi[u * R + i] = NAN;
    return;
  }
  if (info && tid == 0) info[u] = 0;

  // ================================================= 2. W = G^{-1}
  // slots: off-diagonal G_ij (then B_ij, then W_ij); diagonal G_kk^{-1} = W_kk
  float* rowb = buf;                       // W_kj^T row-major (tile j)
  float* ncol = buf + RR_MAXNB * RR_TILE;  // -G_ik row-major (tile i - k - 1)
  {
    uint64_t dm = 0;  // diagonal slots: the last tile of each block row
    for (int i = 0; i < nb; ++i) {
      const int t = i * (i + 1) / 2 + i;
      if ((t & (RR_NW - 1)) == wave) dm |= 1ull << (t >> 3);
    }
    RR_FOR_MASK(dm, {
      const float* dk = dinv + ti * RR_TILE;
_Pragma("unroll")
      for (int r = 0; r < 4; ++r) tl[s][r] = dk[swz(4 * q16 + r, l16)];
    });
  }
  done = 0;
  for (int k = 0; k < nb; ++k) {
    const uint64_t ck = col_mask(k);
    const uint64_t lo = rows_below(k), hi = rows_below(k + 1);
    const uint64_t below = ck & ~hi;  // column k, rows > k
    done |= ck;
    const floatx4 gk = ld4(dinv + k * RR_TILE + frag);
    // block row k: W_kj = G_kk^{-1} B_kj (j < k), W_kk = G_kk^{-1}; to LDS as W_kj^T
    RR_FOR_MASK(hi & ~lo, {
      if (tj < k) tl[s] = mfma4(gk, tl[s], floatx4{0.0f, 0.0f, 0.0f, 0.0f});
      st4(rowb + tj * RR_TILE + frag, tl[s]);  // fragment of W_kj = W_kj^T[l16][4 q16 + r]
    });
    // column k of G below the diagonal, negated, to LDS
    RR_FOR_MASK(below, {
      float* ct = ncol + (ti - k - 1) * RR_TILE;
_Pragma("unroll")
      for (int r = 0; r < 4; ++r) ct[swz(4 * q16 + r, l16)] = -tl[s][r];
    });
    __syncthreads();
    // B_ij -= G_ik W_kj for i > k, j <= k (B_ik starts at zero)
    RR_FOR_MASK(done & ~hi, {
      const floatx4 c0 = (tj == k) ? floatx4{0.0f, 0.0f, 0.0f, 0.0f} : tl[s];
      tl[s] = mfma4(ld4(ncol + (ti - k - 1) * RR_TILE + frag), ld4(rowb + tj * RR_TILE + frag), c0);
    });
    __syncthreads();
  }

  // ================================================= 3. Phi = W^T W
  for (int k = 0; k < nb; ++k) {
    float* rb = buf + (k & 1) * RR_MAXNB * RR_TILE;  // W_kj^T row-major (tile j)
    const uint64_t lo = rows_below(k), hi = rows_below(k + 1);
    RR_FOR_MASK(hi & ~lo, {
      st4(rb + tj * RR_TILE + frag, tl[s]);
      tl[s] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    });
    __syncthreads();
    // Phi_ij^T += W_kj^T W_ki for j <= i <= k
    RR_FOR_MASK(hi, {
      tl[s] = mfma4(ld4(rb + tj * RR_TILE + frag), ld4(rb + ti * RR_TILE + frag), tl[s]);
    });
  }
  __syncthreads();

  // ================================================= 4. phi, objective, Phi
  // slot fragment: Phi_ij[l16][4 q16 + r].  Tile t contributes Phi_ij b_j to
  // block i (part[t][0..15]) and, off the diagonal, Phi_ij^T b_i to block j
  // (part[t][16..31]).
  float* part = buf;
  RR_LAUNDER(pk);
#pragma unroll
  for (int s = 0; s < RR_NT; ++s) {
    const int ti = RR_TI(pk, s), tj = RR_TJ(pk, s);
    if (ti < nb) {
      const int t = wave + RR_NW * s;
      const floatx4 v = tl[s];
      float pr = v[0] * bv[16 * tj + 4 * q16] + v[1] * bv[16 * tj + 4 * q16 + 1] +
                 v[2] * bv[16 * tj + 4 * q16 + 2] + v[3] * bv[16 * tj + 4 * q16 + 3];
      pr += __shfl_xor(pr, 16);
      pr += __shfl_xor(pr, 32);
      if (q16 == 0) part[t * 32 + l16] = pr;
      if (ti != tj) {
        const float bi = bv[16 * ti + l16];
        float c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          c[r] = v[r] * bi;
          c[r] += __shfl_xor(c[r], 1);
          c[r] += __shfl_xor(c[r], 2);
          c[r] += __shfl_xor(c[r], 4);
          c[r] += __shfl_xor(c[r], 8);
        }
        if (l16 == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) part[t * 32 + 16 + 4 * q16 + r] = c[r];
        }
      }
      if (Phi_out) {
        // element (a, c) of the lower tile is (c, a) of the packed upper
        // triangle, row c at c R - c (c - 1) / 2; lanes along a write
        // consecutive words of one packed row
        const int a = 16 * ti + l16;
        float* out = Phi_out + u * ((int64_t)R * (R + 1) / 2);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 16 * tj + 4 * q16 + r;
          if (a < R && c <= a) out[(int64_t)c * R - (int64_t)c * (c - 1) / 2 + (a - c)] = v[r];
        }
      }
    }
  }
  __syncthreads();
  double bp = 0.0, pp = 0.0;
  for (int i = tid; i < R; i += RR_NW * 64) {
    const int bi = i >> 4, e = i & 15;
    float s = 0.0f;
    for (int j = 0; j <= bi; ++j) s += part[(bi * (bi + 1) / 2 + j) * 32 + e];
    for (int i2 = bi + 1; i2 < nb; ++i2) s += part[(i2 * (i2 + 1) / 2 + bi) * 32 + 16 + e];
    phi[u * R + i] = s;
    bp += (double)bv[i] * (double)s;
    pp += p[i] * p[i];
  }
  double v = bp - pp;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) red[32 + wave] = v;
  __syncthreads();
  if (tid == 0) {
    double ls = 0.0;
    for (int kk = 0; kk < nb; ++kk) ls += red[kk];
    double q = 0.0;
    for (int w = 0; w < RR_NW; ++w) q += red[32 + w];
    llu[u] = -0.5 * (2.0 * ls) + 0.5 * q;
  }
}

}  // namespace

bool estep_rr_fits(int R) { return R >= 1 && (R + 15) / 16 <= RR_MAXNB; }

bool estep_rr_setup() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_estep_rr),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)RR_LDS_BYTES) == hipSuccess;
}

void launch_estep_rr(ivx_ctx* ctx, int64_t U, const float* Lb, const float* b, float* phi,
                     double* llu, int* info, float* Phi_packed, hipStream_t s) {
  if (U <= 0) return;
  const int nb = (ctx->R + 15) / 16;
  k_estep_rr<<<(unsigned)U, RR_NW * 64, RR_LDS_BYTES, s>>>(ctx->R, nb, ctx->TP, Lb, b, ctx->p, phi,
                                                          llu, info, Phi_packed, ctx->dev_err);
}

}  // namespace ivx
