// Zeroth- and first-order Baum-Welch statistics (Sec. 2) as fixed-point sums.
//
// Every term gamma_tc (lane 0) and gamma_tc (x_t - m_c)_d (lanes 1..D; m_c = 0
// in the augmented formulation) is formed in FP64, rounded to a multiple of
// 2^-32 and added to a 64-bit integer with a device atomic.  Integer addition
// is exact and associative, so the sums do not depend on the order in which
// frames arrive: n and f are bitwise deterministic however the frames are
// scheduled.  Each term is rounded by at most 2^-33; a sum over T frames is
// within T 2^-33 of the exact sum of the terms (3.5e-7 at T = 3000).  The
// integers hold sums of magnitude below 2^31 after scaling: an utterance's
// sum of |gamma (x - m)| must stay below 2.1e9 (two million frames at
// |x| <= 1000); a single term of magnitude 2^24 or more raises IVX_ENUMERIC.
#pragma once

#include "ivx_internal.h"

namespace ivx {

constexpr double kFix = 4294967296.0;           // 2^32
constexpr double kFixInv = 1.0 / 4294967296.0;  // 2^-32
constexpr double kFixMaxTerm = 16777216.0;      // 2^24

// Adds entry (component c, posterior gm) of a frame with features xv (lane
// l holds x_{l-1} for l = 1..D) to row (row0 + c) of acc [.][D+1]: column 0
// is n, columns 1..D are f.  mb: FP32 bias m [C][D] or null.
__device__ inline void nf_add_entry(unsigned long long* __restrict__ acc, int64_t row0, int D,
                                    int lane, float xv, const float* __restrict__ mb, int c,
                                    double gm, int* __restrict__ err) {
  if (lane > D) return;
  double term = gm;
  if (lane >= 1) {
    double xc = (double)xv;
    if (mb) xc -= (double)mb[(int64_t)c * D + lane - 1];
    term = gm * xc;
  }
  if (!(fabs(term) < kFixMaxTerm)) {
    raise_error(err, IVX_ENUMERIC, PK_STATS_NF, c);
    return;
  }
  const long long q = __double2ll_rn(term * kFix);
  atomicAdd(acc + (row0 + c) * (D + 1) + lane, (unsigned long long)q);
}

}  // namespace ivx
