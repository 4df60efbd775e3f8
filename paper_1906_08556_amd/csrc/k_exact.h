// FP64 exact component log-likelihood shared by the rescoring kernels.
#pragma once

#include "ivx_internal.h"

namespace ivx {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Exact FP64 log w_c N(x; mu_c, Sigma_c) = cst_c - 1/2 ||L_c^-1 (x - mu_c)||^2
// for the wave's frame; every lane returns the same value.  xd: lane's
// feature (0 for lanes >= D); dsh: 64 doubles of wave-private LDS.  linv
// holds L_c^-1 packed by columns (column j: rows j..D-1), D(D+1)/2 per c.
__device__ inline double exact_ll(int c, double xd, int lane, int D, int Dp,
                                  const double* __restrict__ mu, const double* __restrict__ linv,
                                  const double* __restrict__ cst, double* dsh) {
  const double d = (lane < D) ? (xd - mu[(size_t)c * D + lane]) : 0.0;
  dsh[lane] = d;
  __builtin_amdgcn_wave_barrier();
  const double* Lc = linv + (size_t)c * Dp;
  double y = 0.0;
  int col = 0;
  for (int j = 0; j < D; ++j) {
    const double dj = dsh[j];
    if (lane >= j && lane < D) y += Lc[col + (lane - j)] * dj;
    col += D - j;
  }
  __builtin_amdgcn_wave_barrier();
  return cst[c] - 0.5 * wave_sum(y * y);
}

}  // namespace ivx
