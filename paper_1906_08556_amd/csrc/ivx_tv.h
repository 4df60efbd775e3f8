// Launchers of the E-step / M-step kernels (k_tv.hip, k_mstep.hip).
#pragma once

#include "ivx_internal.h"

namespace ivx {

// ---- k_tv.hip
void launch_tv_prep(ivx_ctx* ctx, hipStream_t s);
void launch_add_identity(ivx_ctx* ctx, float* L, int64_t U, hipStream_t s);
void launch_reduce_b(ivx_ctx* ctx, const float* part, int nsplit, int64_t sstride, int64_t U,
                     float* b, hipStream_t s);
// Phi (packed upper, may be null: no covariance wanted) is written here
// whichever form runs.
void launch_estep_chol(ivx_ctx* ctx, int64_t U, float* Lb, float* Wb, const float* b, float* phi,
                       double* llu, int* info, float* Phi, hipStream_t s);
// k_estep_rr.hip: the same operation with the matrix held in registers
bool estep_rr_fits(int R);
bool estep_rr_setup();
void launch_estep_rr(ivx_ctx* ctx, int64_t U, const float* Lb, const float* b, float* phi,
                     double* llu, int* info, float* Phi_packed, hipStream_t s);
void launch_tp_to_packed(ivx_ctx* ctx, const float* Ptp, int64_t U, float* out, hipStream_t s);
void launch_packed_to_psi(ivx_ctx* ctx, const float* Phi, const float* phi, int64_t U, double* Psi,
                          hipStream_t s);
void launch_colsums(ivx_ctx* ctx, const float* n, const float* phi, const double* Psi, int64_t U,
                    const ivx_accum* acc, hipStream_t s);

// ---- k_mstep.hip
void launch_objective(ivx_ctx* ctx, const double* N, const double* S, const double* ll_sum,
                      double* objective, hipStream_t s);
void launch_mstep_solve(ivx_ctx* ctx, const ivx_accum* acc, const double* S, int update_sigma,
                        int* status, hipStream_t s);
// standard: M = L_G only (Sec. 3.1); update_mean (standard only): bias += T h/U first.
// IVX_EDEVICE (message set) when the copy of the updated T cannot be queued.
ivx_status launch_mindiv(ivx_ctx* ctx, const ivx_accum* acc, bool standard, bool update_mean,
                         hipStream_t s);

}  // namespace ivx
