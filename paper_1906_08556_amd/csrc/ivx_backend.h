// Launchers of the scoring back-end kernels (k_backend.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ivx {

constexpr int kBackendMaxDim = 512;

void be_zero(double* p, int64_t n, hipStream_t s);
// sums [K][dim] += rows of X by class, counts [K] += 1; labels NULL: one class
void be_class_sums(const float* X, int64_t n, int dim, const int* labels, int K, double* sums,
                   double* counts, int* bad, hipStream_t s);
void be_scatter(const double* M2, const double* sums, const double* counts, int K, int dim,
                double* Sw, double* Sb, double* mean, hipStream_t s);
// Eigendecomposition of the symmetric A [n][n] (n even; overwritten) into
// w [n] and the columns of V [n][n]; synchronises s once per sweep.  rot
// [n/2], part [128] workspace.  Returns the sweeps taken, -2 if max_sweeps
// did not reach the tolerance, -1 on a HIP error.
int be_jacobi(double* A, double* V, int n, int max_sweeps, double tol, double* w, double2* rot,
              double* part, hipStream_t s);
void be_dgemm(const void* A, bool a_float, int64_t lda, bool ta, const double* B, int64_t ldb,
              bool tb, void* C, int64_t ldc, bool c_float, int M, int N, int K,
              const double* colsub, hipStream_t s);
void be_whiten_cols(const double* Q, int ld, const double* lam, int dim, double floor_rel,
                    bool trans, double* Wh, int* bad, hipStream_t s);
void be_pad_sym(const double* src, int dim, double* dst, int n, hipStream_t s);
void be_rank_desc(const double* w, int valid, int keep, int* idx, hipStream_t s);
void be_gather_cols(const double* src, int ld, const int* idx, int rows, int keep,
                    const double* w, double* out, double* vals, hipStream_t s);
void be_lnorm(const float* X, int64_t n, int dim, const double* mean, const double* W, float* Y,
              hipStream_t s);
void be_plda_coef(const double* psi, int d, double* coef, hipStream_t s);
void be_plda_score(const float* Z1, int64_t n1, const float* Z2, int64_t n2, int d,
                   const double* coef, const int* trials, int64_t T, float* scores, int* bad,
                   hipStream_t s);

}  // namespace ivx
