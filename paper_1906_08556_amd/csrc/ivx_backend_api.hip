// C ABI of the scoring back-end (Sec. 4.1): whitening, length normalisation,
// LDA, two-covariance PLDA and trial scoring on the GPU, and the EER of a set
// of scores on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ivx_backend.h"
#include "ivx_internal.h"
#include "k_gemm.h"

using namespace ivx;

struct ivx_backend {
  int device = 0;
  int max_dim = 0, max_classes = 0;
  int64_t max_n = 0;
  double* sums = nullptr;    // [max_classes][max_dim]
  double* counts = nullptr;  // [max_classes]
  double* M2 = nullptr;      // [max_dim^2]
  double* Sw = nullptr;      // [max_dim^2]
  double* Sb = nullptr;      // [max_dim^2]
  double* mean = nullptr;    // [max_dim]
  double* Aj = nullptr;      // [nev^2] Jacobi matrix (padded to even order)
  double* Vj = nullptr;      // [nev^2] Jacobi eigenvectors
  double* wj = nullptr;      // [nev] eigenvalues
  double* Wh = nullptr;      // [max_dim^2]
  double* T1 = nullptr;      // [max_dim^2]
  double* T2 = nullptr;      // [max_dim^2]
  double* coef = nullptr;    // [2 max_dim + 1]
  double* muA = nullptr;     // [max_dim]
  float* Z1 = nullptr;       // [max_n][max_dim]
  float* Z2 = nullptr;       // [max_n][max_dim]
  int* idx = nullptr;        // [max_dim]
  double2* rot = nullptr;    // [nev / 2] Jacobi rotations of one step
  double* part = nullptr;    // [128] Jacobi norm partials
  int sweeps = 0;            // sweeps of the last Jacobi run (-1: HIP error)
  int* flags = nullptr;      // [4]: bad labels, singular whitening, bad trials, unused
};

namespace {

#define BE_CHECK(cond, ...)   \
  do {                        \
    if (!(cond)) {            \
      set_error(__VA_ARGS__); \
      return IVX_EINVAL;      \
    }                         \
  } while (0)

#define BE_HIP(call)                                                   \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) {                                            \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));        \
      return IVX_EDEVICE;                                              \
    }                                                                  \
  } while (0)

constexpr int kSweeps = 30;
constexpr double kTol = 1e-13;  // off-diagonal Frobenius norm relative to ||A||_F
constexpr double kFloor = 1e-13;  // eigenvalue floor relative to the largest

int even(int n) { return n + (n & 1); }

void be_free(ivx_backend* b) {
  void* ptrs[] = {b->sums, b->counts, b->M2, b->Sw, b->Sb, b->mean, b->Aj, b->Vj, b->wj,
                  b->Wh, b->T1, b->T2, b->coef, b->muA, b->Z1, b->Z2, b->idx, b->flags,
                  b->rot, b->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);  // teardown
  delete b;
}

template <typename T>
bool alloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1)) == hipSuccess;
}

// Reads and clears the flags after synchronising `s`; also reports a Jacobi
// run that failed or did not converge since the last call.
ivx_status read_flags(ivx_backend* b, hipStream_t s, int out[4]) {
  BE_HIP(hipStreamSynchronize(s));
  BE_HIP(hipMemcpy(out, b->flags, sizeof(int) * 4, hipMemcpyDeviceToHost));
  BE_HIP(hipMemset(b->flags, 0, sizeof(int) * 4));
  const int sw = b->sweeps;
  b->sweeps = 0;
  if (sw == -1) {
    set_error("ivx_backend: HIP error in the Jacobi eigensolver");
    return IVX_EDEVICE;
  }
  if (sw == -2) {
    set_error("ivx_backend: Jacobi eigensolver did not converge in %d sweeps", kSweeps);
    return IVX_ENUMERIC;
  }
  return IVX_OK;
}

// Sw, Sb (divisor N) and the mean of X [n][dim] by class (labels NULL: one).
void scatter(ivx_backend* b, const float* X, int64_t n, int dim, const int* labels, int K,
             hipStream_t s) {
  be_zero(b->sums, (int64_t)K * dim, s);
  be_zero(b->counts, K, s);
  be_zero(b->M2, (int64_t)dim * dim, s);
  be_class_sums(X, n, dim, labels, K, b->sums, b->counts, b->flags + 0, s);
  gemm64_tn(X, dim, X, false, dim, b->M2, dim, dim, dim, (int)n, s);
  be_scatter(b->M2, b->sums, b->counts, K, dim, b->Sw, b->Sb, b->mean, s);
}

// Eigendecomposition of the symmetric part of S [dim][dim]: eigenvectors in
// the first dim columns of b->Vj (leading dimension even(dim)), values in b->wj.
void eig(ivx_backend* b, const double* S, int dim, hipStream_t s) {
  const int n = even(dim);
  be_pad_sym(S, dim, b->Aj, n, s);
  const int sw = be_jacobi(b->Aj, b->Vj, n, kSweeps, kTol, b->wj, b->rot, b->part, s);
  if (b->sweeps >= 0) b->sweeps = sw < 0 ? sw : std::max(b->sweeps, sw);
}

// Wh = Q Lambda^{-1/2} of S (S = Q Lambda Q^T), so that Wh^T S Wh = I.
void whitener(ivx_backend* b, const double* S, int dim, double* Wh, bool trans, hipStream_t s) {
  eig(b, S, dim, s);
  be_whiten_cols(b->Vj, even(dim), b->wj, dim, kFloor, trans, Wh, b->flags + 1, s);
}

// Generalised symmetric problem Sb v = lambda Sw v: Wh whitens Sw, the
// eigenvectors U of Wh^T Sb Wh give V = Wh U (V^T Sw V = I).  Leaves Wh in
// b->Wh and U in b->Vj, the eigenvalues in b->wj.
void gen_eig(ivx_backend* b, int dim, hipStream_t s) {
  whitener(b, b->Sw, dim, b->Wh, false, s);
  be_dgemm(b->Sb, false, dim, false, b->Wh, dim, false, b->T1, dim, false, dim, dim, dim, nullptr,
           s);                                                   // T1 = Sb Wh
  be_dgemm(b->Wh, false, dim, true, b->T1, dim, false, b->T2, dim, false, dim, dim, dim, nullptr,
           s);                                                   // T2 = Wh^T T1
  eig(b, b->T2, dim, s);
}

}  // namespace

extern "C" {

ivx_status ivx_backend_create(int32_t max_dim, int64_t max_n, int32_t max_classes, int device,
                              ivx_backend** out) {
  BE_CHECK(out, "ivx_backend_create: null argument");
  *out = nullptr;
  BE_CHECK(max_dim >= 2 && max_dim <= kBackendMaxDim,
           "ivx_backend_create: max_dim=%d outside [2, %d]", max_dim, kBackendMaxDim);
  BE_CHECK(max_n >= 1 && max_n <= ((int64_t)1 << 31) - 1,
           "ivx_backend_create: max_n=%lld outside [1, 2^31)", (long long)max_n);
  BE_CHECK(max_classes >= 1, "ivx_backend_create: max_classes must be >= 1");
  BE_HIP(hipSetDevice(device));
  ivx_backend* b = new ivx_backend();
  b->device = device;
  b->max_dim = max_dim;
  b->max_n = max_n;
  b->max_classes = max_classes;
  const size_t d = max_dim, d2 = d * d, ne = even(max_dim), ne2 = ne * ne;
  bool ok = alloc(&b->sums, (size_t)max_classes * d) && alloc(&b->counts, max_classes) &&
            alloc(&b->M2, d2) && alloc(&b->Sw, d2) && alloc(&b->Sb, d2) && alloc(&b->mean, d) &&
            alloc(&b->Aj, ne2) && alloc(&b->Vj, ne2) && alloc(&b->wj, ne) &&
            alloc(&b->Wh, d2) && alloc(&b->T1, d2) && alloc(&b->T2, d2) &&
            alloc(&b->coef, 2 * d + 1) && alloc(&b->muA, d) &&
            alloc(&b->Z1, (size_t)max_n * d) && alloc(&b->Z2, (size_t)max_n * d) &&
            alloc(&b->idx, d) && alloc(&b->flags, 4) && alloc(&b->rot, ne / 2) &&
            alloc(&b->part, 128) &&
            hipMemset(b->flags, 0, sizeof(int) * 4) == hipSuccess;
  if (!ok) {
    be_free(b);
    set_error("ivx_backend_create: allocation failed");
    return IVX_ENOMEM;
  }
  *out = b;
  return IVX_OK;
}

void ivx_backend_destroy(ivx_backend* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);  // teardown: best effort
  (void)hipDeviceSynchronize();
  be_free(b);
}

ivx_status ivx_backend_whitening(ivx_backend* b, const float* X, int64_t n, int32_t dim,
                                 double* mean, double* W, void* stream) {
  BE_CHECK(b && X && mean && W, "ivx_backend_whitening: null argument");
  BE_CHECK(dim >= 2 && dim <= b->max_dim, "ivx_backend_whitening: dim outside [2, max_dim]");
  BE_CHECK(n >= 2 && n <= b->max_n, "ivx_backend_whitening: n outside [2, max_n]");
  BE_HIP(hipSetDevice(b->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  scatter(b, X, n, dim, nullptr, 1, s);  // one class: Sw is the covariance
  whitener(b, b->Sw, dim, W, true, s);
  BE_HIP(hipMemcpyAsync(mean, b->mean, sizeof(double) * dim, hipMemcpyDeviceToDevice, s));
  int f[4];
  ivx_status st = read_flags(b, s, f);
  if (st != IVX_OK) return st;
  if (f[1]) {
    set_error("ivx_backend_whitening: covariance is singular (%d eigenvalues below %g of the "
              "largest)", f[1], kFloor);
    return IVX_ENOTPD;
  }
  return IVX_OK;
}

ivx_status ivx_backend_lnorm(ivx_backend* b, const float* X, int64_t n, int32_t dim,
                             const double* mean, const double* W, float* Y, void* stream) {
  BE_CHECK(b && X && Y, "ivx_backend_lnorm: null argument");
  BE_CHECK(dim >= 1 && dim <= b->max_dim, "ivx_backend_lnorm: dim outside [1, max_dim]");
  BE_CHECK(n >= 0, "ivx_backend_lnorm: negative n");
  BE_HIP(hipSetDevice(b->device));
  be_lnorm(X, n, dim, mean, W, Y, reinterpret_cast<hipStream_t>(stream));
  return IVX_OK;
}

ivx_status ivx_backend_lda(ivx_backend* b, const float* X, int64_t n, int32_t dim,
                           const int32_t* labels, int32_t K, int32_t out_dim, double* V,
                           double* eigval, void* stream) {
  BE_CHECK(b && X && labels && V, "ivx_backend_lda: null argument");
  BE_CHECK(dim >= 2 && dim <= b->max_dim, "ivx_backend_lda: dim outside [2, max_dim]");
  BE_CHECK(n >= 2 && n <= b->max_n, "ivx_backend_lda: n outside [2, max_n]");
  BE_CHECK(K >= 2 && K <= b->max_classes, "ivx_backend_lda: K outside [2, max_classes]");
  BE_CHECK(out_dim >= 1 && out_dim <= dim, "ivx_backend_lda: out_dim outside [1, dim]");
  BE_HIP(hipSetDevice(b->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  scatter(b, X, n, dim, labels, K, s);
  gen_eig(b, dim, s);
  be_rank_desc(b->wj, dim, out_dim, b->idx, s);
  be_gather_cols(b->Vj, even(dim), b->idx, dim, out_dim, b->wj, b->T1, eigval, s);
  be_dgemm(b->Wh, false, dim, false, b->T1, out_dim, false, V, out_dim, false, dim, out_dim, dim,
           nullptr, s);                                          // V = Wh U_top
  int f[4];
  ivx_status st = read_flags(b, s, f);
  if (st != IVX_OK) return st;
  BE_CHECK(f[0] == 0, "ivx_backend_lda: %d labels outside [0, K)", f[0]);
  if (f[1]) {
    set_error("ivx_backend_lda: within-class scatter is singular (fewer vectors than classes "
              "plus dimensions?)");
    return IVX_ENOTPD;
  }
  return IVX_OK;
}

ivx_status ivx_backend_project(ivx_backend* b, const float* X, int64_t n, int32_t dim,
                               const double* V, int32_t out_dim, float* Y, void* stream) {
  BE_CHECK(b && X && V && Y, "ivx_backend_project: null argument");
  BE_CHECK(dim >= 1 && dim <= b->max_dim && out_dim >= 1 && out_dim <= b->max_dim,
           "ivx_backend_project: dimensions outside [1, max_dim]");
  BE_CHECK(n >= 0 && n <= ((int64_t)1 << 31) - 1, "ivx_backend_project: bad n");
  BE_HIP(hipSetDevice(b->device));
  be_dgemm(X, true, dim, false, V, out_dim, false, Y, out_dim, true, (int)n, out_dim, dim, nullptr,
           reinterpret_cast<hipStream_t>(stream));
  return IVX_OK;
}

ivx_status ivx_backend_plda_fit(ivx_backend* b, const float* Y, int64_t n, int32_t d,
                                const int32_t* labels, int32_t K, double* mu, double* A,
                                double* psi, void* stream) {
  BE_CHECK(b && Y && labels && mu && A && psi, "ivx_backend_plda_fit: null argument");
  BE_CHECK(d >= 2 && d <= b->max_dim, "ivx_backend_plda_fit: d outside [2, max_dim]");
  BE_CHECK(n >= 2 && n <= b->max_n, "ivx_backend_plda_fit: n outside [2, max_n]");
  BE_CHECK(K >= 2 && K <= b->max_classes, "ivx_backend_plda_fit: K outside [2, max_classes]");
  BE_HIP(hipSetDevice(b->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  scatter(b, Y, n, d, labels, K, s);  // W = Sw, B = Sb
  gen_eig(b, d, s);                   // Wh^T W Wh = I, U^T (Wh^T B Wh) U = diag(psi)
  be_dgemm(b->Wh, false, d, false, b->Vj, even(d), false, A, d, false, d, d, d, nullptr, s);
  BE_HIP(hipMemcpyAsync(psi, b->wj, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
  BE_HIP(hipMemcpyAsync(mu, b->mean, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
  int f[4];
  ivx_status st = read_flags(b, s, f);
  if (st != IVX_OK) return st;
  BE_CHECK(f[0] == 0, "ivx_backend_plda_fit: %d labels outside [0, K)", f[0]);
  if (f[1]) {
    set_error("ivx_backend_plda_fit: within-speaker covariance is singular");
    return IVX_ENOTPD;
  }
  return IVX_OK;
}

ivx_status ivx_backend_plda_score(ivx_backend* b, const double* mu, const double* A,
                                  const double* psi, int32_t d, const float* Y1, int64_t n1,
                                  const float* Y2, int64_t n2, const int32_t* trials, int64_t T,
                                  float* scores, void* stream) {
  BE_CHECK(b && mu && A && psi && Y1 && Y2 && (T == 0 || (trials && scores)),
           "ivx_backend_plda_score: null argument");
  BE_CHECK(d >= 1 && d <= b->max_dim, "ivx_backend_plda_score: d outside [1, max_dim]");
  BE_CHECK(n1 >= 1 && n1 <= b->max_n && n2 >= 1 && n2 <= b->max_n,
           "ivx_backend_plda_score: n1, n2 outside [1, max_n]");
  BE_CHECK(T >= 0, "ivx_backend_plda_score: negative T");
  BE_HIP(hipSetDevice(b->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // z = A^T (y - mu) = (y^T A) - (mu^T A), rows of Z1 / Z2
  be_dgemm(mu, false, d, false, A, d, false, b->muA, d, false, 1, d, d, nullptr, s);
  be_dgemm(Y1, true, d, false, A, d, false, b->Z1, d, true, (int)n1, d, d, b->muA, s);
  const float* Z2 = b->Z1;
  if (Y2 != Y1 || n2 != n1) {
    be_dgemm(Y2, true, d, false, A, d, false, b->Z2, d, true, (int)n2, d, d, b->muA, s);
    Z2 = b->Z2;
  }
  be_plda_coef(psi, d, b->coef, s);
  be_plda_score(b->Z1, n1, Z2, n2, d, b->coef, trials, T, scores, b->flags + 2, s);
  return IVX_OK;
}

ivx_status ivx_backend_status(ivx_backend* b, void* stream) {
  BE_CHECK(b, "ivx_backend_status: null argument");
  BE_HIP(hipSetDevice(b->device));
  int f[4];
  ivx_status st = read_flags(b, reinterpret_cast<hipStream_t>(stream), f);
  if (st != IVX_OK) return st;
  BE_CHECK(f[2] == 0, "ivx_backend_plda_score: %d trials index outside the score sets", f[2]);
  return IVX_OK;
}

ivx_status ivx_eer(const float* scores, const uint8_t* is_target, int64_t n, double* eer) {
  BE_CHECK(scores && is_target && eer && n >= 2, "ivx_eer: null argument or n < 2");
  std::vector<float> tg, nt, all(scores, scores + n);
  for (int64_t i = 0; i < n; ++i) (is_target[i] ? tg : nt).push_back(scores[i]);
  BE_CHECK(!tg.empty() && !nt.empty(), "ivx_eer: needs target and non-target trials");
  std::sort(tg.begin(), tg.end());
  std::sort(nt.begin(), nt.end());
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  // operating points at every distinct score and above all of them: misses
  // are targets < t, false alarms non-targets >= t; the EER is where the
  // segments between consecutive points cross P_miss = P_fa
  all.push_back(INFINITY);
  double best = 1.0;
  double pm0 = 0.0, pf0 = 1.0;
  bool first = true;
  size_t im = 0, ifa = 0;  // targets / non-targets below t
  for (float t : all) {
    while (im < tg.size() && tg[im] < t) ++im;
    while (ifa < nt.size() && nt[ifa] < t) ++ifa;
    const double pm = (double)im / tg.size();
    const double pf = (double)(nt.size() - ifa) / nt.size();
    if (!first && pm0 <= pf0 && pm >= pf) {
      const double d0 = pf0 - pm0, d1 = pf - pm;
      const double lam = d0 != d1 ? d0 / (d0 - d1) : 0.0;
      best = pm0 + lam * (pm - pm0);
      break;
    }
    pm0 = pm;
    pf0 = pf;
    first = false;
  }
  *eer = best;
  return IVX_OK;
}

}  // extern "C"
