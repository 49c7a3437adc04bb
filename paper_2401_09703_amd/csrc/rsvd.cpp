// Initial truncated SVD of a sparse matrix on the GPU: the randomised range
// finder with power iterations (Halko, Martinsson and Tropp, 2011, Algorithms
// 4.4 and 5.1), the method the paper's introduction points to for the
// starting factors that every experiment of Section 5 updates from.
//
//   Q = orth(A Omega);  q times: Z = orth(A^T Q), Q = orth(A Z)
//   W = A^T Q (= B^T for B = Q^T A);  W^T W = F diag(lambda) F^T
//   U = orth(Q F_k),  sigma = sqrt(lambda_k),  V = orth(W F_k diag(1/sigma))
//
// Every product with A or A^T is the CSR-times-panel kernel on the CSR of A
// and on the CSR of A^T that the radix-sort transpose builds once; every
// orth() is Cholesky QR with column dropping and random completion (one pass
// where the basis only feeds the next product, two where it becomes a
// factor, the second of U's and V's only when their first had work to do);
// the l x l eigenproblem is the Rayleigh-Ritz eigensolver of the
// update path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/svlcov.h"
#include "k_rsvd.hpp"
#include "kernels.hpp"

namespace {

svlcov_status herr(hipError_t e) {
  if (e == hipSuccess) return SVLCOV_OK;
  if (e == hipErrorOutOfMemory) return SVLCOV_E_NOMEM;
  return SVLCOV_E_DEVICE;
}

#define RV_TRY(expr)                     \
  do {                                   \
    svlcov_status _s = herr(expr);       \
    if (_s != SVLCOV_OK) return _s;      \
  } while (0)

// after the workspace exists: free it (ordered after the work already
// enqueued) before reporting the failure
#define RV_TRY_WS(expr)                                  \
  do {                                                   \
    svlcov_status _s = herr(expr);                       \
    if (_s != SVLCOV_OK) {                               \
      (void)hipFreeAsync(mem, st);                       \
      (void)hipStreamSynchronize(st);                    \
      return _s;                                         \
    }                                                    \
  } while (0)

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// pivots at or below this fraction of the largest squared column norm are
// dropped (relative singular value ~3e-7: below what an FP64 Gram resolves)
constexpr double ORTH_RTOL = 1e-13;
// right vectors of singular values below this fraction of sigma_0 are
// completed instead of divided by sigma (their eigenvalue is rounding noise)
constexpr double SIGMA_TOL = 1e-7;

struct PhaseTimer {
  hipStream_t st;
  bool on;
  std::vector<int> ph;
  std::vector<hipEvent_t> ev;
  int cur = -1;
  PhaseTimer(hipStream_t s, bool enabled) : st(s), on(enabled) {}
  void mark(int phase) {   // the work enqueued from here on counts to phase
    if (!on) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
    (void)hipEventRecord(e, st);
    ph.push_back(phase);
    ev.push_back(e);
  }
  void collect(double *ms, int count) {
    for (int i = 0; i < count; ++i) ms[i] = 0.0;
    for (size_t i = 0; i + 1 < ev.size(); ++i) {
      float t = 0.f;
      if (ph[i] >= 0 && ph[i] < count && hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess)
        ms[ph[i]] += t;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

}  // namespace

extern "C" {

svlcov_status svlcov_rsvd(const svlcov_csr *A, int32_t k, int32_t l, int32_t power,
                          const double *Omega, double *U, double *sigma, double *V,
                          double *phase_ms, void *stream) {
  if (!A || !Omega || !U || !sigma || !V) return SVLCOV_E_INVALID;
  if (l != 16 && l != 32 && l != 64 && l != 128) return SVLCOV_E_UNSUPPORTED;
  if (k < 1 || k > l || power < 0 || power > 64) return SVLCOV_E_INVALID;
  const int64_t m = A->rows, n = A->cols, nnz = A->nnz;
  if (m < 0 || n < 0 || nnz < 0 || !A->row_ptr) return SVLCOV_E_INVALID;
  if (nnz > 0 && (!A->col_idx || !A->val)) return SVLCOV_E_INVALID;
  if (A->val_dtype != SVLCOV_F32 && A->val_dtype != SVLCOV_F64) return SVLCOV_E_INVALID;
  if (m < l || n < l) return SVLCOV_E_SHAPE;
  if (m > INT32_MAX || n > INT32_MAX || nnz > INT32_MAX) return SVLCOV_E_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int vdt = A->val_dtype;
  const size_t vsz = vdt == SVLCOV_F64 ? sizeof(double) : sizeof(float);
  const bool host = A->on_device == 0;

  const size_t ewd = svl::eig_work_doubles(l, k);
  const size_t ws_len = std::max((size_t)64 * l * l, svl::ts_gram_ws(std::max(m, n), l));
  size_t total = al(sizeof(SvDevInfo)) + al(svl::TRI_FLAG_WORDS * sizeof(unsigned));
  if (host) total += al((size_t)(m + 1) * 8) + al((size_t)nnz * 4) + al((size_t)nnz * vsz);
  total += al(svl::csr_transpose_bytes(nnz, n)) + al((size_t)(n + 1) * 8) + al((size_t)nnz * 4) +
           al((size_t)nnz * 8);
  total += 2 * al((size_t)m * l * 8) + 2 * al((size_t)n * l * 8);
  total += 2 * al((size_t)l * l * 8) + al((size_t)l * 4) + al(ws_len * 8) + al(ewd * 8) +
           al((size_t)k * 8) + al((size_t)k * l * 8) + al(sizeof(int32_t));
  char *mem = nullptr;
  RV_TRY(hipMallocAsync((void **)&mem, total, st));
  char *p = mem;
  auto take = [&p](size_t bytes) { char *r = p; p += al(bytes); return r; };
  SvDevInfo *info = (SvDevInfo *)take(sizeof(SvDevInfo));
  unsigned *flags = (unsigned *)take(svl::TRI_FLAG_WORDS * sizeof(unsigned));
  const int64_t *rp = A->row_ptr;
  const int32_t *ci = A->col_idx;
  const void *v = A->val;
  if (host) {
    int64_t *rpd = (int64_t *)take((size_t)(m + 1) * 8);
    int32_t *cid = (int32_t *)take((size_t)nnz * 4);
    void *vd = take((size_t)nnz * vsz);
    RV_TRY_WS(hipMemcpyAsync(rpd, rp, (size_t)(m + 1) * 8, hipMemcpyHostToDevice, st));
    if (nnz > 0) {
      RV_TRY_WS(hipMemcpyAsync(cid, ci, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
      RV_TRY_WS(hipMemcpyAsync(vd, v, (size_t)nnz * vsz, hipMemcpyHostToDevice, st));
    }
    rp = rpd;
    ci = cid;
    v = vd;
  }
  void *tscr = take(svl::csr_transpose_bytes(nnz, n));
  int64_t *rpT = (int64_t *)take((size_t)(n + 1) * 8);
  int32_t *ciT = (int32_t *)take((size_t)nnz * 4);
  double *vT = (double *)take((size_t)nnz * 8);
  double *Pm = (double *)take((size_t)m * l * 8);
  double *Qm = (double *)take((size_t)m * l * 8);
  double *Pn = (double *)take((size_t)n * l * 8);
  double *Qn = (double *)take((size_t)n * l * 8);
  double *G = (double *)take((size_t)l * l * 8);
  double *Out = (double *)take((size_t)l * l * 8);
  int32_t *complete = (int32_t *)take((size_t)l * 4);
  double *ws = (double *)take(ws_len * 8);
  double *ework = (double *)take(ewd * 8);
  double *lam = (double *)take((size_t)k * 8);
  double *Fv = (double *)take((size_t)k * l * 8);
  int32_t *need = (int32_t *)take(sizeof(int32_t));

  PhaseTimer tm(st, phase_ms != nullptr);
  RV_TRY_WS(hipMemsetAsync(info, 0, al(sizeof(SvDevInfo)) + svl::TRI_FLAG_WORDS * sizeof(unsigned),
                        st));
  tm.mark(0);
  svl::validate_csr(st, m, n, nnz, rp, ci, v, vdt, info, 0);
  svl::check_finite_wide(st, n * l, Omega, info);
  svl::csr_transpose(st, m, n, nnz, rp, ci, v, vdt, rpT, ciT, vT, tscr, info);
  uint64_t seed = 0x5EEDull;
  auto prod_A = [&](const double *X, double *Y) {
    tm.mark(1);
    svl::csr_dense(st, l, m, rp, ci, v, vdt, X, Y, info);
  };
  auto prod_AT = [&](const double *X, double *Y) {
    tm.mark(1);
    svl::csr_dense(st, l, n, rpT, ciT, vT, SVLCOV_F64, X, Y, info);
  };
  // an orthonormalisation that only feeds the next product needs a
  // well-conditioned basis (one pass); the bases that become factors need
  // two passes
  auto orth = [&](int64_t R, int L, double *&X, double *&Y, int passes) {
    tm.mark(2);
    double *r = svl::orth_cols(st, R, L, X, Y, passes, G, Out, complete, ws, ws_len, ++seed,
                               ORTH_RTOL, info);
    if (r != Y) std::swap(X, Y);   // the result is always left in Y
  };
  prod_A(Omega, Pm);
  orth(m, l, Pm, Qm, power > 0 ? 1 : 2);
  for (int it = 0; it < power; ++it) {
    prod_AT(Qm, Pn);
    orth(n, l, Pn, Qn, 1);
    prod_A(Qn, Pm);
    orth(m, l, Pm, Qm, it == power - 1 ? 2 : 1);
  }
  prod_AT(Qm, Pn);   // W = A^T Q
  tm.mark(3);
  svl::ts_gram(st, n, l, Pn, G, ws, info);   // W^T W, both triangles
  unsigned epoch = 0;
  const int er = svl::eig_topk(st, l, G, k, lam, Fv, ework, flags, &epoch, info);
  tm.mark(4);
  // U = Q F is orthonormal when F is; the vectors of a (near-)zero cluster
  // of eigenvalues need not be, so U too is orthonormalised in column order
  // (the columns of resolved singular values come first and stay as they
  // are), with the second pass only where the first had work to do
  svl::gemm_f64(st, false, true, m, k, l, 1.0, Qm, l, Fv, l, 0.0, U, k, info);
  tm.mark(2);
  (void)svl::orth_cols_cond(st, m, k, U, Pm, G, Out, complete, need, ws, ws_len, ++seed,
                            ORTH_RTOL, info);   // result in U
  tm.mark(4);
  svl::gemm_f64(st, false, true, n, k, l, 1.0, Pn, l, Fv, l, 0.0, V, k, info);
  svl::inv_sigma_cols(st, n, k, lam, sigma, V, SIGMA_TOL, info);
  tm.mark(2);
  (void)svl::orth_cols_cond(st, n, k, V, Qn, G, Out, complete, need, ws, ws_len, ++seed,
                            ORTH_RTOL, info);   // result in V
  tm.mark(4);
  svl::check_finite(st, k, sigma, info, 0);
  tm.mark(-1);
  int32_t status = 0;
  const hipError_t ce = hipMemcpyAsync(&status, &info->status, sizeof(int32_t),
                                       hipMemcpyDeviceToHost, st);
  const hipError_t fe = hipFreeAsync(mem, st);
  const hipError_t se = hipStreamSynchronize(st);
  if (phase_ms) tm.collect(phase_ms, SVLCOV_RSVD_PHASES);
  if (ce != hipSuccess || fe != hipSuccess || se != hipSuccess || er != 0)
    return SVLCOV_E_DEVICE;
  return status ? (svlcov_status)status : SVLCOV_OK;
}

}  // extern "C"
