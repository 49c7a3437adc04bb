// Update engine and C ABI: the factor state of one matrix in the extended
// decomposition (Section 3.2), host-side validation, workspace management and
// the step sequence of each update (Algorithms 3, 4 and 11), every step of
// which is a kernel on the state's stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/svlcov.h"
#include "kernels.hpp"
#include "state.hpp"

using svl_state::DevBuf;
using svl_state::EvRec;
using svl_state::Snapshot;

namespace {

constexpr double DEF_TOL[3] = {1e-13, 1e-6, 1e-5};   // FP64, FP32, BF16X3
constexpr double DEF_COND[3] = {1e4, 1e2, 1e2};   // FP64, FP32, BF16X3

// Phases of one update, timed with HIP events on the state's stream when
// profiling is enabled (names in svlcov_phase_name).
enum Phase {
  PH_VALIDATE, PH_SPMM, PH_SGRAM, PH_RGRAM, PH_CHOL, PH_BUILDK, PH_KKT, PH_TRIDIAG, PH_BISECT,
  PH_STEIN, PH_BACK, PH_RECOVER, PH_ORTH, PH_SMALL, PH_TRSM, PH_COMMIT, PH_ITER, PH_COUNT
};
const char *PHASE_NAMES[PH_COUNT] = {
    "validate", "spmm_w", "sparse_gram", "resid_gram", "cholesky", "build_K", "kkt_gemm",
    "tridiag", "bisect", "stein", "backtransform", "recover_G", "orthonormalize",
    "small_factor", "trsm", "commit", "subspace_iter"};

}  // namespace

namespace {

struct BusyGuard {
  svlcov_state *h;
  bool ok;
  explicit BusyGuard(svlcov_state *hh) : h(hh) {
    bool expected = false;
    ok = h->busy.compare_exchange_strong(expected, true);
  }
  ~BusyGuard() {
    if (ok) h->busy.store(false);
  }
};

svlcov_status dev_err(hipError_t e) {
  if (e == hipSuccess) return SVLCOV_OK;
  if (e == hipErrorOutOfMemory) return SVLCOV_E_NOMEM;
  return SVLCOV_E_DEVICE;
}

hipEvent_t get_event(svlcov_state *h) {
  if (!h->evpool.empty()) {
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct PhaseScope {
  svlcov_state *h;
  int ph;
  hipStream_t st;
  hipEvent_t a = nullptr;
  PhaseScope(svlcov_state *hh, int p, hipStream_t s = nullptr)
      : h(hh), ph(p), st(s ? s : hh->stream) {
    if (h->prof && ((h->prof_mask >> p) & 1u)) {
      a = get_event(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~PhaseScope() {
    if (!a) return;
    hipEvent_t b = get_event(h);
    if (!b) return;
    (void)hipEventRecord(b, st);
    h->recs.push_back({ph, a, b});
  }
};

// The append form's M = K K^T is assembled from sigma, C' and the sparse Gram
// alone, so the eigensolver does not wait for the residual Gram's Cholesky:
// when the eigensolver is the subspace iteration without cooperative kernels
// (basis of at most EIG_ONE_BLOCK_N columns), the Cholesky and K go to a
// second stream and the two meet before G = K^T F.  SVLCOV_NO_OVERLAP=1
// keeps one stream.
bool side_stream(svlcov_state *h, int64_t N, int K) {
  static const bool off = [] {
    const char *ev = getenv("SVLCOV_NO_OVERLAP");
    return ev && atoi(ev) != 0;
  }();
  if (off || !h->side_ok || h->prec == SVLCOV_FP64 || !svl::chefsi_applies(N, K) ||
      svl::chefsi_block(K) > svl::EIG_ONE_BLOCK_N)
    return false;
  if (!h->side) {
    hipStream_t sd = nullptr;
    if (hipStreamCreateWithFlags(&sd, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
      h->ev_fork = nullptr;
      (void)hipStreamDestroy(sd);
      return false;
    }
    h->side = sd;
    int n = 0;
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, h->device);
    h->ncu = n > 0 ? n : 1;
  }
  return true;
}

#define SV_TRY(expr)                                   \
  do {                                                 \
    svlcov_status _s = dev_err(expr);                  \
    if (_s != SVLCOV_OK) return _s;                    \
  } while (0)

svlcov_status ensure(svlcov_state *h, DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes) return SVLCOV_OK;
  size_t want = bytes + bytes / 4 + 4096;
  const bool hooks = !h->lent;   // a server's lent buffer stays plain HIP memory
  svl_state::state_free(h, b.p, b.bytes, hooks);
  b.p = nullptr;
  b.bytes = 0;
  SV_TRY(svl_state::state_alloc(h, &b.p, want, hooks));
  b.bytes = want;
  return SVLCOV_OK;
}

// Grow the row capacity of a tall factor (rows x k), keeping its contents.
svlcov_status grow_base(svlcov_state *h, void **base, int64_t *cap, int64_t rows_used,
                        int64_t need) {
  if (need <= *cap) return SVLCOV_OK;
  int64_t ncap = *cap + *cap / 2;
  if (ncap < need) ncap = need;
  void *nb = nullptr;
  SV_TRY(svl_state::state_alloc(h, &nb, (size_t)ncap * h->k * h->elem()));
  if (rows_used > 0)
    SV_TRY(hipMemcpyAsync(nb, *base, (size_t)rows_used * h->k * h->elem(),
                          hipMemcpyDeviceToDevice, h->stream));
  svl_state::state_free(h, *base, (size_t)*cap * h->k * h->elem());
  *base = nb;
  *cap = ncap;
  return SVLCOV_OK;
}

bool finite_vals(const void *v, int dt, int64_t n) {
  if (dt == SVLCOV_F64) {
    const double *x = (const double *)v;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(x[i])) return false;
  } else {
    const float *x = (const float *)v;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(x[i])) return false;
  }
  return true;
}

// Host check of a canonical CSR (only for host-resident inputs).
svlcov_status check_host_csr(const svlcov_csr *E) {
  if (!E->row_ptr || (E->nnz > 0 && (!E->col_idx || !E->val))) return SVLCOV_E_INVALID;
  if (E->row_ptr[0] != 0 || E->row_ptr[E->rows] != E->nnz) return SVLCOV_E_INVALID;
  for (int64_t i = 0; i < E->rows; ++i) {
    const int64_t p0 = E->row_ptr[i], p1 = E->row_ptr[i + 1];
    if (p0 < 0 || p1 < p0 || p1 > E->nnz) return SVLCOV_E_INVALID;
    int32_t prev = -1;
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t c = E->col_idx[p];
      if (c <= prev || c >= E->cols) return SVLCOV_E_INVALID;
      prev = c;
    }
  }
  if (!finite_vals(E->val, E->val_dtype, E->nnz)) return SVLCOV_E_NUMERIC;
  return SVLCOV_OK;
}

svlcov_status check_csr_header(const svlcov_csr *E) {
  if (!E) return SVLCOV_E_INVALID;
  if (E->rows < 0 || E->cols < 0 || E->nnz < 0) return SVLCOV_E_INVALID;
  if (E->val_dtype != SVLCOV_F32 && E->val_dtype != SVLCOV_F64) return SVLCOV_E_INVALID;
  if (E->nnz > INT32_MAX || E->cols > INT32_MAX) return SVLCOV_E_UNSUPPORTED;
  return SVLCOV_OK;
}

// Device view of a CSR input (host inputs are copied into `stage` at `off`).
struct DevCsr {
  int64_t rows, cols, nnz;
  const int64_t *rp;
  const int32_t *ci;
  const void *v;
  int vdt;
};

size_t csr_stage_bytes(const svlcov_csr *E) {
  if (E->on_device) return 0;
  const size_t vb = E->val_dtype == SVLCOV_F64 ? 8 : 4;
  return ((size_t)(E->rows + 1) * 8 + 255) / 256 * 256 + ((size_t)E->nnz * 4 + 255) / 256 * 256 +
         ((size_t)E->nnz * vb + 255) / 256 * 256;
}

svlcov_status to_device(svlcov_state *h, const svlcov_csr *E, char *&cursor, DevCsr *out) {
  out->rows = E->rows;
  out->cols = E->cols;
  out->nnz = E->nnz;
  out->vdt = E->val_dtype == SVLCOV_F64 ? 1 : 0;
  if (E->on_device) {
    out->rp = E->row_ptr;
    out->ci = E->col_idx;
    out->v = E->val;
    return SVLCOV_OK;
  }
  const size_t vb = E->val_dtype == SVLCOV_F64 ? 8 : 4;
  const size_t b_rp = (size_t)(E->rows + 1) * 8, b_ci = (size_t)E->nnz * 4,
               b_v = (size_t)E->nnz * vb;
  char *prp = cursor;
  cursor += (b_rp + 255) / 256 * 256;
  char *pci = cursor;
  cursor += (b_ci + 255) / 256 * 256;
  char *pv = cursor;
  cursor += (b_v + 255) / 256 * 256;
  SV_TRY(hipMemcpyAsync(prp, E->row_ptr, b_rp, hipMemcpyHostToDevice, h->stream));
  if (b_ci) SV_TRY(hipMemcpyAsync(pci, E->col_idx, b_ci, hipMemcpyHostToDevice, h->stream));
  if (b_v) SV_TRY(hipMemcpyAsync(pv, E->val, b_v, hipMemcpyHostToDevice, h->stream));
  out->rp = (const int64_t *)prp;
  out->ci = (const int32_t *)pci;
  out->v = pv;
  return SVLCOV_OK;
}

// Workspace carving (all regions 256-byte aligned).
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    T *p = (T *)(base ? base + off : nullptr);
    off += (count * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

int mode_of(int prec) { return prec == SVLCOV_FP64 ? 0 : (prec == SVLCOV_FP32 ? 1 : 2); }

}  // namespace

// Device workspace of one update (the carving of op_append / op_weights
// below, replayed without memory): op 0 add_rows, 1 add_cols, 2 weights.
// Words of the per-nonzero row-id buffer of the sparse Gram; it is free again
// by the commit, where it holds the deterministic scatter's sort.
static int64_t rid_words(int64_t nnz) {
  const int64_t a = nnz > 0 ? nnz : 1;
  const int64_t b = (int64_t)((svl::scatter_det_bytes(nnz) + 3) / 4);
  return a > b ? a : b;
}

// Scratch of F's row orthonormalisation on the side stream: Gram, inverse,
// product and split-K partials of the k x k Gram (at most 64).
static size_t orth_side_doubles(int K, int64_t N) {
  return (size_t)66 * K * K + (size_t)K * N;
}

size_t svl_state::op_workspace_bytes(int op, int K, int64_t s, int64_t nnzA, int64_t nnzB) {
  Carver c{nullptr};
  const int64_t N = K + s;
  const size_t nbl = ((s + svl::CHOL_NB - 1) / svl::CHOL_NB) * svl::CHOL_NB * svl::CHOL_NB;
  const int64_t nnz = nnzA > nnzB ? nnzA : nnzB;
  const int sides = op == 2 ? 2 : 1;
  for (int q = 0; q < sides; ++q) {
    c.take<double>(s * K);   // C'
    c.take<float>(s * K);    // C' (FP32)
    c.take<double>(s);       // row norms
    c.take<double>(s * s);   // Gram / Cholesky factor
    c.take<double>(nbl);     // diagonal-block inverses
    c.take<double>(s * K);   // Y
    c.take<double>(s * K);   // M rows
  }
  if (op == 2) {
    c.take<double>(N * s);
    c.take<double>(N * s);
  }
  c.take<double>(N * N);
  c.take<double>(N * N);
  c.take<double>(K);
  c.take<double>(K);
  c.take<int32_t>(K);
  c.take<double>(K * N);
  c.take<double>(K * N);
  c.take<double>(svl::eig_update_work_doubles(N, K));
  c.take<double>(K * K);
  for (int q = 0; q < 4; ++q) c.take<double>(K * K);
  c.take<int32_t>(2);
  c.take<double>(2 * K * K + 9 * K * N);
  c.take<double>(orth_side_doubles(K, N));
  c.take<int32_t>(rid_words(nnz));
  return c.off;
}

void svl_state::proj_offsets(int op, int K, int64_t s, int q, size_t *cp64, size_t *cp32,
                             size_t *rown) {
  Carver c{nullptr};
  if (op != 2) {   // op_append: C', C' (FP32), row norms first
    *cp64 = c.off; c.take<double>(s * K);
    *cp32 = c.off; c.take<float>(s * K);
    *rown = c.off; c.take<double>(s);
    return;
  }
  // op_weights: C'_D, C'_E, FP32 copies, row norms of D and of E_m
  size_t o[6];
  o[0] = c.off; c.take<double>(s * K);
  o[1] = c.off; c.take<double>(s * K);
  o[2] = c.off; c.take<float>(s * K);
  o[3] = c.off; c.take<float>(s * K);
  o[4] = c.off; c.take<double>(s);
  o[5] = c.off; c.take<double>(s);
  *cp64 = o[q];
  *cp32 = o[2 + q];
  *rown = o[4 + q];
}

namespace {


// One side's orthogonalisation: projection, sparse Gram, residual Gram and its
// Cholesky (Algorithm 2 realised as R^T R = E E^T - (E V)(E V)^T, Lemma 3).
// cst: the stream of the residual Gram and the Cholesky (the state's unless
// the caller runs them beside the eigensolver; it then orders cst after the
// sparse Gram here and joins cst itself).
template <typename T>
void orthogonalise(svlcov_state *h, const DevCsr &E, const T *base, const double *W, double *Cp64,
                   float *Cp32, double *rown, double *Gm, double *Linv, int32_t *rid, int which,
                   bool chol = true, double *dws = nullptr, size_t dws_len = 0,
                   double *Scopy = nullptr, int64_t lds_copy = 0, hipStream_t cst = nullptr) {
  const int K = h->k;
  const int64_t s = E.rows;
  hipStream_t st = h->stream;
  if (!cst) cst = st;
  if (!h->proj_ready[which]) {
    PhaseScope ps(h, PH_SPMM);
    // the variants (no Cholesky) take C' accumulated in FP64: a Lanczos
    // basis of a nearly flat spectrum turns the rounding of an FP32 sum into
    // a different subspace
    svl::spmm_w<T>(st, K, s, E.rp, E.ci, E.v, E.vdt, base, W, Cp64,
                   h->prec == SVLCOV_FP64 ? nullptr : Cp32, rown, h->info, !chol);
  }
  // the Cholesky's drop scale max_i ||e_i||^2, also the sparse Gram's
  // fixed-point scale
  svl::max_into(st, s, rown, h->info, which);
  {
    PhaseScope ps(h, PH_SGRAM);
    svl::sparse_gram(st, s, E.cols, E.nnz, E.rp, E.ci, E.v, E.vdt, rid, Gm, s, dws, dws_len,
                     h->info, which);
    // S = E E^T is also the trailing block of M = K K^T (R^T R = S - C' C'^T)
    if (Scopy) svl::copy_strided(st, s, s, Gm, s, 1, Scopy, lds_copy, h->info);
  }
  if (cst != st) {
    (void)hipEventRecord(h->ev_fork, st);
    (void)hipStreamWaitEvent(cst, h->ev_fork, 0);
  }
  {
    // the approximate variants build their basis by a Lanczos or power
    // process on this Gram, which amplifies its rounding: FP64 for them in
    // every mode (the MFMA Gram otherwise)
    PhaseScope ps(h, PH_RGRAM, cst);
    if (h->prec == SVLCOV_FP64 || !chol)
      svl::gemm_f64(cst, false, true, s, s, K, -1.0, Cp64, K, Cp64, K, 1.0, Gm, s, h->info);
    else
      svl::gram_lowp(cst, mode_of(h->prec), s, K, Cp32, Gm, s, h->info);
  }
  if (!chol) return;   // the approximate variants use the Gram itself
  // beside the eigensolver the Cholesky leaves CUs to it: with a block per
  // CU it kept the eigensolver's products from starting.  Up to s ~ 2000 its
  // chain of diagonal blocks, not its trailing products, sets its time (at
  // s = 1000 it runs as fast with 125 blocks as with 250): half the CUs;
  // beyond, the trailing products count (s = 5000: 7.2 ms with 256 blocks
  // alone, 8.9 ms with 224 beside the iteration, 13.4 ms with 128): 7/8
  PhaseScope ps(h, PH_CHOL, cst);
  coop_enter(h, cst);
  static const int side_blocks = [] {   // SVLCOV_SIDE_BLOCKS overrides it for sweeps
    const char *ev = getenv("SVLCOV_SIDE_BLOCKS");
    return ev ? atoi(ev) : 0;
  }();
  const int cap = side_blocks > 0 ? side_blocks
                                  : std::max(1, s <= 2048 ? h->ncu / 2 : h->ncu * 7 / 8);
  const int crc = svl::cholesky_coop(cst, s, Gm, s, Linv, h->rank_tol, h->info, which, h->flags,
                                     &h->epoch, cst != st ? cap : 0);
  coop_exit(h, cst);
  if (crc) {
    h->launch_failed = true;
    svl::set_status(cst, h->info, SVLCOV_E_DEVICE);
  }
}

// The (k+s) Rayleigh-Ritz SVD of K (N x N) through the eigenpairs of K K^T:
// F (rows of Fv) are the left singular vectors, theta the singular values,
// G = K^T F diag(theta)^{-1} the right ones (rows of Gv); both sets are
// re-orthonormalised, with an orthonormal completion where theta vanishes.
// join: an event on the stream that forms K (NULL: K is formed on the
// state's stream); the state's stream waits for it before anything needs K
// and before a cooperative kernel could run beside the Cholesky.
// orth2 (with join): scratch of orth_side_doubles(K, N) for F's
// orthonormalisation, which then runs on the side stream (from after G is
// formed; the caller joins it) while the state's stream takes G's.
svlcov_status rayleigh_ritz(svlcov_state *h, int64_t N, double *Kmat, double *Mmat, double *lam,
                            double *theta, int32_t *complete, double *Fv, double *Gv,
                            double *eigw, double *gram_kk, const double *Cp_border = nullptr,
                            hipEvent_t join = nullptr, double *orth2 = nullptr) {
  const int K = h->k;
  hipStream_t st = h->stream;
  {
    PhaseScope ps(h, PH_KKT);
    if (Cp_border)   // append form: M from sigma, C' and the sparse Gram, no product
      svl::build_M_border(st, K, N - K, h->sigma, Cp_border, Mmat, h->info);
    else
      svl::gemm_f64(st, false, true, N, N, N, 1.0, Kmat, N, Kmat, N, 0.0, Mmat, N, h->info);
  }
  // FP32 / BF16x3: the k leading eigenpairs by Chebyshev-filtered subspace
  // iteration (dense products on MFMA) to residuals below 1e-9 of the
  // largest eigenvalue, two orders under the rounding of the FP32-stored
  // factors that M is computed from; FP64 keeps the direct solver, whose
  // backward error is at rounding level.  A run that does not converge falls
  // back to the direct solver.
  bool solved = false;
  if (h->prec != SVLCOV_FP64 && svl::chefsi_applies(N, K)) {
    PhaseScope ps(h, PH_ITER);
    if (!h->ctl_host) {
      if (hipHostMalloc((void **)&h->ctl_host, 64 * sizeof(double), 0) != hipSuccess)
        h->ctl_host = nullptr;
      else
        for (int q = 0; q < 64; ++q) h->ctl_host[q] = 0.0;   // no bounds hint yet
    }
    if (h->ctl_host) {
      int iters = 0;
      double fl = 0.0;
      // a basis wider than the one-block tridiagonalisation takes uses the
      // cooperative eigensolver inside
      const bool coop = svl::chefsi_block(K) > svl::EIG_ONE_BLOCK_N;
      if (coop) coop_enter(h);
      const int rc = svl::eig_topk_chefsi(st, N, Mmat, K, lam, Fv, eigw,
                                          svl::eig_update_work_doubles(N, K), h->ctl_host,
                                          1e-9, 8, (uint64_t)h->seq * 7919 + 17, h->info,
                                          &iters, &fl, h->flags, &h->epoch);
      if (coop) coop_exit(h);
      ++h->iter_runs;
      h->iter_steps += iters;
      h->iter_flops += fl;
      if (rc == 0) solved = true;
      else if (rc == 1) ++h->iter_fallbacks;
      else {
        h->launch_failed = true;
        svl::set_status(st, h->info, SVLCOV_E_DEVICE);
      }
    }
  }
  if (join) (void)hipStreamWaitEvent(st, join, 0);
  if (!solved) {
    {
      PhaseScope ps(h, PH_TRIDIAG);
      coop_enter(h);
      const int trc = svl::eig_tridiag(st, N, Mmat, eigw, h->flags, &h->epoch, h->info);
      coop_exit(h);
      if (trc != 0) {
        h->launch_failed = true;
        svl::set_status(st, h->info, SVLCOV_E_DEVICE);
      }
    }
    {
      PhaseScope ps(h, PH_BISECT);
      svl::eig_bisect(st, N, K, lam, eigw, h->info);
    }
    {
      PhaseScope ps(h, PH_STEIN);
      svl::eig_stein(st, N, K, lam, Fv, eigw, h->info);
    }
    {
      PhaseScope ps(h, PH_BACK);
      svl::eig_back(st, N, K, Mmat, Fv, eigw, h->info);
    }
  }
  {
    PhaseScope ps(h, PH_RECOVER);
    svl::gemm_f64_sk(st, false, false, K, N, N, 1.0, Fv, N, Kmat, N, 0.0, Gv, N,
                     gram_kk + 2 * K * K + K * N, (size_t)8 * K * N, h->info);
    svl::theta_scale(st, K, lam, theta, Gv, N, complete, h->info);
  }
  double *linv_kk = gram_kk + K * K, *xtmp = gram_kk + 2 * K * K;
  double *gws = xtmp + K * N;
  const size_t gws_len = (size_t)8 * K * N;
  const bool split = join && orth2;
  if (!split) {
    PhaseScope ps(h, PH_ORTH);
    svl::orthonormalize_rows(st, K, N, Fv, nullptr, (uint64_t)h->seq * 2 + 1, gram_kk, linv_kk,
                             xtmp, gws, gws_len, h->info);
  }
  {
    PhaseScope ps(h, PH_ORTH);
    svl::orthonormalize_rows(st, K, N, Gv, complete, (uint64_t)h->seq * 2 + 2, gram_kk, linv_kk,
                             xtmp, gws, gws_len, h->info);
  }
  if (split) {
    // F's rows on the side stream (the host enqueues G's first: they lead to
    // the triangular solve, the longer chain, and the host's launches are
    // what the device waits for here)
    (void)hipEventRecord(h->ev_fork, st);
    (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
    PhaseScope ps(h, PH_ORTH, h->side);
    svl::orthonormalize_rows(h->side, K, N, Fv, nullptr, (uint64_t)h->seq * 2 + 1, orth2,
                             orth2 + K * K, orth2 + 2 * K * K, orth2 + 2 * K * K + K * N,
                             (size_t)64 * K * K, h->info);
  }
  svl::check_finite(st, K, theta, h->info, h->seq);
  if (hipGetLastError() != hipSuccess) {   // a launch was refused: stop here
    h->launch_failed = true;
    svl::set_status(st, h->info, SVLCOV_E_DEVICE);
  }
  return SVLCOV_OK;
}

// Wnew = W (X[:k] - Cp^T Y), its inverse and condition (X by rows, K x N).
void sparse_side_small(svlcov_state *h, int64_t s, int64_t N, const double *Xv,
                       const double *Cp64, const double *W, const double *Y, double *T1,
                       double *Wnew, double *Winv, int32_t *flag, int side, double *gws,
                       size_t gws_len, bool do_inverse = true) {
  const int K = h->k;
  hipStream_t st = h->stream;
  PhaseScope ps(h, PH_SMALL);
  svl::copy_strided(st, K, K, Xv, 1, N, T1, K, h->info);
  svl::gemm_f64_sk(st, true, false, K, K, s, -1.0, Cp64, K, Y, K, 1.0, T1, K, gws, gws_len,
                   h->info);
  svl::gemm_f64(st, false, false, K, K, K, 1.0, W, K, T1, K, 0.0, Wnew, K, h->info);
  if (do_inverse) svl::inverse_cond(st, K, Wnew, Winv, flag, h->cond_reset, h->info, side);
}

// The sparse-side factor update (Equation (1)): Y = T X[k:] with T = L^{-T}
// (the normalisation of Algorithm 2), Wnew = W (X[:k] - C_n X[k:]) with
// C_n X[k:] = Cp^T Y.  X is given by rows (Xv, K x N).
void sparse_side_math(svlcov_state *h, int64_t s, int64_t N, const double *Xv, const double *Cp64,
                      const double *L, const double *Linv, const double *W, double *Y,
                      double *T1, double *Wnew, double *Winv, int32_t *flag, int side,
                      double *gws, size_t gws_len, bool do_inverse = true) {
  const int K = h->k;
  hipStream_t st = h->stream;
  {
    PhaseScope ps(h, PH_TRSM);
    svl::copy_strided(st, s, K, Xv + K, 1, N, Y, K, h->info);
    coop_enter(h);
    const int src = svl::trsm_coop(st, s, K, L, s, Linv, Y, h->info, h->flags, &h->epoch);
    coop_exit(h);
    if (src) {
      h->launch_failed = true;
      svl::set_status(st, h->info, SVLCOV_E_DEVICE);
    }
  }
  sparse_side_small(h, s, N, Xv, Cp64, W, Y, T1, Wnew, Winv, flag, side, gws, gws_len,
                    do_inverse);
}

template <typename T>
void sparse_side_commit(svlcov_state *h, const DevCsr &E, int64_t rows_used, T *base,
                        const double *Y, double *Mupd, const double *Wnew, const double *Winv,
                        const int32_t *flag, double *W, const double *theta, double *sig,
                        int side, void *scat) {
  const int K = h->k;
  hipStream_t st = h->stream;
  const int mode = mode_of(h->prec);
  PhaseScope ps(h, PH_COMMIT);
  svl::realise<T, T>(st, mode, K, rows_used, base, Wnew, base, flag, h->info);
  svl::append_rows<double>(st, K, E.rows, Y, K, 1, Winv, flag, Mupd, h->info);
  if (h->deterministic)
    svl::scatter_det<T>(st, K, E.rows, E.cols, E.nnz, E.rp, E.ci, E.v, E.vdt, Mupd, base, scat,
                        h->info);
  else
    svl::scatter<T>(st, K, E.rows, E.rp, E.ci, E.v, E.vdt, Mupd, base, h->info);
  svl::commit_small(st, K, Wnew, flag, W, theta, sig, h->info, side);
}

// Row-append form shared by add_rows (append side U, sparse side V) and
// add_cols (append side V, sparse side U, the transpose of the same problem).
template <typename T>
svlcov_status op_append(svlcov_state *h, const svlcov_csr *E, bool rows_form) {
  svlcov_status r = check_csr_header(E);
  if (r != SVLCOV_OK) return r;
  const int K = h->k;
  const int64_t s = E->rows;
  const int64_t nB = rows_form ? h->n : h->m;   // width of E
  const int64_t nA = rows_form ? h->m : h->n;   // rows of the append side
  if (E->cols != nB) return SVLCOV_E_SHAPE;
  if (s == 0) return SVLCOV_OK;
  if (K + s > svl::eig_max_n()) return SVLCOV_E_UNSUPPORTED;
  if (!E->on_device) {
    r = check_host_csr(E);
    if (r != SVLCOV_OK) return r;
  }
  void **Abase = rows_form ? &h->Ubase : &h->Vbase;
  int64_t *Acap = rows_form ? &h->capU : &h->capV;
  r = grow_base(h, Abase, Acap, nA, nA + s);
  if (r != SVLCOV_OK) return r;
  T *A_base = (T *)*Abase;
  T *B_base = (T *)(rows_form ? h->Vbase : h->Ubase);
  double *W_A = rows_form ? h->WU : h->WV;
  double *W_B = rows_form ? h->WV : h->WU;
  const int sideA = rows_form ? 0 : 1, sideB = 1 - sideA;
  const int64_t N = K + s;
  // workspace
  Carver c{nullptr};
  double *orthw_p = nullptr;
  double **orthw = &orthw_p;
  double *orth2 = nullptr;  // F's orthonormalisation on the side stream
  int32_t *rid = nullptr;   // row id per nonzero of E (sparse Gram)
  auto layout = [&](Carver &cv, double **Cp64, float **Cp32, double **rown, double **Gm,
                    double **Linv, double **Kmat, double **Mmat, double **lam, double **theta,
                    int32_t **complete, double **Fv, double **Gv, double **eigw, double **Y,
                    double **T1, double **WnA, double **WiA, double **WnB, double **WiB,
                    double **Mupd, int32_t **flags) {
    *Cp64 = cv.take<double>(s * K);
    *Cp32 = cv.take<float>(s * K);
    *rown = cv.take<double>(s);
    *Gm = cv.take<double>(s * s);
    *Linv = cv.take<double>(((s + svl::CHOL_NB - 1) / svl::CHOL_NB) * svl::CHOL_NB * svl::CHOL_NB);
    *Kmat = cv.take<double>(N * N);
    *Mmat = cv.take<double>(N * N);
    *lam = cv.take<double>(K);
    *theta = cv.take<double>(K);
    *complete = cv.take<int32_t>(K);
    *Fv = cv.take<double>(K * N);
    *Gv = cv.take<double>(K * N);
    *eigw = cv.take<double>(svl::eig_update_work_doubles(N, K));
    *Y = cv.take<double>(s * K);
    *T1 = cv.take<double>(K * K);
    *WnA = cv.take<double>(K * K);
    *WiA = cv.take<double>(K * K);
    *WnB = cv.take<double>(K * K);
    *WiB = cv.take<double>(K * K);
    *Mupd = cv.take<double>(s * K);
    *flags = cv.take<int32_t>(2);
    *orthw = cv.take<double>(2 * K * K + 9 * K * N);
    orth2 = cv.take<double>(orth_side_doubles(K, N));
    rid = cv.take<int32_t>(rid_words(E->nnz));
  };
  double *Cp64, *rown, *Gm, *Linv, *Kmat, *Mmat, *lam, *theta, *Fv, *Gv, *eigw, *Y, *T1, *WnA,
      *WiA, *WnB, *WiB, *Mupd;
  float *Cp32;
  int32_t *complete, *flags;
  layout(c, &Cp64, &Cp32, &rown, &Gm, &Linv, &Kmat, &Mmat, &lam, &theta, &complete, &Fv, &Gv,
         &eigw, &Y, &T1, &WnA, &WiA, &WnB, &WiB, &Mupd, &flags);
  r = ensure(h, h->ws, c.off);
  if (r != SVLCOV_OK) return r;
  r = ensure(h, h->stage, csr_stage_bytes(E) + 256);
  if (r != SVLCOV_OK) return r;
  Carver c2{(char *)h->ws.p};
  layout(c2, &Cp64, &Cp32, &rown, &Gm, &Linv, &Kmat, &Mmat, &lam, &theta, &complete, &Fv, &Gv,
         &eigw, &Y, &T1, &WnA, &WiA, &WnB, &WiB, &Mupd, &flags);
  char *cursor = (char *)h->stage.p;
  DevCsr dE;
  r = to_device(h, E, cursor, &dE);
  if (r != SVLCOV_OK) return r;

  h->seq += 1;
  h->history.push_back({h->seq, h->m, h->n});
  hipStream_t st = h->stream;
  if (E->on_device && h->validate) {
    PhaseScope ps(h, PH_VALIDATE);
    svl::validate_csr(st, dE.rows, dE.cols, dE.nnz, dE.rp, dE.ci, dE.v, dE.vdt, h->info, h->seq);
  }
  svl::op_begin(st, h->info, 0);
  // the residual Gram's Cholesky and K beside the eigensolver where they can
  const bool overlap = side_stream(h, N, K);
  hipStream_t cst = overlap ? h->side : st;
  // orthogonalise the augmented matrix of the sparse side
  orthogonalise<T>(h, dE, B_base, W_B, Cp64, Cp32, rown, Gm, Linv, rid, 0, true, Kmat,
                   (size_t)N * N,    // K is formed only after the Gram
                   Mmat + (size_t)K * N + K, N, cst);
  // K = [[Sigma, 0], [E V, R^T]] and its Rayleigh-Ritz SVD
  {
    PhaseScope ps(h, PH_BUILDK, cst);
    svl::build_K_rows(cst, K, s, h->sigma, Cp64, Gm, s, Kmat, h->info);
  }
  if (overlap) (void)hipEventRecord(h->ev_join, cst);
  r = rayleigh_ritz(h, N, Kmat, Mmat, lam, theta, complete, Fv, Gv, eigw, orthw_p, Cp64,
                    overlap ? h->ev_join : nullptr, overlap ? orth2 : nullptr);
  if (r != SVLCOV_OK) return r;
  const int mode = mode_of(h->prec);
  if (overlap) {
    // sparse side: W_B (G[:k] - C_n G[k:]) and its inverse (enqueued first:
    // the longer chain)
    sparse_side_math(h, s, N, Gv, Cp64, Gm, Linv, W_B, Y, T1, WnB, WiB, flags + 1, sideB,
                     orthw_p + 2 * K * K + K * N, (size_t)8 * K * N, false);
    {
      PhaseScope ps(h, PH_SMALL);
      svl::inverse_cond_one(st, K, WnB, WiB, flags + 1, sideB, h->cond_reset, h->info);
    }
    // the append side (F's rows orthonormalised on the side stream already:
    // W_A F[:k], its inverse, the realisation on reset and the appended rows
    // F[k:] W^{-1}) stays there, beside the sparse side's triangular solve
    hipStream_t sd = h->side;
    {
      PhaseScope ps(h, PH_SMALL, sd);
      svl::gemm_f64(sd, false, true, K, K, K, 1.0, W_A, K, Fv, N, 0.0, WnA, K, h->info);
      svl::inverse_cond_one(sd, K, WnA, WiA, flags, sideA, h->cond_reset, h->info);
    }
    svl::check_finite(sd, K * K, WnA, h->info, h->seq);
    {
      PhaseScope ps(h, PH_COMMIT, sd);
      svl::realise<T, T>(sd, mode, K, nA, A_base, WnA, A_base, flags, h->info);
      svl::append_rows<T>(sd, K, s, Fv + K, 1, N, WiA, flags, A_base + nA * K, h->info);
    }
    (void)hipEventRecord(h->ev_join, sd);
    svl::check_finite(st, K * K, WnB, h->info, h->seq);
    (void)hipStreamWaitEvent(st, h->ev_join, 0);
    PhaseScope ps(h, PH_COMMIT);
    svl::commit_small(st, K, WnA, flags, W_A, theta, h->sigma, h->info, sideA);
  } else {
    // append side: W_A F[:k]; its inverse and condition
    {
      PhaseScope ps(h, PH_SMALL);
      svl::gemm_f64(st, false, true, K, K, K, 1.0, W_A, K, Fv, N, 0.0, WnA, K, h->info);
    }
    // sparse side: W_B (G[:k] - C_n G[k:]); then both inverses in one launch
    sparse_side_math(h, s, N, Gv, Cp64, Gm, Linv, W_B, Y, T1, WnB, WiB, flags + 1, sideB,
                     orthw_p + 2 * K * K + K * N, (size_t)8 * K * N, false);
    {
      PhaseScope ps(h, PH_SMALL);
      svl::inverse_cond_pair(st, K, WnA, WiA, flags, sideA, WnB, WiB, flags + 1, sideB,
                             h->cond_reset, h->info);
    }
    svl::check_finite(st, K * K, WnB, h->info, h->seq);
    svl::check_finite(st, K * K, WnA, h->info, h->seq);
    // commit: append side (realise on reset, appended rows F[k:] W^{-1})
    PhaseScope ps(h, PH_COMMIT);
    svl::realise<T, T>(st, mode, K, nA, A_base, WnA, A_base, flags, h->info);
    svl::append_rows<T>(st, K, s, Fv + K, 1, N, WiA, flags, A_base + nA * K, h->info);
    svl::commit_small(st, K, WnA, flags, W_A, theta, h->sigma, h->info, sideA);
  }
  // commit: sparse side
  sparse_side_commit<T>(h, dE, nB, B_base, Y, Mupd, WnB, WiB, flags + 1, W_B, nullptr, nullptr,
                        sideB, rid);
  svl::op_end(st, h->info);
  if (rows_form) h->m += s; else h->n += s;
  if (h->launch_failed) {
    h->launch_failed = false;
    return SVLCOV_E_DEVICE;
  }
  return SVLCOV_OK;
}

// The -GKL / -RPI variants of the row-append form (the appendix's variants
// with an approximate augmented space): the projection and the residual Gram
// G = Z^T Z are those of the exact path; an l-dimensional basis Q = Z Y of a
// Krylov (GKL) or power-iteration (RPI) subspace of range(Z) and P = Z^T Q
// replace the Cholesky factor, so K = [[Sigma, 0], [E V, P]] is (k+s) x (k+l)
// and its Rayleigh-Ritz SVD is taken through the eigenpairs of K^T K
// ((k+l) square): G from them, F = K G diag(theta)^{-1}.  The sparse side's
// rotation uses Y G[k:] where the exact path uses T G[k:].
// Drop floor of the variants' bases.  Their Gram is FP64 and their C' is
// accumulated in FP64 in every mode, so in the FP32 / BF16x3 modes the floor
// is set by the orthonormality of FP32-stored factors (~1e-7, a direction
// of the augmented space below ~1e-7 of the largest row is not resolved):
// 1e-12 on the squared scale, a GKL breakdown at 1e-6 of the largest row.
// The exact path's floor in those modes (the MFMA Gram's rounding, 1e-5)
// would end GKL after one step on a nearly flat spectrum (a selection D
// against a tall U), where every Krylov increment is small but genuine.
double approx_tol(const svlcov_state *h) {
  return h->prec == SVLCOV_FP64 ? h->rank_tol : std::min(h->rank_tol, 1e-12);
}

template <typename T>
svlcov_status op_append_approx(svlcov_state *h, const svlcov_csr *E, bool rows_form,
                               const svlcov_approx *ap) {
  svlcov_status r = check_csr_header(E);
  if (r != SVLCOV_OK) return r;
  if (!ap || (ap->method != SVLCOV_APPROX_GKL && ap->method != SVLCOV_APPROX_RPI) ||
      ap->l < 1 || ap->l > svl::AP_LMAX)
    return SVLCOV_E_INVALID;
  if (ap->method == SVLCOV_APPROX_RPI && (!ap->start || ap->t < 1 || ap->t > 16))
    return SVLCOV_E_INVALID;
  const int K = h->k;
  const int64_t s = E->rows;
  const int64_t nB = rows_form ? h->n : h->m;
  const int64_t nA = rows_form ? h->m : h->n;
  if (E->cols != nB) return SVLCOV_E_SHAPE;
  if (s == 0) return SVLCOV_OK;
  const int l = (int)(ap->l < s ? ap->l : s);
  const int64_t N = K + s, N2 = K + l;
  if (N2 > svl::eig_max_n() || s > svl::gram_max_rows()) return SVLCOV_E_UNSUPPORTED;
  if (!E->on_device) {
    r = check_host_csr(E);
    if (r != SVLCOV_OK) return r;
  }
  const bool gkl = ap->method == SVLCOV_APPROX_GKL;
  void **Abase = rows_form ? &h->Ubase : &h->Vbase;
  int64_t *Acap = rows_form ? &h->capU : &h->capV;
  r = grow_base(h, Abase, Acap, nA, nA + s);
  if (r != SVLCOV_OK) return r;
  T *A_base = (T *)*Abase;
  T *B_base = (T *)(rows_form ? h->Vbase : h->Ubase);
  double *W_A = rows_form ? h->WU : h->WV;
  double *W_B = rows_form ? h->WV : h->WU;
  const int sideA = rows_form ? 0 : 1, sideB = 1 - sideA;
  // a dense update's Gram goes through column blocks of up to 8192 columns
  const size_t dws_want = (size_t)s * (8192 + 1);
  const size_t dws_len =
      svl::gram_dense_block(s, E->cols, E->nnz, dws_want) > 0 ? dws_want : 1;
  struct Bufs {
    double *Cp64, *rown, *Gm, *Kmat, *Mmat, *lam, *theta, *Fv, *Gv, *eigw, *Y, *T1, *WnA, *WiA,
        *WnB, *WiB, *Mupd, *orthw, *Pv, *Yc, *gv, *ab, *Xl, *Tl, *Gm2, *Om, *Dws;
    float *Cp32;
    int32_t *complete, *flags, *rid, *brk;
  } b;
  auto layout = [&](Carver &cv) {
    b.Cp64 = cv.take<double>(s * K);
    b.Cp32 = cv.take<float>(s * K);
    b.rown = cv.take<double>(s);
    b.Gm = cv.take<double>(s * s);
    b.Kmat = cv.take<double>(N * N2);
    b.Mmat = cv.take<double>(N2 * N2);
    b.lam = cv.take<double>(K);
    b.theta = cv.take<double>(K);
    b.complete = cv.take<int32_t>(K);
    b.Fv = cv.take<double>(K * N);
    b.Gv = cv.take<double>(K * N2);
    b.eigw = cv.take<double>(svl::eig_work_doubles(N2, K));
    b.Y = cv.take<double>(s * K);
    b.T1 = cv.take<double>(K * K);
    b.WnA = cv.take<double>(K * K);
    b.WiA = cv.take<double>(K * K);
    b.WnB = cv.take<double>(K * K);
    b.WiB = cv.take<double>(K * K);
    b.Mupd = cv.take<double>(s * K);
    b.flags = cv.take<int32_t>(2);
    b.orthw = cv.take<double>(2 * K * K + 9 * K * N);
    b.rid = cv.take<int32_t>(rid_words(E->nnz));
    b.Pv = cv.take<double>((int64_t)(l + 1) * s);
    b.Yc = cv.take<double>((int64_t)l * s);
    b.gv = cv.take<double>(s);
    b.ab = cv.take<double>(2 * svl::AP_LMAX);
    b.brk = cv.take<int32_t>(1);
    b.Xl = cv.take<double>((int64_t)l * s);
    b.Tl = cv.take<double>((int64_t)l * s);
    b.Gm2 = cv.take<double>((int64_t)l * l);
    b.Om = cv.take<double>((int64_t)l * l);
    b.Dws = cv.take<double>(dws_len);
  };
  Carver c{nullptr};
  layout(c);
  r = ensure(h, h->ws, c.off);
  if (r != SVLCOV_OK) return r;
  r = ensure(h, h->stage, csr_stage_bytes(E) + 256);
  if (r != SVLCOV_OK) return r;
  Carver c2{(char *)h->ws.p};
  layout(c2);
  char *cursor = (char *)h->stage.p;
  DevCsr dE;
  r = to_device(h, E, cursor, &dE);
  if (r != SVLCOV_OK) return r;
  hipStream_t st = h->stream;
  // the start vectors: GKL's p_1 into gv (read once by the first step), RPI's
  // P_0 into the rows of Pv that the iteration overwrites
  if (ap->start) {
    const hipMemcpyKind kind = ap->start_on_device ? hipMemcpyDeviceToDevice
                                                   : hipMemcpyHostToDevice;
    double *dst = gkl ? b.gv : b.Pv;
    const size_t bytes = (size_t)(gkl ? s : (int64_t)l * s) * sizeof(double);
    if (!ap->start_on_device) {
      for (int64_t e = 0; e < (int64_t)(bytes / 8); ++e)
        if (!std::isfinite(ap->start[e])) return SVLCOV_E_NUMERIC;
    }
    SV_TRY(hipMemcpyAsync(dst, ap->start, bytes, kind, st));
  }

  h->seq += 1;
  h->history.push_back({h->seq, h->m, h->n});
  if (E->on_device && h->validate) {
    PhaseScope ps(h, PH_VALIDATE);
    svl::validate_csr(st, dE.rows, dE.cols, dE.nnz, dE.rp, dE.ci, dE.v, dE.vdt, h->info, h->seq);
  }
  svl::op_begin(st, h->info, 0);
  orthogonalise<T>(h, dE, B_base, W_B, b.Cp64, b.Cp32, b.rown, b.Gm, nullptr, b.rid, 0, false,
                   dws_len > 1 ? b.Dws : nullptr, dws_len > 1 ? dws_len : 0);
  double *gws = b.orthw + 2 * K * K + K * N;
  const size_t gws_len = (size_t)8 * K * N;
  {
    PhaseScope ps(h, PH_CHOL);   // the basis takes the Cholesky's place
    svl::sym_lower(st, s, b.Gm, s, h->info);
    if (gkl) {
      svl::gkl_basis(st, s, l, b.Gm, s, ap->start ? b.gv : nullptr, b.Pv, b.Yc, b.gv, b.ab,
                     b.brk, approx_tol(h), h->info);
    } else {
      svl::rpi_basis(st, s, l, ap->t, b.Gm, s, b.Pv, b.Yc, b.Xl, b.Tl, b.Gm2, b.Om, gws,
                     gws_len, approx_tol(h), h->info);
    }
  }
  {
    PhaseScope ps(h, PH_BUILDK);
    svl::build_K_approx(st, K, s, l, h->sigma, b.Cp64, b.Kmat, h->info);
    if (gkl)
      svl::gkl_pblock(st, s, l, b.Pv, b.ab, b.Kmat, N2, K, K, h->info);
    else
      svl::rows_to_block(st, s, l, b.Pv, b.Kmat, N2, K, K, h->info);
  }
  {
    PhaseScope ps(h, PH_KKT);
    svl::gemm_f64_sk(st, true, false, N2, N2, N, 1.0, b.Kmat, N2, b.Kmat, N2, 0.0, b.Mmat, N2,
                     gws, gws_len, h->info);
  }
  {
    PhaseScope ps(h, PH_TRIDIAG);
    coop_enter(h);
    const int trc = svl::eig_tridiag(st, N2, b.Mmat, b.eigw, h->flags, &h->epoch, h->info);
    coop_exit(h);
    if (trc != 0) {
      h->launch_failed = true;
      svl::set_status(st, h->info, SVLCOV_E_DEVICE);
    }
  }
  {
    PhaseScope ps(h, PH_BISECT);
    svl::eig_bisect(st, N2, K, b.lam, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_STEIN);
    svl::eig_stein(st, N2, K, b.lam, b.Gv, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_BACK);
    svl::eig_back(st, N2, K, b.Mmat, b.Gv, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_RECOVER);   // F = K G diag(theta)^{-1}
    svl::gemm_f64(st, false, true, K, N, N2, 1.0, b.Gv, N2, b.Kmat, N2, 0.0, b.Fv, N, h->info);
    svl::theta_scale(st, K, b.lam, b.theta, b.Fv, N, b.complete, h->info);
  }
  {
    PhaseScope ps(h, PH_ORTH);
    double *gram_kk = b.orthw, *linv_kk = b.orthw + K * K, *xtmp = b.orthw + 2 * K * K;
    svl::orthonormalize_rows(st, K, N, b.Fv, b.complete, (uint64_t)h->seq * 2 + 1, gram_kk,
                             linv_kk, xtmp, gws, gws_len, h->info);
    svl::orthonormalize_rows(st, K, N2, b.Gv, nullptr, (uint64_t)h->seq * 2 + 2, gram_kk,
                             linv_kk, xtmp, gws, gws_len, h->info);
    svl::check_finite(st, K, b.theta, h->info, h->seq);
  }
  {
    PhaseScope ps(h, PH_SMALL);
    svl::gemm_f64(st, false, true, K, K, K, 1.0, W_A, K, b.Fv, N, 0.0, b.WnA, K, h->info);
  }
  {
    PhaseScope ps(h, PH_TRSM);   // Y G[k:] in place of T G[k:]
    svl::gemm_f64(st, true, true, s, K, l, 1.0, b.Yc, s, b.Gv + K, N2, 0.0, b.Y, K, h->info);
  }
  sparse_side_small(h, s, N2, b.Gv, b.Cp64, W_B, b.Y, b.T1, b.WnB, b.WiB, b.flags + 1, sideB,
                    gws, gws_len, false);
  {
    PhaseScope ps(h, PH_SMALL);
    svl::inverse_cond_pair(st, K, b.WnA, b.WiA, b.flags, sideA, b.WnB, b.WiB, b.flags + 1,
                           sideB, h->cond_reset, h->info);
  }
  svl::check_finite(st, K * K, b.WnB, h->info, h->seq);
  svl::check_finite(st, K * K, b.WnA, h->info, h->seq);
  if (hipGetLastError() != hipSuccess) {
    h->launch_failed = true;
    svl::set_status(st, h->info, SVLCOV_E_DEVICE);
  }
  const int mode = mode_of(h->prec);
  {
    PhaseScope ps(h, PH_COMMIT);
    svl::realise<T, T>(st, mode, K, nA, A_base, b.WnA, A_base, b.flags, h->info);
    svl::append_rows<T>(st, K, s, b.Fv + K, 1, N, b.WiA, b.flags, A_base + nA * K, h->info);
    svl::commit_small(st, K, b.WnA, b.flags, W_A, b.theta, h->sigma, h->info, sideA);
  }
  sparse_side_commit<T>(h, dE, nB, B_base, b.Y, b.Mupd, b.WnB, b.WiB, b.flags + 1, W_B, nullptr,
                        nullptr, sideB, b.rid);
  svl::op_end(st, h->info);
  if (rows_form) h->m += s; else h->n += s;
  if (h->launch_failed) {
    h->launch_failed = false;
    return SVLCOV_E_DEVICE;
  }
  return SVLCOV_OK;
}

// The -GKL / -RPI variant of the weight form (the appendix's weight
// algorithm): one l-dimensional basis Q_D = Z_D Y_D^T of the augmented space
// of D against U and one Q_E of E_m against V, each in coefficient space on
// its residual Gram as in the append variants; K_w = [C_D; P_D^T] [C_E;
// P_E^T]^T + diag(Sigma, 0) of (k + l_D) x (k + l_E); SVD_k of K_w through
// K_w^T K_w; then both sides are updated as sparse sides with Y = Yc^T X[k:]
// in place of the Cholesky solve.
bool approx_ok(const svlcov_approx *ap) {
  if (!ap || (ap->method != SVLCOV_APPROX_GKL && ap->method != SVLCOV_APPROX_RPI) || ap->l < 1 ||
      ap->l > svl::AP_LMAX)
    return false;
  if (ap->method == SVLCOV_APPROX_RPI && (!ap->start || ap->t < 1 || ap->t > 16)) return false;
  return true;
}

template <typename T>
svlcov_status op_weights_approx(svlcov_state *h, const svlcov_csr *D, const svlcov_csr *Em,
                                const svlcov_approx *apD, const svlcov_approx *apE) {
  svlcov_status r = check_csr_header(D);
  if (r != SVLCOV_OK) return r;
  r = check_csr_header(Em);
  if (r != SVLCOV_OK) return r;
  if (!approx_ok(apD) || !approx_ok(apE)) return SVLCOV_E_INVALID;
  const int K = h->k;
  if (D->rows != Em->rows) return SVLCOV_E_SHAPE;
  if (D->cols != h->m || Em->cols != h->n) return SVLCOV_E_SHAPE;
  const int64_t s = D->rows;
  if (s == 0) return SVLCOV_OK;
  const svlcov_approx *ap[2] = {apD, apE};
  int lq[2];
  for (int q = 0; q < 2; ++q) lq[q] = (int)(ap[q]->l < s ? ap[q]->l : s);
  const int64_t ND = K + lq[0], NE = K + lq[1], N0 = K + s;
  if (ND > svl::eig_max_n() || NE > svl::eig_max_n() || s > svl::gram_max_rows())
    return SVLCOV_E_UNSUPPORTED;
  if (!D->on_device) { r = check_host_csr(D); if (r != SVLCOV_OK) return r; }
  if (!Em->on_device) { r = check_host_csr(Em); if (r != SVLCOV_OK) return r; }
  const svlcov_csr *Eq[2] = {D, Em};
  const size_t dws_want = (size_t)s * (8192 + 1);
  size_t dws_len = 1;
  for (int q = 0; q < 2; ++q)
    if (svl::gram_dense_block(s, Eq[q]->cols, Eq[q]->nnz, dws_want) > 0) dws_len = dws_want;
  const int64_t nnz_max = D->nnz > Em->nnz ? D->nnz : Em->nnz;
  struct Side {
    double *Cp64, *rown, *Gm, *Pv, *Yc, *gv, *ab, *Xl, *Tl, *Gm2, *Om, *XT, *Y, *M;
    float *Cp32;
    int32_t *brk;
  } sd[2];
  struct Shared {
    double *Kmat, *Mmat, *lam, *theta, *Fv, *Gv, *eigw, *T1, *WnU, *WiU, *WnV, *WiV, *orthw, *Dws;
    int32_t *complete, *flags, *rid;
  } b;
  auto layout = [&](Carver &cv) {
    for (int q = 0; q < 2; ++q) {
      const int l = lq[q];
      sd[q].Cp64 = cv.take<double>(s * K);
      sd[q].Cp32 = cv.take<float>(s * K);
      sd[q].rown = cv.take<double>(s);
      sd[q].Gm = cv.take<double>(s * s);
      sd[q].Pv = cv.take<double>((int64_t)(l + 1) * s);
      sd[q].Yc = cv.take<double>((int64_t)l * s);
      sd[q].gv = cv.take<double>(s);
      sd[q].ab = cv.take<double>(2 * svl::AP_LMAX);
      sd[q].brk = cv.take<int32_t>(1);
      sd[q].Xl = cv.take<double>((int64_t)l * s);
      sd[q].Tl = cv.take<double>((int64_t)l * s);
      sd[q].Gm2 = cv.take<double>((int64_t)l * l);
      sd[q].Om = cv.take<double>((int64_t)l * l);
      sd[q].XT = cv.take<double>(s * (K + l));
      sd[q].Y = cv.take<double>(s * K);
      sd[q].M = cv.take<double>(s * K);
    }
    b.Kmat = cv.take<double>(ND * NE);
    b.Mmat = cv.take<double>(NE * NE);
    b.lam = cv.take<double>(K);
    b.theta = cv.take<double>(K);
    b.complete = cv.take<int32_t>(K);
    b.Fv = cv.take<double>(K * ND);
    b.Gv = cv.take<double>(K * NE);
    b.eigw = cv.take<double>(svl::eig_work_doubles(NE, K));
    b.T1 = cv.take<double>(K * K);
    b.WnU = cv.take<double>(K * K);
    b.WiU = cv.take<double>(K * K);
    b.WnV = cv.take<double>(K * K);
    b.WiV = cv.take<double>(K * K);
    b.flags = cv.take<int32_t>(2);
    b.orthw = cv.take<double>(2 * K * K + 9 * K * N0);
    b.rid = cv.take<int32_t>(rid_words(nnz_max));
    b.Dws = cv.take<double>(dws_len);
  };
  Carver c{nullptr};
  layout(c);
  r = ensure(h, h->ws, c.off);
  if (r != SVLCOV_OK) return r;
  r = ensure(h, h->stage, csr_stage_bytes(D) + csr_stage_bytes(Em) + 512);
  if (r != SVLCOV_OK) return r;
  Carver c2{(char *)h->ws.p};
  layout(c2);
  char *cursor = (char *)h->stage.p;
  DevCsr dq[2];
  r = to_device(h, D, cursor, &dq[0]);
  if (r != SVLCOV_OK) return r;
  r = to_device(h, Em, cursor, &dq[1]);
  if (r != SVLCOV_OK) return r;
  hipStream_t st = h->stream;
  for (int q = 0; q < 2; ++q) {   // start vectors as in the append variants
    const svlcov_approx *a = ap[q];
    if (!a->start) continue;
    const bool gkl = a->method == SVLCOV_APPROX_GKL;
    const hipMemcpyKind kind = a->start_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    double *dst = gkl ? sd[q].gv : sd[q].Pv;
    const size_t bytes = (size_t)(gkl ? s : (int64_t)lq[q] * s) * sizeof(double);
    if (!a->start_on_device)
      for (int64_t e = 0; e < (int64_t)(bytes / 8); ++e)
        if (!std::isfinite(a->start[e])) return SVLCOV_E_NUMERIC;
    SV_TRY(hipMemcpyAsync(dst, a->start, bytes, kind, st));
  }

  h->seq += 1;
  h->history.push_back({h->seq, h->m, h->n});
  if (h->validate) {
    PhaseScope ps(h, PH_VALIDATE);
    for (int q = 0; q < 2; ++q)
      if (Eq[q]->on_device)
        svl::validate_csr(st, dq[q].rows, dq[q].cols, dq[q].nnz, dq[q].rp, dq[q].ci, dq[q].v,
                          dq[q].vdt, h->info, h->seq);
  }
  svl::op_begin(st, h->info, 1);
  T *Ub = (T *)h->Ubase, *Vb = (T *)h->Vbase;
  const T *baseq[2] = {Ub, Vb};
  const double *Wq[2] = {h->WU, h->WV};
  double *gws = b.orthw + 2 * K * K + K * N0;
  const size_t gws_len = (size_t)8 * K * N0;
  for (int q = 0; q < 2; ++q) {
    const int l = lq[q];
    orthogonalise<T>(h, dq[q], baseq[q], Wq[q], sd[q].Cp64, sd[q].Cp32, sd[q].rown, sd[q].Gm,
                     nullptr, b.rid, q, false, dws_len > 1 ? b.Dws : nullptr,
                     dws_len > 1 ? dws_len : 0);
    // the basis reads its drop scale from the first slot
    if (q == 1) svl::max_into(st, s, sd[q].rown, h->info, 0);
    PhaseScope ps(h, PH_CHOL);
    svl::sym_lower(st, s, sd[q].Gm, s, h->info);
    const bool gkl = ap[q]->method == SVLCOV_APPROX_GKL;
    if (gkl)
      svl::gkl_basis(st, s, l, sd[q].Gm, s, ap[q]->start ? sd[q].gv : nullptr, sd[q].Pv, sd[q].Yc,
                     sd[q].gv, sd[q].ab, sd[q].brk, approx_tol(h), h->info);
    else
      svl::rpi_basis(st, s, l, ap[q]->t, sd[q].Gm, s, sd[q].Pv, sd[q].Yc, sd[q].Xl, sd[q].Tl,
                     sd[q].Gm2, sd[q].Om, gws, gws_len, approx_tol(h), h->info);
    // XT = [C' | P] (s x (k + l)), P = Z^T Q
    svl::copy_strided(st, s, K, sd[q].Cp64, K, 1, sd[q].XT, K + l, h->info);
    if (gkl)
      svl::gkl_pblock(st, s, l, sd[q].Pv, sd[q].ab, sd[q].XT, K + l, 0, K, h->info);
    else
      svl::rows_to_block(st, s, l, sd[q].Pv, sd[q].XT, K + l, 0, K, h->info);
  }
  {
    PhaseScope ps(h, PH_BUILDK);   // K_w = XT_D^T XT_E + diag(Sigma, 0)
    svl::gemm_f64_sk(st, true, false, ND, NE, s, 1.0, sd[0].XT, ND, sd[1].XT, NE, 0.0, b.Kmat, NE,
                     gws, gws_len, h->info);
    svl::add_sigma_diag(st, K, h->sigma, b.Kmat, NE, h->info);
  }
  {
    PhaseScope ps(h, PH_KKT);
    svl::gemm_f64_sk(st, true, false, NE, NE, ND, 1.0, b.Kmat, NE, b.Kmat, NE, 0.0, b.Mmat, NE,
                     gws, gws_len, h->info);
  }
  {
    PhaseScope ps(h, PH_TRIDIAG);
    coop_enter(h);
    const int trc = svl::eig_tridiag(st, NE, b.Mmat, b.eigw, h->flags, &h->epoch, h->info);
    coop_exit(h);
    if (trc != 0) {
      h->launch_failed = true;
      svl::set_status(st, h->info, SVLCOV_E_DEVICE);
    }
  }
  {
    PhaseScope ps(h, PH_BISECT);
    svl::eig_bisect(st, NE, K, b.lam, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_STEIN);
    svl::eig_stein(st, NE, K, b.lam, b.Gv, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_BACK);
    svl::eig_back(st, NE, K, b.Mmat, b.Gv, b.eigw, h->info);
  }
  {
    PhaseScope ps(h, PH_RECOVER);   // F = K_w G diag(theta)^{-1}
    svl::gemm_f64(st, false, true, K, ND, NE, 1.0, b.Gv, NE, b.Kmat, NE, 0.0, b.Fv, ND, h->info);
    svl::theta_scale(st, K, b.lam, b.theta, b.Fv, ND, b.complete, h->info);
  }
  {
    PhaseScope ps(h, PH_ORTH);
    double *gram_kk = b.orthw, *linv_kk = b.orthw + K * K, *xtmp = b.orthw + 2 * K * K;
    svl::orthonormalize_rows(st, K, ND, b.Fv, b.complete, (uint64_t)h->seq * 2 + 1, gram_kk,
                             linv_kk, xtmp, gws, gws_len, h->info);
    svl::orthonormalize_rows(st, K, NE, b.Gv, nullptr, (uint64_t)h->seq * 2 + 2, gram_kk, linv_kk,
                             xtmp, gws, gws_len, h->info);
    svl::check_finite(st, K, b.theta, h->info, h->seq);
  }
  {
    PhaseScope ps(h, PH_TRSM);   // Y = Yc^T X[k:] on both sides
    svl::gemm_f64(st, true, true, s, K, lq[0], 1.0, sd[0].Yc, s, b.Fv + K, ND, 0.0, sd[0].Y, K,
                  h->info);
    svl::gemm_f64(st, true, true, s, K, lq[1], 1.0, sd[1].Yc, s, b.Gv + K, NE, 0.0, sd[1].Y, K,
                  h->info);
  }
  sparse_side_small(h, s, ND, b.Fv, sd[0].Cp64, h->WU, sd[0].Y, b.T1, b.WnU, b.WiU, b.flags, 0,
                    gws, gws_len, false);
  sparse_side_small(h, s, NE, b.Gv, sd[1].Cp64, h->WV, sd[1].Y, b.T1, b.WnV, b.WiV, b.flags + 1, 1,
                    gws, gws_len, false);
  {
    PhaseScope ps(h, PH_SMALL);
    svl::inverse_cond_pair(st, K, b.WnU, b.WiU, b.flags, 0, b.WnV, b.WiV, b.flags + 1, 1,
                           h->cond_reset, h->info);
  }
  svl::check_finite(st, K * K, b.WnU, h->info, h->seq);
  svl::check_finite(st, K * K, b.WnV, h->info, h->seq);
  if (hipGetLastError() != hipSuccess) {
    h->launch_failed = true;
    svl::set_status(st, h->info, SVLCOV_E_DEVICE);
  }
  sparse_side_commit<T>(h, dq[0], h->m, Ub, sd[0].Y, sd[0].M, b.WnU, b.WiU, b.flags, h->WU,
                        b.theta, h->sigma, 0, b.rid);
  sparse_side_commit<T>(h, dq[1], h->n, Vb, sd[1].Y, sd[1].M, b.WnV, b.WiV, b.flags + 1, h->WV,
                        nullptr, nullptr, 1, b.rid);
  svl::op_end(st, h->info);
  if (h->launch_failed) {
    h->launch_failed = false;
    return SVLCOV_E_DEVICE;
  }
  return SVLCOV_OK;
}

template <typename T>
svlcov_status op_weights(svlcov_state *h, const svlcov_csr *D, const svlcov_csr *Em) {
  svlcov_status r = check_csr_header(D);
  if (r != SVLCOV_OK) return r;
  r = check_csr_header(Em);
  if (r != SVLCOV_OK) return r;
  const int K = h->k;
  if (D->rows != Em->rows) return SVLCOV_E_SHAPE;
  if (D->cols != h->m || Em->cols != h->n) return SVLCOV_E_SHAPE;
  const int64_t s = D->rows;
  if (s == 0) return SVLCOV_OK;
  if (K + s > svl::eig_max_n()) return SVLCOV_E_UNSUPPORTED;
  if (!D->on_device) { r = check_host_csr(D); if (r != SVLCOV_OK) return r; }
  if (!Em->on_device) { r = check_host_csr(Em); if (r != SVLCOV_OK) return r; }
  const int64_t N = K + s;
  T *Ub = (T *)h->Ubase, *Vb = (T *)h->Vbase;
  double *orthw_p = nullptr;
  double **orthw = &orthw_p;
  int32_t *rid = nullptr;   // row id per nonzero of D^T, then of E_m^T (sparse Gram)
  const int64_t nnz_max = D->nnz > Em->nnz ? D->nnz : Em->nnz;
  auto layout = [&](Carver &cv, double **CpD, double **CpE, float **C32D, float **C32E,
                    double **rnD, double **rnE, double **GD, double **GE, double **LiD,
                    double **LiE, double **X, double **Yx, double **Kmat, double **Mmat,
                    double **lam, double **theta, int32_t **complete, double **Fv, double **Gv,
                    double **eigw, double **YD, double **YE, double **T1, double **WnU,
                    double **WiU, double **WnV, double **WiV, double **MD, double **ME,
                    int32_t **flags) {
    const size_t nbl = ((s + svl::CHOL_NB - 1) / svl::CHOL_NB) * svl::CHOL_NB * svl::CHOL_NB;
    *CpD = cv.take<double>(s * K); *CpE = cv.take<double>(s * K);
    *C32D = cv.take<float>(s * K); *C32E = cv.take<float>(s * K);
    *rnD = cv.take<double>(s); *rnE = cv.take<double>(s);
    *GD = cv.take<double>(s * s); *GE = cv.take<double>(s * s);
    *LiD = cv.take<double>(nbl); *LiE = cv.take<double>(nbl);
    *X = cv.take<double>(N * s); *Yx = cv.take<double>(N * s);
    *Kmat = cv.take<double>(N * N); *Mmat = cv.take<double>(N * N);
    *lam = cv.take<double>(K); *theta = cv.take<double>(K);
    *complete = cv.take<int32_t>(K);
    *Fv = cv.take<double>(K * N); *Gv = cv.take<double>(K * N);
    *eigw = cv.take<double>(svl::eig_update_work_doubles(N, K));
    *YD = cv.take<double>(s * K); *YE = cv.take<double>(s * K);
    *T1 = cv.take<double>(K * K);
    *WnU = cv.take<double>(K * K); *WiU = cv.take<double>(K * K);
    *WnV = cv.take<double>(K * K); *WiV = cv.take<double>(K * K);
    *MD = cv.take<double>(s * K); *ME = cv.take<double>(s * K);
    *flags = cv.take<int32_t>(2);
    *orthw = cv.take<double>(2 * K * K + 9 * K * N);
    rid = cv.take<int32_t>(rid_words(nnz_max));
  };
  double *CpD, *CpE, *rnD, *rnE, *GD, *GE, *LiD, *LiE, *X, *Yx, *Kmat, *Mmat, *lam, *theta, *Fv,
      *Gv, *eigw, *YD, *YE, *T1, *WnU, *WiU, *WnV, *WiV, *MD, *ME;
  float *C32D, *C32E;
  int32_t *complete, *flags;
  Carver c{nullptr};
  layout(c, &CpD, &CpE, &C32D, &C32E, &rnD, &rnE, &GD, &GE, &LiD, &LiE, &X, &Yx, &Kmat, &Mmat,
         &lam, &theta, &complete, &Fv, &Gv, &eigw, &YD, &YE, &T1, &WnU, &WiU, &WnV, &WiV, &MD,
         &ME, &flags);
  r = ensure(h, h->ws, c.off);
  if (r != SVLCOV_OK) return r;
  r = ensure(h, h->stage, csr_stage_bytes(D) + csr_stage_bytes(Em) + 512);
  if (r != SVLCOV_OK) return r;
  Carver c2{(char *)h->ws.p};
  layout(c2, &CpD, &CpE, &C32D, &C32E, &rnD, &rnE, &GD, &GE, &LiD, &LiE, &X, &Yx, &Kmat, &Mmat,
         &lam, &theta, &complete, &Fv, &Gv, &eigw, &YD, &YE, &T1, &WnU, &WiU, &WnV, &WiV, &MD,
         &ME, &flags);
  char *cursor = (char *)h->stage.p;
  DevCsr dD, dEm;
  r = to_device(h, D, cursor, &dD);
  if (r != SVLCOV_OK) return r;
  r = to_device(h, Em, cursor, &dEm);
  if (r != SVLCOV_OK) return r;

  h->seq += 1;
  h->history.push_back({h->seq, h->m, h->n});
  hipStream_t st = h->stream;
  if (h->validate) {
    PhaseScope ps(h, PH_VALIDATE);
    if (D->on_device)
      svl::validate_csr(st, dD.rows, dD.cols, dD.nnz, dD.rp, dD.ci, dD.v, dD.vdt, h->info, h->seq);
    if (Em->on_device)
      svl::validate_csr(st, dEm.rows, dEm.cols, dEm.nnz, dEm.rp, dEm.ci, dEm.v, dEm.vdt, h->info,
                        h->seq);
  }
  svl::op_begin(st, h->info, 1);
  orthogonalise<T>(h, dD, Ub, h->WU, CpD, C32D, rnD, GD, LiD, rid, 0, true, Kmat, (size_t)N * N);
  orthogonalise<T>(h, dEm, Vb, h->WV, CpE, C32E, rnE, GE, LiE, rid, 1, true, Kmat, (size_t)N * N);
  // K = [[Sigma, 0], [0, 0]] + [U^T D ; R_D] [V^T E_m ; R_E]^T
  {
    PhaseScope ps(h, PH_BUILDK);
    svl::build_X(st, K, s, CpD, GD, s, X, h->info);
    svl::build_X(st, K, s, CpE, GE, s, Yx, h->info);
    svl::gemm_f64(st, false, true, N, N, s, 1.0, X, s, Yx, s, 0.0, Kmat, N, h->info);
    svl::add_sigma_diag(st, K, h->sigma, Kmat, N, h->info);
  }
  r = rayleigh_ritz(h, N, Kmat, Mmat, lam, theta, complete, Fv, Gv, eigw, orthw_p);
  if (r != SVLCOV_OK) return r;
  sparse_side_math(h, s, N, Fv, CpD, GD, LiD, h->WU, YD, T1, WnU, WiU, flags, 0,
                   orthw_p + 2 * K * K + K * N, (size_t)8 * K * N, false);
  sparse_side_math(h, s, N, Gv, CpE, GE, LiE, h->WV, YE, T1, WnV, WiV, flags + 1, 1,
                   orthw_p + 2 * K * K + K * N, (size_t)8 * K * N, false);
  {
    PhaseScope ps(h, PH_SMALL);
    svl::inverse_cond_pair(st, K, WnU, WiU, flags, 0, WnV, WiV, flags + 1, 1, h->cond_reset,
                           h->info);
  }
  svl::check_finite(st, K * K, WnU, h->info, h->seq);
  svl::check_finite(st, K * K, WnV, h->info, h->seq);
  sparse_side_commit<T>(h, dD, h->m, Ub, YD, MD, WnU, WiU, flags, h->WU, theta, h->sigma, 0, rid);
  sparse_side_commit<T>(h, dEm, h->n, Vb, YE, ME, WnV, WiV, flags + 1, h->WV, nullptr, nullptr, 1,
                        rid);
  svl::op_end(st, h->info);
  if (h->launch_failed) {
    h->launch_failed = false;
    return SVLCOV_E_DEVICE;
  }
  return SVLCOV_OK;
}

svlcov_status read_info(svlcov_state *h, SvDevInfo *out) {
  SV_TRY(hipMemcpyAsync(out, h->info, sizeof(SvDevInfo), hipMemcpyDeviceToHost, h->stream));
  SV_TRY(hipStreamSynchronize(h->stream));
  return SVLCOV_OK;
}

// Wait, then turn a device-side failure into a return code and roll the host
// shape back to what it was before the failing update.
svlcov_status settle(svlcov_state *h) {
  SvDevInfo inf;
  svlcov_status r = read_info(h, &inf);
  if (r != SVLCOV_OK) return r;
  if (inf.status == 0) {
    h->history.clear();
    return SVLCOV_OK;
  }
  const svlcov_status code = (svlcov_status)inf.status;
  for (const Snapshot &sn : h->history) {
    if (sn.seq == inf.failed_seq || inf.failed_seq < 0) {
      h->m = sn.m;
      h->n = sn.n;
      break;
    }
  }
  h->history.clear();
  int32_t zero[2] = {0, 0};
  SV_TRY(hipMemcpyAsync(h->info, zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
  SV_TRY(hipStreamSynchronize(h->stream));
  return code;
}

}  // namespace

extern "C" {

void svlcov_default_options(svlcov_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SVLCOV_FP64;
  o->device = 0;
  o->stream = nullptr;
  o->rank_tol = 0.0;
  o->cond_reset = 0.0;
  o->validate_device_inputs = 1;
  o->deterministic = 1;
  o->side_stream = 1;
}

svlcov_status svlcov_init(svlcov_state **out, int64_t m, int64_t n, int32_t k, const double *U,
                          const double *sigma, const double *V, int32_t factors_on_device,
                          const svlcov_options *opt) {
  if (!out) return SVLCOV_E_INVALID;
  *out = nullptr;
  if (m < 0 || n < 0 || !sigma) return SVLCOV_E_INVALID;
  if (k != 16 && k != 32 && k != 64 && k != 128) return SVLCOV_E_UNSUPPORTED;
  if ((m > 0 && !U) || (n > 0 && !V)) return SVLCOV_E_INVALID;
  svlcov_options o;
  if (opt) o = *opt; else svlcov_default_options(&o);
  if (o.precision < 0 || o.precision > 2) return SVLCOV_E_INVALID;
  if (!factors_on_device) {
    for (int i = 0; i < k; ++i)
      if (!std::isfinite(sigma[i]) || sigma[i] < 0 || (i > 0 && sigma[i] > sigma[i - 1]))
        return SVLCOV_E_INVALID;
    if (!finite_vals(U, SVLCOV_F64, m * k) || !finite_vals(V, SVLCOV_F64, n * k))
      return SVLCOV_E_NUMERIC;
  }
  if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) return SVLCOV_E_INVALID;
  svlcov_state *h = new (std::nothrow) svlcov_state();
  if (!h) return SVLCOV_E_NOMEM;
  h->dev_alloc = o.dev_alloc;
  h->dev_free = o.dev_free;
  h->alloc_ctx = o.alloc_ctx;
  h->device = o.device;
  h->prec = o.precision;
  h->k = k;
  h->m = m;
  h->n = n;
  h->rank_tol = o.rank_tol > 0 ? o.rank_tol : DEF_TOL[h->prec];
  h->cond_reset = o.cond_reset > 0 ? o.cond_reset : DEF_COND[h->prec];
  h->validate = o.validate_device_inputs ? 1 : 0;
  h->deterministic = o.deterministic ? 1 : 0;
  h->side_ok = o.side_stream ? 1 : 0;
  auto fail = [&](svlcov_status s) {
    svlcov_destroy(h);
    return s;
  };
  if (hipSetDevice(h->device) != hipSuccess) return fail(SVLCOV_E_DEVICE);
  if (o.stream) {
    h->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
      return fail(SVLCOV_E_DEVICE);
    h->own_stream = true;
  }
  h->capU = o.row_capacity > m ? o.row_capacity : m + m / 4 + 1024;
  h->capV = o.col_capacity > n ? o.col_capacity : n + n / 4 + 1024;
  const size_t es = h->elem();
  using svl_state::state_alloc;
  if (state_alloc(h, &h->Ubase, (size_t)h->capU * k * es) != hipSuccess)
    return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, &h->Vbase, (size_t)h->capV * k * es) != hipSuccess)
    return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, (void **)&h->WU, (size_t)k * k * 8) != hipSuccess) return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, (void **)&h->WV, (size_t)k * k * 8) != hipSuccess) return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, (void **)&h->sigma, (size_t)k * 8) != hipSuccess) return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, (void **)&h->info, sizeof(SvDevInfo)) != hipSuccess)
    return fail(SVLCOV_E_NOMEM);
  if (state_alloc(h, (void **)&h->flags, svl::TRI_FLAG_WORDS * sizeof(unsigned)) != hipSuccess)
    return fail(SVLCOV_E_NOMEM);
  if (hipMemsetAsync(h->flags, 0, svl::TRI_FLAG_WORDS * sizeof(unsigned), h->stream) !=
      hipSuccess)
    return fail(SVLCOV_E_DEVICE);
  SvDevInfo zi;
  std::memset(&zi, 0, sizeof(zi));
  zi.rank2 = -1;
  zi.max_dropped = -1.0;
  hipMemcpyKind kind = factors_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (hipMemcpyAsync(h->info, &zi, sizeof(zi), hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(SVLCOV_E_DEVICE);
  if (hipMemcpyAsync(h->sigma, sigma, (size_t)k * 8, kind, h->stream) != hipSuccess)
    return fail(SVLCOV_E_DEVICE);
  svl::fill_identity(h->stream, k, h->WU);
  svl::fill_identity(h->stream, k, h->WV);
  // U', V' start as the given singular vectors (converted to the storage type)
  for (int side = 0; side < 2; ++side) {
    const int64_t rows = side == 0 ? m : n;
    const double *src = side == 0 ? U : V;
    void *dst = side == 0 ? h->Ubase : h->Vbase;
    if (rows == 0) continue;
    if (h->prec == SVLCOV_FP64) {
      if (hipMemcpyAsync(dst, src, (size_t)rows * k * 8, kind, h->stream) != hipSuccess)
        return fail(SVLCOV_E_DEVICE);
    } else {
      const double *dsrc = src;
      double *tmp = nullptr;
      if (!factors_on_device) {
        if (state_alloc(h, (void **)&tmp, (size_t)rows * k * 8) != hipSuccess)
          return fail(SVLCOV_E_NOMEM);
        if (hipMemcpyAsync(tmp, src, (size_t)rows * k * 8, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
          return fail(SVLCOV_E_DEVICE);
        dsrc = tmp;
      }
      // identity W: the realisation kernel doubles as a converting copy
      svl::realise<double, float>(h->stream, 0, k, rows, dsrc, h->WU, (float *)dst, nullptr,
                                  nullptr);
      svl_state::state_free(h, tmp, (size_t)rows * k * 8);
    }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(SVLCOV_E_DEVICE);
  *out = h;
  return SVLCOV_OK;
}

svlcov_status svlcov_add_rows(svlcov_state *h, const svlcov_csr *E) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r = h->prec == SVLCOV_FP64 ? op_append<double>(h, E, true) : op_append<float>(h, E, true);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_add_cols(svlcov_state *h, const svlcov_csr *E) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r = h->prec == SVLCOV_FP64 ? op_append<double>(h, E, false) : op_append<float>(h, E, false);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_add_rows_approx(svlcov_state *h, const svlcov_csr *E, const svlcov_approx *a) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r = h->prec == SVLCOV_FP64 ? op_append_approx<double>(h, E, true, a)
                                                 : op_append_approx<float>(h, E, true, a);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_add_cols_approx(svlcov_state *h, const svlcov_csr *E, const svlcov_approx *a) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r = h->prec == SVLCOV_FP64 ? op_append_approx<double>(h, E, false, a)
                                                 : op_append_approx<float>(h, E, false, a);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_update_weights_approx(svlcov_state *h, const svlcov_csr *D_T,
                                           const svlcov_csr *E_m_T, const svlcov_approx *a_D,
                                           const svlcov_approx *a_E) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r =
      h->prec == SVLCOV_FP64 ? op_weights_approx<double>(h, D_T, E_m_T, a_D, a_E)
                             : op_weights_approx<float>(h, D_T, E_m_T, a_D, a_E);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_update_weights(svlcov_state *h, const svlcov_csr *D, const svlcov_csr *Em) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const svlcov_status r = h->prec == SVLCOV_FP64 ? op_weights<double>(h, D, Em) : op_weights<float>(h, D, Em);
  h->proj_ready[0] = h->proj_ready[1] = false;
  return r;
}

svlcov_status svlcov_sync(svlcov_state *h) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  return settle(h);
}

svlcov_status svlcov_get_factors(svlcov_state *h, int64_t *m, int64_t *n, int32_t *k,
                                 int32_t out_dtype, int32_t out_on_device, void *U, double *sigma,
                                 void *V) {
  if (!h) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  svlcov_status r = settle(h);
  if (r != SVLCOV_OK) return r;
  if (m) *m = h->m;
  if (n) *n = h->n;
  if (k) *k = h->k;
  const int K = h->k;
  const size_t osz = out_dtype == SVLCOV_F64 ? 8 : 4;
  hipStream_t st = h->stream;
  for (int side = 0; side < 2; ++side) {
    void *dst = side == 0 ? U : V;
    if (!dst) continue;
    const int64_t rows = side == 0 ? h->m : h->n;
    if (rows == 0) continue;
    const double *W = side == 0 ? h->WU : h->WV;
    const void *base = side == 0 ? h->Ubase : h->Vbase;
    void *target = dst;
    if (!out_on_device) {
      r = ensure(h, h->outbuf, (size_t)rows * K * osz);
      if (r != SVLCOV_OK) return r;
      target = h->outbuf.p;
    }
    if (h->prec == SVLCOV_FP64) {
      if (out_dtype == SVLCOV_F64)
        svl::realise<double, double>(st, 0, K, rows, (const double *)base, W, (double *)target,
                                     nullptr, nullptr);
      else
        svl::realise<double, float>(st, 0, K, rows, (const double *)base, W, (float *)target,
                                    nullptr, nullptr);
    } else {
      if (out_dtype == SVLCOV_F64)
        svl::realise<float, double>(st, 0, K, rows, (const float *)base, W, (double *)target,
                                    nullptr, nullptr);
      else
        svl::realise<float, float>(st, 0, K, rows, (const float *)base, W, (float *)target,
                                   nullptr, nullptr);
    }
    if (!out_on_device)
      SV_TRY(hipMemcpyAsync(dst, target, (size_t)rows * K * osz, hipMemcpyDeviceToHost, st));
  }
  if (sigma) SV_TRY(hipMemcpyAsync(sigma, h->sigma, (size_t)K * 8, hipMemcpyDeviceToHost, st));
  SV_TRY(hipStreamSynchronize(st));
  return SVLCOV_OK;
}

svlcov_status svlcov_query_row(svlcov_state *h, int32_t side, int64_t i, double *out_k) {
  if (!h || !out_k || (side != 0 && side != 1)) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  svlcov_status r = settle(h);
  if (r != SVLCOV_OK) return r;
  const int64_t rows = side == 0 ? h->m : h->n;
  if (i < 0 || i >= rows) return SVLCOV_E_SHAPE;
  const int K = h->k;
  r = ensure(h, h->outbuf, (size_t)K * 8);
  if (r != SVLCOV_OK) return r;
  const double *W = side == 0 ? h->WU : h->WV;
  const void *base = side == 0 ? h->Ubase : h->Vbase;
  if (h->prec == SVLCOV_FP64)
    svl::realise<double, double>(h->stream, 0, K, 1, (const double *)base + i * K, W,
                                 (double *)h->outbuf.p, nullptr, nullptr);
  else
    svl::realise<float, double>(h->stream, 0, K, 1, (const float *)base + i * K, W,
                                (double *)h->outbuf.p, nullptr, nullptr);
  SV_TRY(hipMemcpyAsync(out_k, h->outbuf.p, (size_t)K * 8, hipMemcpyDeviceToHost, h->stream));
  SV_TRY(hipStreamSynchronize(h->stream));
  return SVLCOV_OK;
}

svlcov_status svlcov_query_rows(svlcov_state *h, int32_t side, int64_t n, const int64_t *idx,
                                double *out) {
  if (!h || (side != 0 && side != 1) || n < 0 || (n > 0 && (!idx || !out)))
    return SVLCOV_E_INVALID;
  if (n == 0) return SVLCOV_OK;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const int64_t rows = side == 0 ? h->m : h->n;
  const double *W = side == 0 ? h->WU : h->WV;
  const void *base = side == 0 ? h->Ubase : h->Vbase;
  if (h->prec == SVLCOV_FP64)
    svl::query_rows<double>(h->stream, h->k, n, idx, rows, (const double *)base, W, out);
  else
    svl::query_rows<float>(h->stream, h->k, n, idx, rows, (const float *)base, W, out);
  return hipGetLastError() == hipSuccess ? SVLCOV_OK : SVLCOV_E_DEVICE;
}

svlcov_status svlcov_score_pairs(svlcov_state *h, int64_t n, const int64_t *i, const int64_t *j,
                                 int32_t both, double *out, float *kernel_ms) {
  if (!h || n < 0 || (both != 0 && both != 1) || (n > 0 && (!i || !j || !out)))
    return SVLCOV_E_INVALID;
  if (n == 0) return SVLCOV_OK;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  const int K = h->k;
  const bool f64 = h->prec == SVLCOV_FP64;
  const size_t elem = f64 ? 8 : 4;
  hipStream_t st = h->stream;
  if (h->q_seq != h->seq || h->qU.bytes < (size_t)h->m * K * elem ||
      h->qV.bytes < (size_t)h->n * K * elem) {
    // realise U_base (W_U Sigma) and V_base W_V once per factor version
    svlcov_status r = ensure(h, h->qU, (size_t)h->m * K * elem);
    if (r != SVLCOV_OK) return r;
    r = ensure(h, h->qV, (size_t)h->n * K * elem);
    if (r != SVLCOV_OK) return r;
    r = ensure(h, h->qW, (size_t)K * K * 8);
    if (r != SVLCOV_OK) return r;
    svl::scale_cols(st, K, h->WU, h->sigma, (double *)h->qW.p);
    const int mode = f64 ? 0 : 1;   // FP32 MFMA for FP32 storage (no BF16 split here)
    if (f64) {
      svl::realise<double, double>(st, mode, K, h->m, (const double *)h->Ubase,
                                   (const double *)h->qW.p, (double *)h->qU.p, nullptr, nullptr);
      svl::realise<double, double>(st, mode, K, h->n, (const double *)h->Vbase, h->WV,
                                   (double *)h->qV.p, nullptr, nullptr);
    } else {
      svl::realise<float, float>(st, mode, K, h->m, (const float *)h->Ubase,
                                 (const double *)h->qW.p, (float *)h->qU.p, nullptr, nullptr);
      svl::realise<float, float>(st, mode, K, h->n, (const float *)h->Vbase, h->WV,
                                 (float *)h->qV.p, nullptr, nullptr);
    }
    h->q_seq = h->seq;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    return SVLCOV_E_DEVICE;
  if (e0) SV_TRY(hipEventRecord(e0, st));
  if (f64)
    svl::score_pairs<double>(st, K, n, i, j, both, h->m, h->n, (const double *)h->qU.p,
                             (const double *)h->qV.p, out);
  else
    svl::score_pairs<float>(st, K, n, i, j, both, h->m, h->n, (const float *)h->qU.p,
                            (const float *)h->qV.p, out);
  const hipError_t le = hipGetLastError();
  if (e1) {
    SV_TRY(hipEventRecord(e1, st));
    SV_TRY(hipEventSynchronize(e1));
    if (hipEventElapsedTime(kernel_ms, e0, e1) != hipSuccess) *kernel_ms = -1.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return le == hipSuccess ? SVLCOV_OK : SVLCOV_E_DEVICE;
}

svlcov_status svlcov_get_stats(svlcov_state *h, svlcov_stats *out) {
  if (!h || !out) return SVLCOV_E_INVALID;
  BusyGuard g(h);
  if (!g.ok) return SVLCOV_E_BUSY;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  SvDevInfo inf;
  svlcov_status r = read_info(h, &inf);
  if (r != SVLCOV_OK) return r;
  out->updates = inf.updates;
  out->resets_U = inf.resets_U;
  out->resets_V = inf.resets_V;
  out->last_rank = inf.rank;
  out->last_rank2 = inf.rank2;
  out->last_kappa_U = inf.kappa_U;
  out->last_kappa_V = inf.kappa_V;
  out->last_min_kept_pivot = inf.min_kept;
  out->last_max_dropped_pivot = inf.max_dropped;
  out->iter_runs = h->iter_runs;
  out->iter_steps = h->iter_steps;
  out->iter_fallbacks = h->iter_fallbacks;
  out->iter_flops = h->iter_flops;
  return SVLCOV_OK;
}

void *svlcov_stream(svlcov_state *h) { return h ? (void *)h->stream : nullptr; }

svlcov_status svlcov_profile(svlcov_state *h, int32_t enable) {
  if (!h) return SVLCOV_E_INVALID;
  h->prof = enable != 0;
  h->prof_mask = ~0u;
  return SVLCOV_OK;
}

svlcov_status svlcov_profile_phases(svlcov_state *h, uint32_t mask) {
  if (!h) return SVLCOV_E_INVALID;
  if (mask >> SVLCOV_NUM_PHASES) return SVLCOV_E_INVALID;
  h->prof = mask != 0;
  h->prof_mask = mask;
  return SVLCOV_OK;
}

svlcov_status svlcov_phase_times(svlcov_state *h, double *ms, int64_t *count, int32_t n) {
  if (!h || n < 0) return SVLCOV_E_INVALID;
  if (hipSetDevice(h->device) != hipSuccess) return SVLCOV_E_DEVICE;
  SV_TRY(hipStreamSynchronize(h->stream));
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = 0.0;
    if (count) count[i] = 0;
  }
  for (const EvRec &r : h->recs) {
    float t = 0.f;
    SV_TRY(hipEventElapsedTime(&t, r.a, r.b));
    if (r.ph < n) {
      if (ms) ms[r.ph] += t;
      if (count) count[r.ph] += 1;
    }
    h->evpool.push_back(r.a);
    h->evpool.push_back(r.b);
  }
  h->recs.clear();
  return SVLCOV_OK;
}

const char *svlcov_phase_name(int32_t i) {
  return (i >= 0 && i < PH_COUNT) ? PHASE_NAMES[i] : "";
}

void svlcov_destroy(svlcov_state *h) {
  if (!h) return;
  // a state attached to a request server belongs to it until the server is
  // destroyed: the server's worker may be dispatching its update right now
  if (h->coop_chain) return;
  // a call in flight on another thread finishes first
  for (bool expected = false; !h->busy.compare_exchange_weak(expected, true); expected = false)
    std::this_thread::yield();
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  using svl_state::release;
  using svl_state::state_free;
  release(h, h->ws);
  release(h, h->stage);
  release(h, h->outbuf);
  release(h, h->qU);
  release(h, h->qV);
  release(h, h->qW);
  const size_t es = h->elem();
  state_free(h, h->Ubase, (size_t)h->capU * h->k * es);
  state_free(h, h->Vbase, (size_t)h->capV * h->k * es);
  state_free(h, h->WU, (size_t)h->k * h->k * 8);
  state_free(h, h->WV, (size_t)h->k * h->k * 8);
  state_free(h, h->sigma, (size_t)h->k * 8);
  state_free(h, h->info, sizeof(SvDevInfo));
  state_free(h, h->flags, svl::TRI_FLAG_WORDS * sizeof(unsigned));
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (const EvRec &r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  delete h;
}

svlcov_status svlcov_project_batch(int32_t n, svlcov_state *const *states, const int32_t *sides,
                                   const svlcov_csr *E, double *const *out, double *const *rown,
                                   void *stream, float *kernel_ms) {
  if (n <= 0 || n > 65536 || !states || !sides || !E || !out) return SVLCOV_E_INVALID;
  const int dev = states[0] ? states[0]->device : 0;
  std::vector<svl::ProjDesc> d((size_t)n);
  int64_t rown_need = 0;
  for (int32_t q = 0; q < n; ++q) {
    svlcov_state *h = states[q];
    if (!h || h->device != dev || (sides[q] != 0 && sides[q] != 1) || !out[q])
      return SVLCOV_E_INVALID;
    svlcov_status r = check_csr_header(&E[q]);
    if (r != SVLCOV_OK) return r;
    if (!E[q].on_device) return SVLCOV_E_INVALID;
    if (E[q].cols != (sides[q] == 0 ? h->m : h->n)) return SVLCOV_E_SHAPE;
    svl::ProjDesc &x = d[(size_t)q];
    x.row_ptr = E[q].row_ptr;
    x.col_idx = E[q].col_idx;
    x.val = E[q].val;
    x.base = sides[q] == 0 ? h->Ubase : h->Vbase;
    x.W = sides[q] == 0 ? h->WU : h->WV;
    x.Cp64 = out[q];
    x.Cp32 = nullptr;
    x.rown = rown ? rown[q] : nullptr;
    x.info = h->info;
    x.s = E[q].rows;
    x.row0 = 0;
    x.nnz = E[q].nnz;
    x.vdtype = E[q].val_dtype;
    x.K = h->k;
    x.fp64 = h->prec == SVLCOV_FP64 ? 1 : 0;
    x.pad = 0;
    if (!x.rown) rown_need += E[q].rows;
  }
  if (hipSetDevice(dev) != hipSuccess) return SVLCOV_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  double *scratch = nullptr;
  if (rown_need > 0) SV_TRY(hipMallocAsync((void **)&scratch, (size_t)rown_need * 8, st));
  int64_t off = 0;
  for (svl::ProjDesc &x : d)
    if (!x.rown) { x.rown = scratch + off; off += x.s; }
  const svl::ProjBatch pb = svl::spmm_batch_prepare(std::move(d));
  std::vector<char> blob(pb.bytes());
  pb.pack(blob.data());
  void *dd = nullptr;
  SV_TRY(hipMallocAsync(&dd, blob.size(), st));
  SV_TRY(hipMemcpyAsync(dd, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    return SVLCOV_E_DEVICE;
  if (e0) SV_TRY(hipEventRecord(e0, st));
  svl::spmm_batch(st, pb, dd);
  const hipError_t le = hipGetLastError();
  if (e1) SV_TRY(hipEventRecord(e1, st));
  (void)hipFreeAsync(dd, st);
  if (scratch) (void)hipFreeAsync(scratch, st);
  SV_TRY(hipStreamSynchronize(st));   // the host blob must outlive the copy
  if (e0 && e1) {
    if (hipEventElapsedTime(kernel_ms, e0, e1) != hipSuccess) *kernel_ms = -1.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return le == hipSuccess ? SVLCOV_OK : SVLCOV_E_DEVICE;
}

int32_t svlcov_spmm_variant_count(void) { return svl::spmm_variant_count(); }

svlcov_status svlcov_spmm_variant_shape(int32_t v, int32_t *loads_in_flight,
                                        int32_t *rows_per_tile) {
  int u = 0, rb = 0;
  if (!loads_in_flight || !rows_per_tile || !svl::spmm_variant_shape(v, &u, &rb))
    return SVLCOV_E_INVALID;
  *loads_in_flight = u;
  *rows_per_tile = rb;
  return SVLCOV_OK;
}

svlcov_status svlcov_spmm_tune_set(int32_t fp64, int32_t k, int32_t row_bin, int32_t variant) {
  return svl::spmm_tune_set(fp64, k, row_bin, variant) ? SVLCOV_OK : SVLCOV_E_INVALID;
}

svlcov_status svlcov_spmm_tune_get(int32_t fp64, int32_t k, int32_t row_bin, int32_t *variant) {
  if (!variant) return SVLCOV_E_INVALID;
  const int v = svl::spmm_tune_get(fp64, k, row_bin);
  if (v < 0) return SVLCOV_E_INVALID;
  *variant = v;
  return SVLCOV_OK;
}

svlcov_status svlcov_sym_eig_topk(int64_t N, const double *M, int32_t k, double *lam,
                                  double *vecs, void *stream) {
  if (N < 1 || k < 1 || k > N || !M || !lam || !vecs) return SVLCOV_E_INVALID;
  if (N > svl::eig_max_n() || k > 128) return SVLCOV_E_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const size_t wd = svl::eig_work_doubles(N, k);
  char *mem = nullptr;
  const size_t bytes = ((size_t)N * N + wd) * sizeof(double) + sizeof(SvDevInfo) +
                       svl::TRI_FLAG_WORDS * sizeof(unsigned) + 1024;
  SV_TRY(hipMallocAsync((void **)&mem, bytes, st));
  double *A = (double *)mem;
  double *work = A + (size_t)N * N;
  SvDevInfo *info = (SvDevInfo *)(work + wd);
  unsigned *flags = (unsigned *)(info + 1);
  SV_TRY(hipMemsetAsync(info, 0, sizeof(SvDevInfo) + svl::TRI_FLAG_WORDS * sizeof(unsigned), st));
  SV_TRY(hipMemcpyAsync(A, M, (size_t)N * N * sizeof(double), hipMemcpyDeviceToDevice, st));
  unsigned epoch = 0;
  const int r = svl::eig_topk(st, N, A, k, lam, vecs, work, flags, &epoch, info);
  SV_TRY(hipFreeAsync(mem, st));
  return r == 0 ? SVLCOV_OK : SVLCOV_E_DEVICE;
}

}  // extern "C"

// Workspace of svlcov_sym_eig_topk_noalloc: one fixed array per GPU, held
// until the process ends.  In host code `scratch` names a host-side stand-in;
// the device address of each GPU's copy is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.
namespace {
constexpr size_t EIG_SCRATCH_BYTES = (size_t)SVLCOV_EIG_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[EIG_SCRATCH_BYTES / sizeof(double)];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES];   // per device, null until looked up

size_t eig_scratch_need(int64_t N, int32_t k) {
  const size_t wd = svl::eig_work_doubles(N, k);
  return ((size_t)N * N + wd) * sizeof(double) + 256 + sizeof(SvDevInfo) +
         svl::TRI_FLAG_WORDS * sizeof(unsigned);
}
}  // namespace

extern "C" {

svlcov_status svlcov_sym_eig_topk_noalloc(int64_t N, const double *M, int32_t k, double *lam,
                                          double *vecs, void *stream) {
  if (N < 1 || k < 1 || k > N || !M || !lam || !vecs) return SVLCOV_E_INVALID;
  if (N > svl::eig_max_n() || k > 128) return SVLCOV_E_UNSUPPORTED;
  if (eig_scratch_need(N, k) > EIG_SCRATCH_BYTES) return SVLCOV_E_UNSUPPORTED;
  int dev = 0;
  SV_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return SVLCOV_E_UNSUPPORTED;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
      void *p = nullptr;
      SV_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p) return SVLCOV_E_DEVICE;
      scratch_dev[dev] = p;
    }
    base = scratch_dev[dev];
  }
  hipStream_t st = (hipStream_t)stream;
  double *A = (double *)base;
  double *work = A + (size_t)N * N;
  const size_t wd = svl::eig_work_doubles(N, k);
  SvDevInfo *info = (SvDevInfo *)(((uintptr_t)(work + wd) + 255) & ~(uintptr_t)255);
  unsigned *flags = (unsigned *)(info + 1);
  // status word and barrier flags start at zero on every call (a fill kernel,
  // not a memset node, so that a captured graph replays it faithfully)
  svl::zero_words(st, (unsigned *)info,
                  sizeof(SvDevInfo) / sizeof(unsigned) + svl::TRI_FLAG_WORDS);
  svl::copy_strided(st, N, N, M, N, 1, A, N, info);
  unsigned epoch = 0;
  const int r = svl::eig_topk(st, N, A, k, lam, vecs, work, flags, &epoch, info);
  if (r != 0) return SVLCOV_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SVLCOV_OK : SVLCOV_E_DEVICE;
}

const char *svlcov_status_str(svlcov_status s) {
  switch (s) {
    case SVLCOV_OK: return "ok";
    case SVLCOV_E_INVALID: return "invalid argument";
    case SVLCOV_E_SHAPE: return "shape mismatch";
    case SVLCOV_E_NOMEM: return "out of device memory";
    case SVLCOV_E_NUMERIC: return "non-finite value";
    case SVLCOV_E_DEVICE: return "HIP runtime error";
    case SVLCOV_E_BUSY: return "state busy";
    case SVLCOV_E_UNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

}  // extern "C"
