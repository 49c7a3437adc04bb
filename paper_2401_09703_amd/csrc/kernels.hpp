// Host-side launchers of the gfx950 kernels (all enqueue on the given stream).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

namespace svl {

// ---- sparse (k_sparse.hip)
void validate_csr(hipStream_t st, int64_t rows, int64_t cols, int64_t nnz,
                  const int64_t *rp, const int32_t *ci, const void *v, int vdt,
                  SvDevInfo *info, int seq);
// C' = E base W (FP64 out, FP32 copy when Cp32) and the row norms of E;
// accumulated in the storage type, or in FP64 when acc64.
template <typename T>
void spmm_w(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
            const void *v, int vdt, const T *base, const double *W, double *Cp64,
            float *Cp32, double *rownorm2, const SvDevInfo *info, bool acc64 = false);
// One projection of a fused batch (k_spmm_batch): C' = E base W and the row
// norms of E for s rows; row0 is the offset of its first tile (tiles of
// spmm_batch_rows_per_block() rows) within its group.
struct ProjDesc {
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *val;
  const void *base;
  const double *W;
  double *Cp64;
  float *Cp32;
  double *rown;
  const SvDevInfo *info;
  int64_t s, row0;
  int64_t nnz;   // nonzeros of E (host-side balance and tile-shape choice)
  int32_t vdtype, K, fp64, pad;   // pad: the tile-shape variant (set by prepare)
};
// A fused batch as uploaded: the descriptors ordered by (storage type, rank),
// one group per launch, followed by each group's block-to-tile table (-1 marks
// an idle block).  The table keeps the tiles of one update on one XCD where
// the load balance allows it, so the rows of its base are gathered through
// one L2 instead of all eight.
struct ProjBatch {
  std::vector<ProjDesc> d;
  std::vector<int32_t> order;
  std::vector<size_t> g_desc, g_order;   // group starts in d and order, plus the ends
  size_t bytes() const { return d.size() * sizeof(ProjDesc) + order.size() * sizeof(int32_t); }
  void pack(void *host) const;
};
int spmm_batch_rows_per_block();
// Tile shapes of the fused projection and the process-wide tuning table:
// variant per (FP64 storage, rank, bin of nonzeros per row).
constexpr int PB_ROW_BINS = 4;   // < 16, < 64, < 256, >= 256 nonzeros per row
int spmm_variant_count();
bool spmm_variant_shape(int v, int *loads_in_flight, int *rows_per_tile);
int spmm_row_bin(int64_t nnz, int64_t s);
bool spmm_tune_set(int fp64, int K, int bin, int v);
int spmm_tune_get(int fp64, int K, int bin);   // -1 for a bad key
ProjBatch spmm_batch_prepare(std::vector<ProjDesc> d);
// blob_dev holds pack()'s bytes (device memory).
void spmm_batch(hipStream_t st, const ProjBatch &b, const void *blob_dev);
// S = E E^T; rid receives the row id of every nonzero (nnz int32 scratch).
// s <= gram_max_rows().
int gram_max_rows();
// Dense updates use dws (dws_len doubles, s of them cursors) for column
// blocks of E made dense; gram_dense_block gives the block width, 0 for the
// sparse kernel.
int64_t gram_dense_block(int64_t s, int64_t cols, int64_t nnz, size_t dws_len);
// The sparse kernel accumulates in fixed point against info->scale (which =
// 0) or info->scale2 (which = 1), max_i ||e_i||^2, which must be set first.
void sparse_gram(hipStream_t st, int64_t s, int64_t cols, int64_t nnz, const int64_t *rp,
                 const int32_t *ci, const void *v, int vdt, int32_t *rid, double *S, int64_t lds,
                 double *dws, size_t dws_len, const SvDevInfo *info, int which);
template <typename T>
void scatter(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
             const void *v, int vdt, const double *M, T *base, const SvDevInfo *info);
// out[i] = X[i,:] Winv (or X[i,:] when *reset_flag), X[i][l] = src[i*rs + l*cs].
template <typename T>
void append_rows(hipStream_t st, int K, int64_t s, const double *src, int64_t rs, int64_t cs,
                 const double *Winv, const int32_t *reset_flag, T *out,
                 const SvDevInfo *info);

// ---- dense (k_dense.hip)
// C = alpha op(A) op(B) + beta C, FP64, row-major; op(X) = X^T when trans.
void gemm_f64(hipStream_t st, bool transA, bool transB, int64_t M, int64_t N, int64_t K,
              double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
              double beta, double *C, int64_t ldc, const SvDevInfo *info);
// The same, split over K into at most ws_len / (M N) partial products (in ws)
// when the output has few tiles; deterministic (fixed-order reduction).
void gemm_f64_sk(hipStream_t st, bool transA, bool transB, int64_t M, int64_t N, int64_t K,
                 double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc, double *ws, size_t ws_len,
                 const SvDevInfo *info);
// The number of partial products gemm_f64_sk splits an M x N x K product
// into when ws_len does not limit it (1: not split).
int64_t gemm_f64_splits(int64_t M, int64_t N, int64_t K);
// G[i][j] -= sum_l C[i][l] C[j][l] on the lower-triangular tiles, with C
// (s x K, float) multiplied on MFMA: mode 1 FP32, mode 2 BF16x3.
void gram_lowp(hipStream_t st, int mode, int64_t s, int K, const float *C, double *G,
               int64_t ldg, const SvDevInfo *info);
// dst[i][j] = src[i*rs + j*cs], i < R, j < C (FP64).
void copy_strided(hipStream_t st, int64_t R, int64_t C, const double *src, int64_t rs,
                  int64_t cs, double *dst, int64_t ldd, const SvDevInfo *info);
// max_i v[i] into info->scale (which = 0) or info->scale2 (which = 1).
void max_into(hipStream_t st, int64_t n, const double *v, SvDevInfo *info, int which);
constexpr int CHOL_NB = 32;
// ---- cooperative (k_coop.hip): one launch each; flags/epoch as for eig_topk
// G = L L^T in place (lower triangle); Linv receives the inverses of L's
// diagonal blocks (ceil(s / CHOL_NB) blocks of CHOL_NB^2 doubles, rows and
// columns of dropped pivots zero), which trsm_coop reads.  max_blocks > 0
// caps the launch (it then leaves CUs to work on other streams).
int cholesky_coop(hipStream_t st, int64_t s, double *G, int64_t ld, double *Linv,
                  double rank_tol, SvDevInfo *info, int which, unsigned *flags,
                  unsigned *epoch, int max_blocks = 0);
// Y <- L^{-T} Y (s x K) with the factor and its block inverses.
int trsm_coop(hipStream_t st, int64_t s, int K, const double *L, int64_t ld,
              const double *Linv, double *Y, const SvDevInfo *info, unsigned *flags,
              unsigned *epoch);
// mark the update failed on the device (every later kernel becomes a no-op)
void set_status(hipStream_t st, SvDevInfo *info, int code);
// reserve count + 1 barrier epochs; zero the flags first when close to wrap
unsigned take_epochs(hipStream_t st, unsigned *flags, unsigned *epoch, unsigned count);
// K = [[diag(sig), 0], [Cp, L]]  (N = K+s square, the add-rows form).
// M = K K^T of the append form without a product: the border (rows and
// columns < K) from sigma and C' (s x K); the block M[K:, K:] = E E^T must be
// in place already (copied from the sparse Gram).
void build_M_border(hipStream_t st, int K, int64_t s, const double *sig, const double *Cp,
                    double *M, const SvDevInfo *info);
void build_K_rows(hipStream_t st, int K, int64_t s, const double *sig, const double *Cp,
                  const double *L, int64_t ldl, double *Kout, const SvDevInfo *info);
// X = [Cp^T ; L^T]  ((K+s) x s) for the weight form.
void build_X(hipStream_t st, int K, int64_t s, const double *Cp, const double *L,
             int64_t ldl, double *X, const SvDevInfo *info);
// Kout[i][i] += sig[i] for i < K.
void add_sigma_diag(hipStream_t st, int K, const double *sig, double *Kout, int64_t ld,
                    const SvDevInfo *info);
// theta = sqrt(max(lambda, 0)); scale rows of Gv by 1/theta; mark rows whose
// theta is below tol * theta_0 for completion.
void theta_scale(hipStream_t st, int K, const double *lam, double *theta, double *Gv,
                 int64_t N, int32_t *complete, const SvDevInfo *info);
// Orthonormalise the K rows of X (K x N) by Cholesky QR applied twice,
// replacing rows flagged in complete (may be NULL) by pseudo-random rows
// first.  Gm, Linv: K x K scratch; Xtmp: K x N scratch.
void orthonormalize_rows(hipStream_t st, int K, int64_t N, double *X,
                         const int32_t *complete, uint64_t seed, double *Gm, double *Linv,
                         double *Xtmp, double *ws, size_t ws_len, const SvDevInfo *info);
// Winv = W^{-1} (k x k) by Gauss-Jordan with partial pivoting; kappa_1 into
// info; *flag = 1 when kappa > cond_reset or W is singular.
void inverse_cond(hipStream_t st, int K, const double *W, double *Winv, int32_t *flag,
                  double cond_reset, SvDevInfo *info, int side);
// Both sides' inverses of one update in one launch (two blocks).
void inverse_cond_pair(hipStream_t st, int K, const double *Wa, double *Wia, int32_t *fa, int sa,
                       const double *Wb, double *Wib, int32_t *fb, int sb, double cond_reset,
                       SvDevInfo *info);
// One side's inverse (the same kernels, one block).
void inverse_cond_one(hipStream_t st, int K, const double *W, double *Winv, int32_t *flag,
                      int side, double cond_reset, SvDevInfo *info);
// W = (reset ? I : Wnew); sig = theta (when sig_out != NULL); count resets.
void commit_small(hipStream_t st, int K, const double *Wnew, const int32_t *flag, double *W,
                  const double *theta, double *sig_out, SvDevInfo *info, int side);
// out[r] = in[r] * W for r < rows (tall-skinny).  When flag != NULL the kernel
// does nothing unless *flag.  mode 0: FP64 FMA, 1: FP32 MFMA, 2: BF16x3 MFMA.
template <typename Tin, typename Tout>
void realise(hipStream_t st, int mode, int K, int64_t rows, const Tin *in, const double *W,
             Tout *out, const int32_t *flag, const SvDevInfo *info);
// status = E_NUMERIC if any of x[0..n) is not finite.
void check_finite(hipStream_t st, int64_t n, const double *x, SvDevInfo *info, int seq);
void fill_identity(hipStream_t st, int K, double *W);
// Per-update bookkeeping in the device status block.
void op_begin(hipStream_t st, SvDevInfo *info, int two_sided);
void op_end(hipStream_t st, SvDevInfo *info);

// ---- approximate augmented space (k_approx.hip): the -GKL / -RPI variants
constexpr int AP_LMAX = 64;   // largest dimension l of the approximate space
// Copy the lower triangle of the symmetric s x s G onto its strict upper one.
void sym_lower(hipStream_t st, int64_t s, double *G, int64_t ld, const SvDevInfo *info);
// Y[j] = G X[j] for the nv rows of X and Y (s each); a no-op once *brk != 0.
void symv_rows(hipStream_t st, int64_t s, int nv, const double *G, int64_t ld, const double *X,
               double *Y, const int32_t *brk, const SvDevInfo *info);
// GKL in coefficient space on G = Z^T Z: Pv ((l+1) x s) the p vectors, Yc
// (l x s) the coefficients of q_i = Z y_i, ab alpha (AP_LMAX) then beta
// (AP_LMAX); g (s) scratch; start (s, device) or NULL for all ones.
void gkl_basis(hipStream_t st, int64_t s, int l, const double *G, int64_t ld,
               const double *start, double *Pv, double *Yc, double *g, double *ab,
               int32_t *brk, double rtol, SvDevInfo *info);
// Kout[row0 + t][col0 + i] = alpha_i Pv[i][t] + beta_i Pv[i+1][t].
void gkl_pblock(hipStream_t st, int64_t s, int l, const double *Pv, const double *ab,
                double *Kout, int64_t ldk, int64_t row0, int64_t col0, const SvDevInfo *info);
// Kout[row0 + t][col0 + i] = X[i][t] (X: l rows of s).
void rows_to_block(hipStream_t st, int64_t s, int l, const double *X, double *Kout, int64_t ldk,
                   int64_t row0, int64_t col0, const SvDevInfo *info);
// Kout ((K+s) x (K+l)) = [[diag(sig), 0], [Cp, 0]].
void build_K_approx(hipStream_t st, int K, int64_t s, int l, const double *sig, const double *Cp,
                    double *Kout, const SvDevInfo *info);
// Pivoted Cholesky of an l x l Gram with dropping (pivot <= rtol * scale of
// E, or rtol * the largest diagonal when rel); Out (l x l) maps the Gram's
// vectors to orthonormal ones (zero rows for dropped directions).
void pchol_small(hipStream_t st, int l, const double *A, double *Out, double rtol, int rel,
                 const SvDevInfo *info);
// RPI in coefficient space: t rounds from the rows of P (l x s, overwritten
// with Z^T Q); Yc receives the coefficients of Q.
void rpi_basis(hipStream_t st, int64_t s, int l, int t, const double *G, int64_t ld, double *P,
               double *Yc, double *X, double *T, double *Gm2, double *Om, double *ws,
               size_t ws_len, double rtol, const SvDevInfo *info);

// ---- queries and scores (k_query.hip)
// out[r] = base[idx[r]] W (K FP64 each); NaN rows for indices outside [0, rows).
template <typename T>
void query_rows(hipStream_t st, int K, int64_t n, const int64_t *idx, int64_t rows,
                const T *base, const double *W, double *out);
// WS = W diag(sig).
void scale_cols(hipStream_t st, int K, const double *W, const double *sig, double *WS);
// out[p] = Ut[I[p]] . Vt[J[p]] (max with Ut[J[p]] . Vt[I[p]] when both); NaN
// for a pair outside the factors (m rows of Ut, nn rows of Vt).
template <typename T>
void score_pairs(hipStream_t st, int K, int64_t n, const int64_t *I, const int64_t *J, int both,
                 int64_t m, int64_t nn, const T *Ut, const T *Vt, double *out);

// ---- initial truncated SVD (k_rsvd.hip; the product in k_sparse.hip)
// Y = A X, A a CSR (rows x cols), X cols x L FP64 row-major, L in {16..128}.
void csr_dense(hipStream_t st, int L, int64_t rows, const int64_t *rp, const int32_t *ci,
               const void *v, int vdt, const double *X, double *Y, const SvDevInfo *info);
// CSR of A^T (cols x rows; rows ascending within each row of A^T, FP64
// values) by a stable radix sort; scratch holds csr_transpose_bytes bytes.
size_t csr_transpose_bytes(int64_t nnz, int64_t cols);
// base[c, :] += sum_i E[i, c] M[i, :] (M s x K FP64, base n x K) with no
// floating-point atomics: the nonzeros sorted by column (stable radix sort),
// one wave per distinct column summing its rows in order; scratch holds
// scatter_det_bytes(nnz) bytes.
size_t scatter_det_bytes(int64_t nnz);
template <typename T>
void scatter_det(hipStream_t st, int K, int64_t s, int64_t cols, int64_t nnz, const int64_t *rp,
                 const int32_t *ci, const void *v, int vdt, const double *M, T *base,
                 void *scratch, const SvDevInfo *info);
void csr_transpose(hipStream_t st, int64_t rows, int64_t cols, int64_t nnz, const int64_t *rp,
                   const int32_t *ci, const void *v, int vdt, int64_t *rpT, int32_t *ciT,
                   double *vT, void *scratch, const SvDevInfo *info);
// status = E_NUMERIC when any of x[0..n) is not finite (many blocks).
void check_finite_wide(hipStream_t st, int64_t n, const double *x, SvDevInfo *info);
// Out = L^{-1} of the L x L Gram G (L <= 128) with dropped columns (pivot <=
// rtol * max diag) as zero rows, flagged in complete.
void chol_drop(hipStream_t st, int L, const double *G, double *Out, int32_t *complete,
               double rtol, const SvDevInfo *info);
void fill_cols(hipStream_t st, int64_t R, int L, double *X, const int32_t *complete,
               uint64_t seed, const SvDevInfo *info);
// sig = sqrt(max(lam, 0)); X (R x k) columns scaled by 1/sig, or zeroed when
// sig <= tol * sig_0.
void inv_sigma_cols(hipStream_t st, int64_t R, int k, const double *lam, double *sig, double *X,
                    double tol, const SvDevInfo *info);
// G = Y^T Y (both triangles) for the R x L panel Y (L in {16..128}) on FP64
// MFMA; ws holds ts_gram_ws(R, L) doubles.
size_t ts_gram_ws(int64_t R, int L);
void ts_gram(hipStream_t st, int64_t R, int L, const double *Y, double *G, double *ws,
             const SvDevInfo *info);
// Y = X Out^T for the R x L panel X and a lower-triangular L x L Out.
void ts_mul_lt(hipStream_t st, int64_t R, int L, const double *X, const double *Out, double *Y,
               const SvDevInfo *info);
// Orthonormal basis of the columns of the R x L panel X by `passes` passes
// of Cholesky QR alternating between X and Y; returns the buffer holding the
// result.  G, Out: L x L; complete: L; ws / ws_len: split-K scratch.
double *orth_cols(hipStream_t st, int64_t R, int L, double *X, double *Y, int passes, double *G,
                  double *Out, int32_t *complete, double *ws, size_t ws_len, uint64_t seed,
                  double rtol, const SvDevInfo *info);

// ---- eigen (k_eig.hip)
// Top-k eigenpairs of a symmetric N x N FP64 matrix (A is destroyed):
// lam[0..k) descending, Fv (k x N) row j = eigenvector of lam[j].
// work must hold eig_work_doubles(N, k) doubles.
size_t eig_work_doubles(int64_t N, int k);
// flags: TRI_MAX_BLOCKS * 16 unsigned words, zeroed once by the owner; *epoch
// is the owner's running epoch counter for them (starts at 0).
constexpr int TRI_MAX_BLOCKS = 256;
constexpr size_t TRI_FLAG_WORDS = (size_t)TRI_MAX_BLOCKS * 16;
// p[0..n) = 0 by a fill kernel on st (capturable: no memset node).
void zero_words(hipStream_t st, unsigned *p, size_t n);
int eig_topk(hipStream_t st, int64_t N, double *A, int k, double *lam, double *Fv,
             double *work, unsigned *flags, unsigned *epoch, const SvDevInfo *info);
// The four stages of eig_topk, launched separately (same work layout).
int eig_tridiag(hipStream_t st, int64_t N, double *A, double *work, unsigned *flags,
                unsigned *epoch, const SvDevInfo *info);
void eig_bisect(hipStream_t st, int64_t N, int k, double *lam, double *work,
                const SvDevInfo *info);
void eig_stein(hipStream_t st, int64_t N, int k, const double *lam, double *Fv, double *work,
               const SvDevInfo *info);
void eig_back(hipStream_t st, int64_t N, int k, const double *A, double *Fv, double *work,
              const SvDevInfo *info);
int eig_max_n();
// Largest N whose tridiagonalisation is one block (no cooperative launch,
// flags and epoch unused): eig_topk on such an N can run beside a
// cooperative kernel of another stream.
constexpr int EIG_ONE_BLOCK_N = 160;

// ---- Chebyshev-filtered subspace iteration (k_chefsi.hip)
// Top-k eigenpairs of the positive semidefinite N x N matrix M (not
// modified) with a basis of chefsi_block(k) columns, for the (N, k) that
// chefsi_applies() accepts; ws holds chefsi_work_doubles(N, k) doubles,
// ctl_host 4 doubles of pinned host memory.  Outputs as eig_topk.  The call
// waits for the stream after every Rayleigh-Ritz step (the host picks the
// filter degree and stops when max_j ||M x_j - theta_j x_j|| <= tol theta_0).
// Returns 0 when converged, 1 when not within max_it filter steps (the
// outputs are then not written), < 0 on a launch or argument error; *iters
// receives the number of filter steps.
int chefsi_block(int k);
bool chefsi_applies(int64_t N, int k);
size_t chefsi_work_doubles(int64_t N, int k);
// Work of the update's eigenproblem: the direct solver's, or the iterative
// one's where it applies (the direct solver is its fallback on the same
// memory).
size_t eig_update_work_doubles(int64_t N, int k);
// *flops (may be NULL) receives the run's algorithmic flops.
// flags / epoch as for eig_topk (used when the basis is wider than 128).
int eig_topk_chefsi(hipStream_t st, int64_t N, const double *M, int k, double *lam, double *Fv,
                    double *ws, size_t ws_len, double *ctl_host, double tol, int max_it,
                    uint64_t seed, const SvDevInfo *info, int *iters, double *flops,
                    unsigned *flags, unsigned *epoch);

}  // namespace svl
