// Top-k eigenpairs of a symmetric N x N FP64 matrix M by Chebyshev-filtered
// subspace iteration with Rayleigh-Ritz: the (k+s) Rayleigh-Ritz SVD of the
// update (Section 2.1, step 2; Theorem 1's (k+s)^3 term) needs only the k
// leading eigenpairs of M = K K^T, so instead of reducing all of M to
// tridiagonal form (one grid-wide exchange per column) the solver works on an
// N x p block (p = k + 32 columns, see chefsi_block) with dense products M X on
// FP64 MFMA:
//
//   X <- orth(start);  repeat:  Y = M X,  H = X^T Y,  H = Q diag(theta) Q^T,
//   X <- X Q, Y <- Y Q;  stop when ||Y_j - theta_j X_j|| <= tol ||M|| (j < k);
//   otherwise X <- orth(C_d(M) X) with C_d the degree-d Chebyshev polynomial
//   that is bounded by 1 on [0, theta_p] and grows fast above it.
//
// The filter is the scaled three-term recurrence of Zhou and Saad (2007); the
// orthonormalisation is Cholesky QR with column dropping and completion
// (after the columns are scaled to unit length, since the filter amplifies
// each Ritz direction by a different factor).  The host reads four scalars
// after each Rayleigh-Ritz step (the extreme Ritz values and the largest
// residual) to choose the degree and to stop; a run that has not converged
// after max_it steps reports so, and the caller falls back to the direct
// solver.  Storage: X, Y and the filter's vectors are N x p row-major (one
// basis vector per column), the result is written as the direct solver's
// (lam descending, Fv k x N, row j an eigenvector, its entry of largest
// magnitude positive).
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <initializer_list>

#include "common.hpp"
#include "k_rsvd.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

// Orthonormal start, no factorisation needed: X[:, j] = e_j for j < k (the
// leading coordinates: for M = K K^T of an update they are the previous
// singular directions), and for k <= j < p a vector of pseudo-random signs
// on the coordinates c >= k with (c - k) mod (p - k) = j - k, scaled to unit
// length; the supports are disjoint, so the columns are orthonormal.
__global__ void k_cf_init(int64_t N, int k, int p, double *__restrict__ X, uint64_t seed,
                          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t q = p - k, span = N - k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * p;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / p;
    const int j = (int)(e % p);
    double v = 0.0;
    if (j < k) {
      v = i == j ? 1.0 : 0.0;
    } else if (i >= k && (i - k) % q == j - k) {
      const int64_t cnt = (span - (j - k) + q - 1) / q;   // coordinates of column j
      const double h = hash_unit(seed * 0x9E3779B97F4A7C15ull + (uint64_t)e * 0xD1B54A32D192ED03ull);
      v = (h < 0.0 ? -1.0 : 1.0) / sqrt((double)cnt);
    }
    X[e] = v;
  }
}

// Scale every column of the N x p panel to unit length (a zero column stays
// zero; the orthonormalisation completes it).  One block per column.
__global__ void __launch_bounds__(256)
k_cf_colnorm(int64_t N, int p, double *__restrict__ X, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double v = X[i * p + j];
    s += v * v;
  }
  s = block_sum(s, red);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) X[i * p + j] *= inv;
}

// C = a A + b B (n entries); B may be null (b ignored).
__global__ void k_cf_combine(int64_t n, double a, const double *__restrict__ A, double b,
                             const double *__restrict__ B, double *__restrict__ C,
                             const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    C[e] = B ? a * A[e] + b * B[e] : a * A[e];
}

// H <- (H + H^T) / 2 (p x p): the Rayleigh quotient matrix is symmetric up
// to the rounding of its two products.
__global__ void k_cf_symmetrize(int p, double *__restrict__ H, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e / p, j = e % p;
    if (j < i) {
      const double v = 0.5 * (H[i * p + j] + H[j * p + i]);
      H[i * p + j] = v;
      H[j * p + i] = v;
    }
  }
}

// Residual norms r_j = ||Y[:, j] - theta_j X[:, j]|| (j < k) into rj, one
// block per column; the last block to finish (ticket counter) writes the
// control scalars: ctl = {max_j r_j, theta_0, theta_{k-1}, theta_{p-1}}.
__global__ void __launch_bounds__(256)
k_cf_resid(int64_t N, int p, int k, const double *__restrict__ X, const double *__restrict__ Y,
           const double *__restrict__ theta, double *__restrict__ rj, unsigned *__restrict__ ticket,
           double *__restrict__ ctl, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double red[4];
  __shared__ bool last;
  const int j = blockIdx.x;
  const double t = theta[j];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double r = Y[i * p + j] - t * X[i * p + j];
    s += r * r;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    rj[j] = sqrt(s);
    __threadfence();
    last = atomicAdd(ticket, 1u) == (unsigned)gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int q = 0; q < k; ++q) mx = fmax(mx, __hip_atomic_load(&rj[q], __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT));
    ctl[0] = mx;
    ctl[1] = theta[0];
    ctl[2] = theta[k - 1];
    ctl[3] = theta[p - 1];
    *ticket = 0u;
  }
}

// lam[j] = theta[j], Fv row j = column j of X with the sign that makes its
// entry of largest magnitude positive (the first such entry on ties).
__global__ void __launch_bounds__(256)
k_cf_output(int64_t N, int p, const double *__restrict__ X, const double *__restrict__ theta,
            double *__restrict__ lam, double *__restrict__ Fv, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  double amax = -1.0;
  int64_t amx = 0;
  for (int64_t i = tid; i < N; i += 256) {
    const double a = fabs(X[i * p + j]);
    if (a > amax) { amax = a; amx = i; }
  }
  bv[tid] = amax;
  bi[tid] = amx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      const double ov = bv[tid + o];
      const int64_t oi = bi[tid + o];
      if (ov > bv[tid] || (ov == bv[tid] && oi < bi[tid])) { bv[tid] = ov; bi[tid] = oi; }
    }
    __syncthreads();
  }
  const double sg = X[bi[0] * p + j] < 0.0 ? -1.0 : 1.0;
  for (int64_t i = tid; i < N; i += 256) Fv[(int64_t)j * N + i] = sg * X[i * p + j];
  if (tid == 0) lam[j] = theta[j];
}

// ctl[0] = NaN before every Rayleigh-Ritz step: if an earlier failure has
// turned the step's kernels into no-ops, the host reads a NaN and stops.
__global__ void k_cf_ctl_reset(double *ctl) {
  if (threadIdx.x == 0) ctl[0] = __builtin_nan("");
}

unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

namespace svl {

// basis width p = k + 32 rounded up to a multiple of 16 (at most 256): 32
// guard vectors keep the gap between the k-th wanted and the first damped
// Ritz value wide enough for one Chebyshev step on the graph spectra, and
// every p x p stage (Gram, Cholesky QR, the Rayleigh quotient's eigensolver)
// scales with p (a sweep on the 100k-node graph workload at k = 64:
// p = 128 3.99 ms, 96 3.63 ms, 80 3.45 ms median but with a second filter
// step on some updates).  Beyond 128 columns (k = 128) the p x p eigensolver
// is the cooperative one (flags and epoch needed) and the orthonormalisation
// works in two column blocks.  SVLCOV_CHEFSI_P overrides p for tuning sweeps
// (a multiple of 16 in (k, 256]).
int chefsi_block(int k) {
  static const int forced = [] {
    const char *ev = getenv("SVLCOV_CHEFSI_P");
    return ev ? atoi(ev) : 0;
  }();
  if (forced > k && forced <= 256 && forced % 16 == 0) return forced;
  const int p = (k + 32 + 15) / 16 * 16;
  return p < 256 ? p : 256;
}

bool chefsi_applies(int64_t N, int k) {
  const int p = chefsi_block(k);
  return (k == 8 || k == 16 || k == 32 || k == 64 || k == 128) && N > 128 && N >= p + 32;
}

// Split-K / Gram scratch (doubles): room for every partial product the
// GEMM launcher asks for (M X, X^T Y, and for p > 128 the 128 x (p - 128)
// coupling of the two column blocks), and the Cholesky-QR Gram.
static size_t chefsi_gws(int64_t N, int p) {
  const size_t panel = (size_t)N * p;
  size_t g = std::max(ts_gram_ws(N, p), (size_t)gemm_f64_splits(N, p, N) * panel);
  g = std::max(g, (size_t)gemm_f64_splits(p, p, N) * p * p);
  if (p > 128) g = std::max(g, (size_t)gemm_f64_splits(128, p - 128, N) * 128 * (p - 128));
  return g + 64;
}

// Layout of the workspace (doubles): five N x p panels, the split-K / Gram
// scratch, then the p x p blocks, theta, residuals, control words and the
// direct solver's work for the p x p Rayleigh quotient.
size_t chefsi_work_doubles(int64_t N, int k) {
  const int p = chefsi_block(k);
  const size_t panel = (size_t)N * p;
  const size_t gws = chefsi_gws(N, p);
  return 5 * panel + gws + 4 * (size_t)p * p + 3 * (size_t)p + 64 + eig_work_doubles(p, p);
}

size_t eig_update_work_doubles(int64_t N, int k) {
  const size_t d = eig_work_doubles(N, k);
  return chefsi_applies(N, k) ? std::max(d, chefsi_work_doubles(N, k)) : d;
}

int eig_topk_chefsi(hipStream_t st, int64_t N, const double *M, int k, double *lam, double *Fv,
                    double *ws, size_t ws_len, double *ctl_host, double tol, int max_it,
                    uint64_t seed, const SvDevInfo *info, int *iters, double *flops,
                    unsigned *flags, unsigned *epoch) {
  const int p = chefsi_block(k);
  // algorithmic flops: 2 N^2 p per product with M, 2 N p^2 per Rayleigh
  // quotient and 4 N p^2 per rotation of X and M X
  double fl = 0.0;
  const double f_prod = 2.0 * (double)N * (double)N * p, f_rr = 6.0 * (double)N * p * p;
  struct FlopOut {
    double *dst;
    double *val;
    ~FlopOut() { if (dst) *dst = *val; }
  } flop_out{flops, &fl};
  if (!chefsi_applies(N, k) || ws_len < chefsi_work_doubles(N, k)) return -1;
  const size_t panel = (size_t)N * p;
  double *B[5];
  for (int q = 0; q < 5; ++q) B[q] = ws + q * panel;
  double *gws = ws + 5 * panel;
  const size_t gws_len = chefsi_gws(N, p);
  const size_t pp = (size_t)p * p;
  double *G = gws + gws_len, *Out = G + pp, *H = Out + pp, *Qv = H + pp;
  double *theta = Qv + pp, *rj = theta + p;
  int32_t *complete = (int32_t *)(rj + p);   // p words in the space of p doubles
  double *ctl = rj + 2 * p;                   // 64 doubles: results, then the ticket
  unsigned *ticket = (unsigned *)(ctl + 8);
  double *ews = ctl + 64;
  const double rtol = 1e-13;
  zero_words(st, ticket, 2);

  // basis X (in B[0]), Y = M X (B[1]); B[2..4] are scratch
  double *X = B[0], *Y = B[1];
  // columns scaled to unit length, one pass of Cholesky QR, and a second one
  // when a column was completed or (gate_tau < 1) when the first's input was
  // not orthonormal to within gate_tau per entry of its Gram (at 1e-2 the
  // condition number is at most 1 + 1.27, and one pass then leaves an
  // orthogonality error of a few u)
  int32_t *need = (int32_t *)(ctl + 16);
  // p > 128 (k = 128): block Gram-Schmidt with reorthogonalisation over the
  // first 128 columns and the rest, each block by the same Cholesky QR
  // (its kernels take at most 128 columns); panel and scratch are two free
  // N x p panels, the 128 x r coupling goes through H
  auto orth = [&](double *src, double *scratch, double *spare, double gate_tau) -> double * {
    hipLaunchKernelGGL(k_cf_colnorm, dim3(p), dim3(256), 0, st, N, p, src, info);
    if (p <= 128)
      return orth_cols_cond(st, N, p, src, scratch, G, Out, complete, need, gws, gws_len, ++seed,
                            rtol, info, gate_tau);
    const int r = p - 128;
    double *Xa = spare, *Xb = spare + (size_t)N * 128;
    copy_strided(st, N, 128, src, p, 1, Xa, 128, info);
    copy_strided(st, N, r, src + 128, p, 1, Xb, r, info);
    orth_cols_cond(st, N, 128, Xa, scratch, G, Out, complete, need, gws, gws_len, ++seed, rtol,
                   info, gate_tau);
    for (int pass = 0; pass < 2; ++pass) {
      gemm_f64_sk(st, true, false, 128, r, N, 1.0, Xa, 128, Xb, r, 0.0, H, r, gws, gws_len, info);
      gemm_f64(st, false, false, N, r, 128, -1.0, Xa, 128, H, r, 1.0, Xb, r, info);
    }
    orth_cols_cond(st, N, r, Xb, scratch, G, Out, complete, need, gws, gws_len, ++seed, rtol,
                   info, gate_tau);
    copy_strided(st, N, 128, Xa, 128, 1, src, p, info);
    copy_strided(st, N, r, Xb, r, 1, src + 128, p, info);
    return src;
  };
  auto other = [&](std::initializer_list<const double *> used) -> double * {
    for (int q = 0; q < 5; ++q) {
      bool u = false;
      for (const double *x : used) u |= (x == B[q]);
      if (!u) return B[q];
    }
    return nullptr;
  };
  // Rayleigh-Ritz on the orthonormal X: Y = M X, H = X^T Y = Q diag(theta)
  // Q^T, X <- X Q^T... (Qv holds the eigenvectors of H as rows), Y <- Y Q;
  // then the residuals and the control scalars, read by the host.
  auto rayleigh_ritz = [&]() -> bool {
    fl += f_prod + f_rr;
    gemm_f64_sk(st, false, false, N, p, N, 1.0, M, N, X, p, 0.0, Y, p, gws, gws_len, info);
    gemm_f64_sk(st, true, false, p, p, N, 1.0, X, p, Y, p, 0.0, H, p, gws, gws_len, info);
    hipLaunchKernelGGL(k_cf_symmetrize, dim3(grid_of((int64_t)p * p)), dim3(256), 0, st, p, H,
                       info);
    if (eig_topk(st, p, H, p, theta, Qv, ews, flags, epoch, info) != 0) return false;
    double *Xn = other({X, Y});
    gemm_f64(st, false, true, N, p, p, 1.0, X, p, Qv, p, 0.0, Xn, p, info);
    double *Yn = other({X, Y, Xn});
    gemm_f64(st, false, true, N, p, p, 1.0, Y, p, Qv, p, 0.0, Yn, p, info);
    X = Xn;
    Y = Yn;
    hipLaunchKernelGGL(k_cf_ctl_reset, dim3(1), dim3(64), 0, st, ctl);
    hipLaunchKernelGGL(k_cf_resid, dim3(k), dim3(256), 0, st, N, p, k, X, Y, theta, rj, ticket,
                       ctl, info);
    (void)hipMemcpyAsync(ctl_host, ctl, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    return hipStreamSynchronize(st) == hipSuccess;
  };

  hipLaunchKernelGGL(k_cf_init, dim3(grid_of((int64_t)panel)), dim3(256), 0, st, N, k, p, X,
                     seed, info);
  // two plain power steps before the first Rayleigh-Ritz step: they take
  // the start's residual from ~1e-1 to ~1e-5 of the largest eigenvalue, so
  // that one Chebyshev step (whose degree the spread of amplification over
  // the wanted eigenvalues limits) usually suffices after it
  for (int q = 0; q < 2; ++q) {
    double *Z = other({X});
    fl += f_prod;
    gemm_f64_sk(st, false, false, N, p, N, 1.0, M, N, X, p, 0.0, Z, p, gws, gws_len, info);
    X = Z;
  }
  // the basis after the power steps only feeds the first Rayleigh-Ritz step
  // (bounds and a rotation) and the filter, which needs its span alone: one
  // pass leaves it orthonormal to about u cond(X)^2, which for the two power
  // steps' condition number moves the Ritz values by far less than the
  // residuals they are judged by; a completed column still takes the second
  // pass (it is random, not orthogonal to the kept ones)
  {
    double *sc = other({X});
    X = orth(X, sc, other({X, sc}), 2.0);
  }
  Y = other({X});
  if (!rayleigh_ritz()) return -3;
  bool have_y = true;
  double res = ctl_host[0], th0 = ctl_host[1], thk = ctl_host[2], thp = ctl_host[3];
  int it = 0;
  for (;; ++it) {
    const double scale = std::max(std::fabs(th0), 1e-300);
    if (!(res == res)) break;   // a NaN: let the direct solver take over
    if (res <= tol * scale || th0 == thp) {
      hipLaunchKernelGGL(k_cf_output, dim3(k), dim3(256), 0, st, N, p, X, theta, lam, Fv, info);
      if (iters) *iters = it;
      return 0;
    }
    if (it >= max_it) break;
    // damped interval [a, b] = [0, theta_{p-1}] (M is positive semidefinite;
    // eigenvalues a rounding error below 0 grow by a negligible factor)
    const double a = 0.0;
    double b = thp;
    if (!(b > a)) b = a + 1e-12 * scale;
    const double e = 0.5 * (b - a), c = 0.5 * (b + a);
    const double xk = (thk - c) / e, x1 = (th0 - c) / e;
    int d = 8;
    if (xk > 1.0 + 1e-12) {
      const double ak = std::acosh(xk), a1 = std::acosh(std::max(x1, xk));
      // degree for a reduction of 1e10 of every unwanted component relative
      // to the k-th wanted one, limited so that the spread of amplification
      // over the wanted directions (the largest against the k-th) times the
      // residual level stays below 1e6 (beyond that the smaller wanted
      // directions would drown in the rounding of the larger ones)
      d = (int)std::ceil(std::log(2e10) / ak);
      if (a1 > ak) {
        const int dmax = (int)(std::log(1e6 / std::max(res / scale, 2.2e-16)) / (a1 - ak));
        d = std::min(d, std::max(dmax, 1));
      }
      d = std::min(std::max(d, 1), 32);
    }
    // scaled Chebyshev recurrence, scale point th0 (its component stays ~1)
    const double sigma1 = th0 > c ? e / (th0 - c) : 1.0;
    double sigma = sigma1;
    if (!have_y) {
      Y = other({X});
      fl += f_prod;
      gemm_f64_sk(st, false, false, N, p, N, 1.0, M, N, X, p, 0.0, Y, p, gws, gws_len, info);
    }
    double *Yp = X;
    double *Yc = other({X, Y});
    hipLaunchKernelGGL(k_cf_combine, dim3(grid_of((int64_t)panel)), dim3(256), 0, st,
                       (int64_t)panel, sigma1 / e, Y, -sigma1 * c / e, X, Yc, info);
    for (int q = 2; q <= d; ++q) {
      const double sn = 1.0 / (2.0 / sigma1 - sigma);
      double *T = other({Yp, Yc});
      hipLaunchKernelGGL(k_cf_combine, dim3(grid_of((int64_t)panel)), dim3(256), 0, st,
                         (int64_t)panel, -2.0 * sn * c / e, Yc, -sigma * sn, Yp, T, info);
      fl += f_prod;
      gemm_f64_sk(st, false, false, N, p, N, 2.0 * sn / e, M, N, Yc, p, 1.0, T, p, gws, gws_len,
                  info);
      Yp = Yc;
      Yc = T;
      sigma = sn;
    }
    {
      double *sc = other({Yc});
      X = orth(Yc, sc, other({Yc, sc}), 1e-2);
    }
    Y = other({X});
    if (!rayleigh_ritz()) return -3;
    have_y = true;
    res = ctl_host[0]; th0 = ctl_host[1]; thk = ctl_host[2]; thp = ctl_host[3];
  }
  if (iters) *iters = it;
  return 1;
}

}  // namespace svl
