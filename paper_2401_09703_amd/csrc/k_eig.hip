// Top-k eigenpairs of a symmetric FP64 matrix on the GPU, the core of the
// (k+s) Rayleigh-Ritz SVD (Section 2.1, step 2): the left singular vectors of
// K are the eigenvectors of K K^T and its eigenvalues are the squared singular
// values.
//
//   1. Householder tridiagonalisation Q^T M Q = T in one cooperative kernel.
//      Each block owns the rows r = g, g + G, ... of M (cyclic, so the
//      shrinking trailing matrix stays balanced).  Per column one grid-wide
//      barrier: every block recomputes the next reflector redundantly from the
//      published row, applies the pending rank-2 update to its own rows fused
//      with the product p = tau M v, and publishes its part of p.
//   2. Bisection on Sturm counts for the k largest eigenvalues of T, one wave
//      per eigenvalue with 64-way multisection.
//   3. Inverse iteration with the eigenvalue as shift (tridiagonal LU with
//      partial pivoting), re-orthogonalised inside clusters of close
//      eigenvalues.
//   4. Back-transformation of the k vectors by the stored reflectors.
#include <hip/hip_cooperative_groups.h>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;
namespace cg = cooperative_groups;

namespace {

constexpr int TRI_THREADS = 256;
constexpr double EPS = 1.1102230246251565e-16;     // 2^-53
constexpr double SAFMIN = 2.2250738585072014e-308;

__global__ void __launch_bounds__(TRI_THREADS)
k_tridiag(int N, double *__restrict__ A, int64_t lda, double *__restrict__ d,
          double *__restrict__ e, double *__restrict__ tau, double *__restrict__ pbuf,
          double *__restrict__ rowbuf, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  cg::grid_group grid = cg::this_grid();
  extern __shared__ double sm[];
  __shared__ double red[TRI_THREADS / 64];
  const int G = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, w = tid >> 6, nw = NT >> 6;
  if (N < 3) {
    if (g == 0 && tid == 0) {
      d[0] = A[0];
      if (N == 2) { e[0] = A[1]; d[1] = A[lda + 1]; }
    }
    return;
  }
  double *X = sm, *VP = sm + N, *WP = sm + 2 * N;
  for (int j = tid; j < N; j += NT) X[j] = A[j];
  __syncthreads();
  for (int i = 0; i <= N - 3; ++i) {
    const double dii = X[i];
    double part = 0.0;
    for (int j = i + 2 + tid; j < N; j += NT) part += X[j] * X[j];
    const double xn2 = block_sum(part, red);
    const double alpha = X[i + 1];
    double beta, t, scl;
    if (xn2 == 0.0) {
      t = 0.0; beta = alpha; scl = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xn2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scl = 1.0 / (alpha - beta);
    }
    __syncthreads();
    for (int j = i + 2 + tid; j < N; j += NT) X[j] *= scl;
    if (tid == 0) X[i + 1] = 1.0;
    __syncthreads();
    if (g == i % G) {
      // row i of M is finished: keep the reflector there (columns i+1..)
      for (int j = i + 1 + tid; j < N; j += NT) A[(int64_t)i * lda + j] = X[j];
      if (tid == 0) { d[i] = dii; e[i] = beta; tau[i] = t; }
    }
    double *pb = pbuf + (int64_t)(i & 1) * N;
    double *rb = rowbuf + (int64_t)(i & 1) * N;
    const int first = i + 1 + (((g - (i + 1)) % G) + G) % G;
    for (int r = first + w * G; r < N; r += nw * G) {
      double *Ar = A + (int64_t)r * lda;
      const double vpr = i >= 1 ? VP[r] : 0.0, wpr = i >= 1 ? WP[r] : 0.0;
      const bool pub = (r == i + 1);
      double acc = 0.0;
      for (int j = i + 1 + lane; j < N; j += 64) {
        double a = Ar[j];
        if (i >= 1) {
          a -= vpr * WP[j] + wpr * VP[j];
          Ar[j] = a;
        }
        if (pub) rb[j] = a;
        acc += a * X[j];
      }
      acc = wave_sum(acc);
      if (lane == 0) pb[r] = t * acc;
    }
    grid.sync();
    double part2 = 0.0;
    for (int j = i + 1 + tid; j < N; j += NT) part2 += pb[j] * X[j];
    const double pv = block_sum(part2, red);
    const double aw = -0.5 * t * pv;
    for (int j = i + 1 + tid; j < N; j += NT) WP[j] = pb[j] + aw * X[j];
    __syncthreads();
    double *Xn = VP;
    const double wi1 = WP[i + 1];
    for (int j = i + 1 + tid; j < N; j += NT) Xn[j] = rb[j] - (X[i + 1] * WP[j] + wi1 * X[j]);
    __syncthreads();
    VP = X;
    X = Xn;
  }
  if (g == 0 && tid == 0) {
    d[N - 2] = X[N - 2];
    e[N - 2] = X[N - 1];
  }
  if (g == (N - 1) % G && tid == 0) {
    d[N - 1] = A[(int64_t)(N - 1) * lda + N - 1] - 2.0 * VP[N - 1] * WP[N - 1];
  }
}

__device__ __forceinline__ int sturm_count(int N, const double *__restrict__ d,
                                           const double *__restrict__ e, double x,
                                           double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q <= 0.0) ++cnt;
  for (int i = 1; i < N; ++i) {
    const double ei = e[i - 1];
    q = d[i] - x - (ei * ei) / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q <= 0.0) ++cnt;
  }
  return cnt;
}

// Gershgorin bounds and the 1-norm of T, by one wave.
__device__ void tri_bounds(int N, const double *__restrict__ d, const double *__restrict__ e,
                           double &gl, double &gu, double &onenrm, double &emax2) {
  const int lane = threadIdx.x & 63;
  double lo = INFINITY, hi = -INFINITY, nm = 0.0, em = 0.0;
  for (int i = lane; i < N; i += 64) {
    const double a = i > 0 ? fabs(e[i - 1]) : 0.0;
    const double b = i < N - 1 ? fabs(e[i]) : 0.0;
    lo = fmin(lo, d[i] - a - b);
    hi = fmax(hi, d[i] + a + b);
    nm = fmax(nm, fabs(d[i]) + a + b);
    if (i < N - 1) em = fmax(em, e[i] * e[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    nm = fmax(nm, __shfl_xor(nm, o, 64));
    em = fmax(em, __shfl_xor(em, o, 64));
  }
  gl = lo; gu = hi; onenrm = nm; emax2 = em;
}

// lam[j] = the (N-1-j)-th smallest eigenvalue of T (so lam is descending).
__global__ void __launch_bounds__(64)
k_bisect(int N, const double *__restrict__ d, const double *__restrict__ e, int k,
         double *__restrict__ lam, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int j = blockIdx.x, lane = threadIdx.x;
  if (j >= k) return;
  const int idx = N - 1 - j;
  double gl, gu, onenrm, emax2;
  tri_bounds(N, d, e, gl, gu, onenrm, emax2);
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = SAFMIN * fmax(1.0, emax2);
  gl -= 2.0 * EPS * tnorm * N + 4.0 * pivmin;
  gu += 2.0 * EPS * tnorm * N + 4.0 * pivmin;
  double lo = gl, hi = gu;
  for (int round = 0; round < 40; ++round) {
    const double tol = 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin;
    if (hi - lo <= tol) break;
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count(N, d, e, x, pivmin);
    const unsigned long long mask = __ballot(cnt > idx);
    const double x63 = __shfl(x, 63, 64);
    if (mask == 0ull) {
      lo = x63;
    } else {
      const int f = __builtin_ctzll(mask);
      const double xf = __shfl(x, f, 64);
      const double xp = __shfl(x, f > 0 ? f - 1 : 0, 64);
      hi = xf;
      if (f > 0) lo = xp;
    }
  }
  if (lane == 0) lam[j] = 0.5 * (lo + hi);
}

// Inverse iteration for the clusters of lam (descending).  One wave per
// cluster leader; members of a cluster are computed in order and
// re-orthogonalised against the earlier members after every solve.
__global__ void __launch_bounds__(64)
k_stein(int N, const double *__restrict__ d, const double *__restrict__ e, int k,
        const double *__restrict__ lam, double *__restrict__ Fv, double *__restrict__ scratch,
        const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double xs[];   // N
  const int j0 = blockIdx.x, lane = threadIdx.x;
  double gl, gu, onenrm, emax2;
  tri_bounds(N, d, e, gl, gu, onenrm, emax2);
  const double ortol = 1e-3 * onenrm;
  if (j0 > 0 && lam[j0 - 1] - lam[j0] <= ortol) return;   // not a leader
  int j1 = j0 + 1;
  while (j1 < k && lam[j1 - 1] - lam[j1] <= ortol) ++j1;
  double *dd = scratch + (int64_t)j0 * 6 * N;
  double *dl = dd + N, *du = dl + N, *du2 = du + N;
  int *ipiv = (int *)(du2 + N);
  const double tiny = fmax(EPS * onenrm, 1e-290);
  for (int j = j0; j < j1; ++j) {
    const double lj = lam[j];
    if (onenrm == 0.0) {
      for (int c = lane; c < N; c += 64) Fv[(int64_t)j * N + c] = (c == j) ? 1.0 : 0.0;
      continue;
    }
    // LU with partial pivoting of T - lj I (lane 0), then random start
    if (lane == 0) {
      for (int i = 0; i < N; ++i) dd[i] = d[i] - lj;
      for (int i = 0; i < N - 1; ++i) { dl[i] = e[i]; du[i] = e[i]; }
      for (int i = 0; i < N - 2; ++i) du2[i] = 0.0;
      for (int i = 0; i < N; ++i) ipiv[i] = i;
      for (int i = 0; i < N - 1; ++i) {
        if (fabs(dd[i]) >= fabs(dl[i])) {
          const double piv = fabs(dd[i]) < tiny ? copysign(tiny, dd[i]) : dd[i];
          dd[i] = piv;
          const double fact = dl[i] / piv;
          dl[i] = fact;
          dd[i + 1] -= fact * du[i];
          if (i < N - 2) du2[i] = 0.0;
        } else {
          const double fact = dd[i] / dl[i];
          dd[i] = dl[i];
          dl[i] = fact;
          const double temp = du[i];
          du[i] = dd[i + 1];
          dd[i + 1] = temp - fact * dd[i + 1];
          if (i < N - 2) {
            du2[i] = du[i + 1];
            du[i + 1] = -fact * du[i + 1];
          }
          ipiv[i] = i + 1;
        }
      }
      if (fabs(dd[N - 1]) < tiny) dd[N - 1] = copysign(tiny, dd[N - 1]);
    }
    for (int c = lane; c < N; c += 64)
      xs[c] = hash_unit(0x5bd1e995ull * (uint64_t)(j + 1) + (uint64_t)c * 0x9E3779B97F4A7C15ull);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (lane == 0) {
        // solve with L (row interchanges), then U
        for (int i = 0; i < N - 1; ++i) {
          const int ip = ipiv[i];
          const double temp = xs[i + 1 - ip + i] - dl[i] * xs[ip];
          xs[i] = xs[ip];
          xs[i + 1] = temp;
        }
        xs[N - 1] /= dd[N - 1];
        if (N > 1) xs[N - 2] = (xs[N - 2] - du[N - 2] * xs[N - 1]) / dd[N - 2];
        for (int i = N - 3; i >= 0; --i)
          xs[i] = (xs[i] - du[i] * xs[i + 1] - du2[i] * xs[i + 2]) / dd[i];
      }
      __syncthreads();
      // orthogonalise against earlier members of the cluster, then normalise
      for (int p = j0; p < j; ++p) {
        const double *fp = Fv + (int64_t)p * N;
        double dot = 0.0;
        for (int c = lane; c < N; c += 64) dot += fp[c] * xs[c];
        dot = wave_sum(dot);
        for (int c = lane; c < N; c += 64) xs[c] -= dot * fp[c];
        __syncthreads();
      }
      double amax = 0.0;
      for (int c = lane; c < N; c += 64) amax = fmax(amax, fabs(xs[c]));
      amax = wave_max(amax);
      const double sc = amax > 0.0 ? 1.0 / amax : 1.0;
      double nrm = 0.0;
      for (int c = lane; c < N; c += 64) { xs[c] *= sc; nrm += xs[c] * xs[c]; }
      nrm = sqrt(wave_sum(nrm));
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int c = lane; c < N; c += 64) xs[c] *= inv;
      __syncthreads();
    }
    // fixed sign: the entry of largest magnitude (first on ties) is positive
    double amax = -1.0;
    int amx = 0;
    for (int c = lane; c < N; c += 64) {
      const double a = fabs(xs[c]);
      if (a > amax) { amax = a; amx = c; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double oa = __shfl_xor(amax, o, 64);
      const int oi = __shfl_xor(amx, o, 64);
      if (oa > amax || (oa == amax && oi < amx)) { amax = oa; amx = oi; }
    }
    const double sg = xs[amx] < 0.0 ? -1.0 : 1.0;
    for (int c = lane; c < N; c += 64) Fv[(int64_t)j * N + c] = sg * xs[c];
    __syncthreads();
  }
}

// x <- H_0 H_1 ... H_{N-3} x for every row of Fv; reflector i is stored in
// row i of A (columns i+1 .., with a unit leading entry) and tau[i].
__global__ void k_backtransform(int N, int k, const double *__restrict__ A, int64_t lda,
                                const double *__restrict__ tau, double *__restrict__ Fv,
                                const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double xsh[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int j = blockIdx.x * nw + w;
  if (j >= k) return;
  double *x = xsh + (int64_t)w * N;
  for (int c = lane; c < N; c += 64) x[c] = Fv[(int64_t)j * N + c];
  for (int i = N - 3; i >= 0; --i) {
    const double t = tau[i];
    if (t == 0.0) continue;
    const double *v = A + (int64_t)i * lda;
    double dot = 0.0;
    for (int c = i + 1 + lane; c < N; c += 64) dot += v[c] * x[c];
    dot = wave_sum(dot) * t;
    for (int c = i + 1 + lane; c < N; c += 64) x[c] -= dot * v[c];
  }
  for (int c = lane; c < N; c += 64) Fv[(int64_t)j * N + c] = x[c];
}

}  // namespace

namespace svl {

int eig_max_n() { return 6144; }

size_t eig_work_doubles(int64_t N, int k) {
  // d, e, tau (3N) + pbuf, rowbuf (4N) + stein scratch (6N per eigenvalue)
  return (size_t)(7 * N + 6 * N * (int64_t)k + 64);
}

int eig_topk(hipStream_t st, int64_t N64, double *A, int k, double *lam, double *Fv,
             double *work, const SvDevInfo *info) {
  const int N = (int)N64;
  if (N64 > eig_max_n() || k > N) return -1;
  double *d = work, *e = d + N, *tau = e + N, *pbuf = tau + N, *rowbuf = pbuf + 2 * N;
  double *scratch = rowbuf + 2 * N;
  static int ncu = 0;
  static bool once = false;
  if (!once) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 1;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_stein),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_backtransform),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    once = true;
  }
  int G = N / 8;
  if (G < 1) G = 1;
  if (G > ncu) G = ncu;
  const size_t sh = (size_t)3 * N * sizeof(double);
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(k_tridiag),
                                                     TRI_THREADS, sh);
  if (nb < 1) return -2;
  if (G > nb * ncu) G = nb * ncu;
  int64_t lda = N64;
  void *args[] = {(void *)&N, (void *)&A, (void *)&lda, (void *)&d, (void *)&e, (void *)&tau,
                  (void *)&pbuf, (void *)&rowbuf, (void *)&info};
  hipError_t err = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_tridiag), dim3(G),
                                              dim3(TRI_THREADS), args, sh, st);
  if (err != hipSuccess) return -3;
  hipLaunchKernelGGL(k_bisect, dim3(k), dim3(64), 0, st, N, d, e, k, lam, info);
  hipLaunchKernelGGL(k_stein, dim3(k), dim3(64), (size_t)N * sizeof(double), st, N, d, e, k,
                     lam, Fv, scratch, info);
  int wpb = (int)((150 * 1024) / ((size_t)N * sizeof(double)));
  if (wpb > 4) wpb = 4;
  if (wpb < 1) wpb = 1;
  hipLaunchKernelGGL(k_backtransform, dim3((k + wpb - 1) / wpb), dim3(64 * wpb),
                     (size_t)wpb * N * sizeof(double), st, N, k, A, lda, tau, Fv, info);
  return 0;
}

}  // namespace svl
