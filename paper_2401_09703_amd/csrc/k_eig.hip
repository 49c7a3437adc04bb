// Top-k eigenpairs of a symmetric FP64 matrix on the GPU, the core of the
// (k+s) Rayleigh-Ritz SVD (Section 2.1, step 2): the left singular vectors of
// K are the eigenvectors of K K^T and its eigenvalues are the squared singular
// values.
//
//   1. Householder tridiagonalisation Q^T M Q = T (its own source file).
//   2. Bisection on Sturm counts for the k largest eigenvalues of T, one block
//      per eigenvalue with 513-way multisection.
//   3. Inverse iteration with the eigenvalue as shift (tridiagonal LU with
//      partial pivoting), re-orthogonalised inside clusters of close
//      eigenvalues.
//   4. Back-transformation of the k vectors by the stored reflectors, in
//      panels of 32 reflectors in compact WY form.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

constexpr double EPS = 1.1102230246251565e-16;     // 2^-53
constexpr double SAFMIN = 2.2250738585072014e-308;

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

// Number of eigenvalues of T below x (Sturm count of the LDL^T recurrence
// q_i = d_i - x - e_{i-1}^2 / q_{i-1}); d and e2 = e^2 are in LDS.
__device__ __forceinline__ int sturm_count(int N, const double *__restrict__ d,
                                           const double *__restrict__ e2, double x,
                                           double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q <= 0.0;
#pragma unroll 8
  for (int i = 1; i < N; ++i) {
    // e^2 / q through the hardware reciprocal refined by one Newton step
    // (relative error ~1e-16, the size of a rounding error in e^2)
    double r = __builtin_amdgcn_rcp(q);
    r = r * fma(-q, r, 2.0);
    q = d[i] - x - e2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q <= 0.0;
  }
  return cnt;
}

// lam[j] = the (N-1-j)-th smallest eigenvalue of T (so lam is descending).
// One block of BIS_NT threads per eigenvalue; each round evaluates BIS_NT
// shifts (one per thread) that split the current interval into BIS_NT + 1
// parts, so an FP64 eigenvalue is found in about seven rounds.  256 shifts
// (one wave per SIMD) measured faster on MI355X than 128 (more rounds) and
// than 512 or 1024 (the Sturm recurrences of several waves share a SIMD).
constexpr int BIS_NT = 256;

__global__ void __launch_bounds__(BIS_NT)
k_bisect(int N, const double *__restrict__ d, const double *__restrict__ e, int k,
         double *__restrict__ lam, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double bsm[];
  __shared__ unsigned long long masks[BIS_NT / 64];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (j >= k) return;
  double *sd = bsm, *se2 = bsm + N;
  for (int i = tid; i < N; i += BIS_NT) {
    sd[i] = d[i];
    se2[i] = i < N - 1 ? e[i] * e[i] : 0.0;
  }
  const int idx = N - 1 - j;
  double gl, gu, onenrm, emax2;
  tri_bounds(N, d, e, gl, gu, onenrm, emax2);
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = SAFMIN * fmax(1.0, emax2);
  gl -= 2.0 * EPS * tnorm * N + 4.0 * pivmin;
  gu += 2.0 * EPS * tnorm * N + 4.0 * pivmin;
  __syncthreads();
  constexpr double PARTS = (double)(BIS_NT + 1);
  double lo = gl, hi = gu;
  for (int round = 0; round < 40; ++round) {
    const double tol = 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin;
    if (hi - lo <= tol) break;
    const double h = hi - lo;
    const double x = lo + h * (double)(tid + 1) / PARTS;
    const int cnt = sturm_count(N, sd, se2, x, pivmin);
    const unsigned long long m = __ballot(cnt > idx);
    if (lane == 0) masks[w] = m;
    __syncthreads();
    // the first shift f whose count exceeds idx brackets the eigenvalue
    // between shifts f-1 and f; every thread forms the same shifts
    int f = BIS_NT;
    for (int q = 0; q < BIS_NT / 64; ++q)
      if (masks[q]) { f = 64 * q + __builtin_ctzll(masks[q]); break; }
    __syncthreads();
    const double nlo = f > 0 ? lo + h * (double)f / PARTS : lo;
    const double nhi = f < BIS_NT ? lo + h * (double)(f + 1) / PARTS : hi;
    lo = nlo;
    hi = nhi;
  }
  if (tid == 0) lam[j] = 0.5 * (lo + hi);
}

// Inverse iteration for the clusters of lam (descending).  One wave per
// cluster leader; members of a cluster are computed in order and
// re-orthogonalised against the earlier members after every solve.  The
// tridiagonal LU with partial pivoting of T - lambda I and the two triangular
// solves are sequential (lane 0) with the recurrences carried in registers;
// the factors live in LDS when they fit (IN_LDS), otherwise in scratch.
template <bool IN_LDS>
__global__ void __launch_bounds__(64)
k_stein(int N, const double *__restrict__ d, const double *__restrict__ e, int k,
        const double *__restrict__ lam, double *__restrict__ Fv, double *__restrict__ scratch,
        const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double shm[];
  const int j0 = blockIdx.x, lane = threadIdx.x;
  double gl, gu, onenrm, emax2;
  tri_bounds(N, d, e, gl, gu, onenrm, emax2);
  // Inverse iteration from an eigenvalue accurate to eps*||T|| gives a vector
  // whose angle to the true one is about eps*||T|| / gap, so independent
  // iterations stay orthogonal to ~1e-7 or better unless two eigenvalues are
  // closer than 1e-9*||T||; only such clusters are orthogonalised in turn.
  const double ortol = 1e-9 * onenrm;
  if (j0 > 0 && lam[j0 - 1] - lam[j0] <= ortol) return;   // not a leader
  int j1 = j0 + 1;
  while (j1 < k && lam[j1 - 1] - lam[j1] <= ortol) ++j1;
  double *base = IN_LDS ? shm : scratch + (int64_t)j0 * 7 * N;
  double *__restrict__ xs = base;
  double *__restrict__ rdd = base + N;     // reciprocals of the U diagonal
  double *__restrict__ dl = base + 2 * N;
  double *__restrict__ du = base + 3 * N;
  double *__restrict__ du2 = base + 4 * N;
  int *__restrict__ swp = (int *)(base + 5 * N);
  const double tiny = fmax(EPS * onenrm, 1e-290);
  for (int j = j0; j < j1; ++j) {
    const double lj = lam[j];
    if (onenrm == 0.0) {
      for (int c = lane; c < N; c += 64) Fv[(int64_t)j * N + c] = (c == j) ? 1.0 : 0.0;
      continue;
    }
    if (lane == 0) {
      // The elimination is a chain through di: its entries are loaded 8
      // steps ahead (they do not depend on it), and each step takes one
      // reciprocal (hardware reciprocal refined by one Newton step, relative
      // error ~1e-16) instead of two divisions.
      double di = d[0] - lj;            // current diagonal entry of row i
      double ui = N > 1 ? e[0] : 0.0;   // current super-diagonal entry of row i
      auto step = [&](int i, double sub, double dn, double un) {
        if (fabs(di) >= fabs(sub)) {
          const double piv = fabs(di) < tiny ? copysign(tiny, di) : di;
          double r = __builtin_amdgcn_rcp(piv);
          r = r * fma(-piv, r, 2.0);
          const double fact = sub * r;
          rdd[i] = r;
          dl[i] = fact;
          du[i] = ui;
          du2[i] = 0.0;
          swp[i] = 0;
          dn -= fact * ui;
        } else {
          double r = __builtin_amdgcn_rcp(sub);
          r = r * fma(-sub, r, 2.0);
          const double fact = di * r;
          rdd[i] = r;
          dl[i] = fact;
          du[i] = dn;
          du2[i] = un;
          swp[i] = 1;
          const double t2 = ui - fact * dn;
          un = -fact * un;
          dn = t2;
        }
        di = dn;
        ui = un;
      };
      int i = 0;
      for (; i + 8 <= N - 1; i += 8) {
        double sb[8], dn8[8], un8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          sb[q] = e[i + q];
          dn8[q] = d[i + q + 1] - lj;
          un8[q] = (i + q < N - 2) ? e[i + q + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) step(i + q, sb[q], dn8[q], un8[q]);
      }
      for (; i < N - 1; ++i) step(i, e[i], d[i + 1] - lj, i < N - 2 ? e[i + 1] : 0.0);
      const double piv = fabs(di) < tiny ? copysign(tiny, di) : di;
      rdd[N - 1] = 1.0 / piv;
    }
    for (int c = lane; c < N; c += 64)
      xs[c] = hash_unit(0x5bd1e995ull * (uint64_t)(j + 1) + (uint64_t)c * 0x9E3779B97F4A7C15ull);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (lane == 0) {
        // forward: L with the row interchanges, in batches of 8 so that the
        // loads of a batch are in flight together
        double cur = xs[0];
        int i = 0;
        for (; i + 8 <= N - 1; i += 8) {
          double nx[8], l[8];
          int sw[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) { nx[q] = xs[i + q + 1]; l[q] = dl[i + q]; sw[q] = swp[i + q]; }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double o = sw[q] ? nx[q] : cur;
            cur = sw[q] ? (cur - l[q] * nx[q]) : (nx[q] - l[q] * cur);
            xs[i + q] = o;
          }
        }
        for (; i < N - 1; ++i) {
          const double nxt = xs[i + 1];
          const double o = swp[i] ? nxt : cur;
          cur = swp[i] ? (cur - dl[i] * nxt) : (nxt - dl[i] * cur);
          xs[i] = o;
        }
        // backward: U x = b
        double b1 = cur * rdd[N - 1];   // b[i+1]
        xs[N - 1] = b1;
        double b2 = 0.0;                 // b[i+2]
        i = N - 2;
        for (; i - 7 >= 0; i -= 8) {
          double xv[8], u[8], u2[8], r[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            xv[q] = xs[i - q]; u[q] = du[i - q];
            u2[q] = (i - q < N - 2) ? du2[i - q] : 0.0; r[q] = rdd[i - q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double bi = (xv[q] - u[q] * b1 - u2[q] * b2) * r[q];
            xs[i - q] = bi;
            b2 = b1;
            b1 = bi;
          }
        }
        for (; i >= 0; --i) {
          const double bi = (xs[i] - du[i] * b1 - (i < N - 2 ? du2[i] * b2 : 0.0)) * rdd[i];
          xs[i] = bi;
          b2 = b1;
          b1 = bi;
        }
      }
      __syncthreads();
      // against the earlier members of the cluster, twice: one pass leaves
      // an error of the order of u times the cancellation, which for a
      // (near-)degenerate cluster can be all of the vector
      for (int pass = 0; pass < (j > j0 ? 2 : 0); ++pass)
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

// Blocked back-transformation (compact WY form).  The reflectors are taken
// in panels of WB: H_i0 H_i0+1 ... H_i0+nb-1 = I - Y T Y^T with Y the panel's
// reflector vectors as columns and T upper triangular (forward accumulation:
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (Y[:, 0:j]^T y_j)).
constexpr int WB = 32;

__global__ void __launch_bounds__(256)
k_wy_tfactor(int N, const double *__restrict__ A, int64_t lda, const double *__restrict__ tau,
             double *__restrict__ Tws, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double Ych[WB][65];
  __shared__ double Gs[WB][WB + 1];
  __shared__ double Ts[WB][WB + 1];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int i0 = p * WB;
  const int nb = min(WB, N - 2 - i0);
  // Gram of the panel, 4 entries per thread: (a0 + 8q, b)
  const int a0 = tid >> 5, b = tid & 31;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = i0 + 1; c0 < N; c0 += 64) {
    // loads at clamped (always valid) addresses, masked afterwards
#pragma unroll
    for (int e = tid; e < WB * 64; e += 256) {
      const int a = e >> 6, c = c0 + (e & 63);
      const double v = A[(int64_t)min(i0 + a, N - 1) * lda + min(c, N - 1)];
      Ych[a][e & 63] = (a < nb && c < N && c >= i0 + a + 1) ? v : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
      for (int cc = 0; cc < 64; ++cc) acc[q] += Ych[a0 + 8 * q][cc] * Ych[b][cc];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Gs[a0 + 8 * q][b] = acc[q];
    Ts[a0 + 8 * q][b] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = tau[i0 + j];
    double v = 0.0;
    if (tid < j)
      for (int c = tid; c < j; ++c) v += Ts[tid][c] * Gs[c][j];
    __syncthreads();
    if (tid < j) Ts[tid][j] = -tj * v;
    if (tid == j) Ts[j][j] = tj;
    __syncthreads();
  }
  for (int e = tid; e < WB * WB; e += 256) Tws[(int64_t)p * WB * WB + e] = Ts[e / WB][e % WB];
}

// x <- H_0 H_1 ... H_{N-3} x for each eigenvector x (one block per vector,
// x in LDS), panel by panel from the last: z = Y^T x, z <- T z, x -= Y z.
// The 32 partial dot products of a thread are reduced across the wave by a
// halving exchange (32 shuffles instead of 32 full reductions).
template <int NT>
__global__ void __launch_bounds__(NT)
k_backtransform_wy(int N, int k, const double *__restrict__ A, int64_t lda,
                   const double *__restrict__ Tws, double *__restrict__ Fv,
                   const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double xs[];
  __shared__ double red[NT / 64][WB];
  __shared__ double zs[WB], zt[WB];
  __shared__ double Ts[WB][WB + 1];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (j >= k) return;
  for (int c = tid; c < N; c += NT) xs[c] = Fv[(int64_t)j * N + c];
  const int nr = N - 2;
  const int nP = nr > 0 ? (nr + WB - 1) / WB : 0;
  __syncthreads();
  for (int p = nP - 1; p >= 0; --p) {
    const int i0 = p * WB;
    const int nb = min(WB, nr - i0);
    for (int e = tid; e < WB * WB; e += NT) Ts[e / WB][e % WB] = Tws[(int64_t)p * WB * WB + e];
    const double *Yp = A + (int64_t)i0 * lda;
    const int amax = N - 1 - i0;   // rows i0 + a beyond the matrix are clamped
    double zp[WB];
#pragma unroll
    for (int a = 0; a < WB; ++a) zp[a] = 0.0;
    for (int c = i0 + 1 + tid; c < N; c += NT) {
      const double xc = xs[c];
      double yv[WB];
#pragma unroll
      for (int a = 0; a < WB; ++a) yv[a] = Yp[(int64_t)min(a, amax) * lda + c];
#pragma unroll
      for (int a = 0; a < WB; ++a)
        zp[a] += ((a < nb && c >= i0 + a + 1) ? yv[a] : 0.0) * xc;
    }
    // halving exchange: after the step with offset o, a lane keeps the half
    // of the values selected by its bit o; finally lane l holds index l >> 1
#pragma unroll
    for (int o = 32, n = WB; o >= 2; o >>= 1, n >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < n / 2; ++i) {
        const double send = up ? zp[i] : zp[i + n / 2];
        const double keep = up ? zp[i + n / 2] : zp[i];
        zp[i] = keep + __shfl_xor(send, o, 64);
      }
    }
    const double tot = zp[0] + __shfl_xor(zp[0], 1, 64);
    if ((lane & 1) == 0) red[w][lane >> 1] = tot;
    __syncthreads();
    if (tid < WB) {
      double sacc = 0.0;
      for (int q = 0; q < NT / 64; ++q) sacc += red[q][tid];
      zs[tid] = sacc;
    }
    __syncthreads();
    if (tid < WB) {
      double sacc = 0.0;
      for (int c = tid; c < WB; ++c) sacc += Ts[tid][c] * zs[c];
      zt[tid] = sacc;
    }
    __syncthreads();
    for (int c = i0 + 1 + tid; c < N; c += NT) {
      double yv[WB];
#pragma unroll
      for (int a = 0; a < WB; ++a) yv[a] = Yp[(int64_t)min(a, amax) * lda + c];
      double sacc = 0.0;
#pragma unroll
      for (int a = 0; a < WB; ++a)
        sacc += ((a < nb && c >= i0 + a + 1) ? yv[a] : 0.0) * zt[a];
      xs[c] -= sacc;
    }
    __syncthreads();
  }
  for (int c = tid; c < N; c += NT) Fv[(int64_t)j * N + c] = xs[c];
}

}  // namespace

namespace svl {

int eig_max_n() { return 6144; }

size_t eig_work_doubles(int64_t N, int k) {
  // d, e, tau (3N) + pbuf, rowbuf (4N) + inverse-iteration scratch (7N per
  // eigenvalue, used when the factors do not fit in LDS) + the T factors of
  // the reflector panels (WB x WB per panel)
  return (size_t)(7 * N + 7 * N * (int64_t)k + (N / WB + 1) * WB * WB + 64);
}

void eig_bisect(hipStream_t st, int64_t N, int k, double *lam, double *work,
                const SvDevInfo *info) {
  const double *d = work, *e = work + N;
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_bisect),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  hipLaunchKernelGGL(k_bisect, dim3(k), dim3(BIS_NT), (size_t)2 * N * sizeof(double), st,
                     (int)N, d, e, k, lam, info);
}

void eig_stein(hipStream_t st, int64_t N, int k, const double *lam, double *Fv, double *work,
               const SvDevInfo *info) {
  const double *d = work, *e = work + N;
  double *scratch = work + 7 * N;
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_stein<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  const size_t sh = (size_t)N * 6 * sizeof(double) + (size_t)N * sizeof(int) + 64;
  if (sh <= (size_t)150 * 1024)
    hipLaunchKernelGGL((k_stein<true>), dim3(k), dim3(64), sh, st, (int)N, d, e, k, lam, Fv,
                       scratch, info);
  else
    hipLaunchKernelGGL((k_stein<false>), dim3(k), dim3(64), 0, st, (int)N, d, e, k, lam, Fv,
                       scratch, info);
}

void eig_back(hipStream_t st, int64_t N, int k, const double *A, double *Fv, double *work,
              const SvDevInfo *info) {
  if (N < 3) return;
  const double *tau = work + 2 * N;
  double *Tws = work + 7 * N + 7 * N * (int64_t)k;
  const int n = (int)N;
  const int nP = (n - 2 + WB - 1) / WB;
  hipLaunchKernelGGL(k_wy_tfactor, dim3(nP), dim3(256), 0, st, n, A, N, tau, Tws, info);
  // 512 threads a vector: 15 % faster than 256 at N = 1064 (measured)
  hipLaunchKernelGGL((k_backtransform_wy<512>), dim3(k), dim3(512), (size_t)N * sizeof(double),
                     st, n, k, A, N, Tws, Fv, info);
}

int eig_topk(hipStream_t st, int64_t N, double *A, int k, double *lam, double *Fv,
             double *work, unsigned *flags, unsigned *epoch, const SvDevInfo *info) {
  if (k > N) return -1;
  const int r = eig_tridiag(st, N, A, work, flags, epoch, info);
  if (r != 0) return r;
  eig_bisect(st, N, k, lam, work, info);
  eig_stein(st, N, k, lam, Fv, work, info);
  eig_back(st, N, k, A, Fv, work, info);
  return 0;
}

}  // namespace svl
