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

#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;
namespace cg = cooperative_groups;

namespace {

constexpr int TRI_MAX_BLOCKS = svl::TRI_MAX_BLOCKS;
constexpr double EPS = 1.1102230246251565e-16;     // 2^-53
constexpr double SAFMIN = 2.2250738585072014e-308;

// Householder tridiagonalisation, one cooperative launch (all blocks
// co-resident).  Block g owns rows r = g, g + G, ...; with LDS_ROWS they live
// in LDS for the whole reduction, otherwise in A.  Reflector i is left in row
// i of A (columns i+1 .., unit leading entry), d, e, tau in work arrays.
// NT = 64 (one wave per block: block-wide reductions and barriers are nearly
// free) for moderate N, 256 when the owned rows need more lanes.
template <bool LDS_ROWS, int NT>
__global__ void __launch_bounds__(NT)
k_tridiag(int N, double *__restrict__ A, int64_t lda, double *__restrict__ d,
          double *__restrict__ e, double *__restrict__ tau, double *__restrict__ pbuf,
          double *__restrict__ rowbuf, unsigned *__restrict__ flags, unsigned epoch0,
          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int G = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int nw = NT / 64;
  if (N < 3) {
    if (g == 0 && tid == 0) {
      d[0] = A[0];
      if (N == 2) { e[0] = A[1]; d[1] = A[lda + 1]; }
    }
    return;
  }
  double *X = sm, *VP = sm + N, *WP = sm + 2 * N;
  double *rows = sm + 3 * N;   // LDS_ROWS: owned rows, local index (r - g) / G
  if constexpr (LDS_ROWS) {
    const int nr = (N - g + G - 1) / G;
    for (int lr = w; lr < nr; lr += nw) {
      const double *src = A + (int64_t)(g + lr * G) * lda;
      for (int j = lane; j < N; j += 64) rows[(int64_t)lr * N + j] = src[j];
    }
  }
  double part = 0.0;   // sum of X[j]^2 over j >= i + 2, carried between iterations
  for (int j = tid; j < N; j += NT) {
    const double x = A[j];
    X[j] = x;
    if (j >= 2) part += x * x;
  }
  __syncthreads();
  for (int i = 0; i <= N - 3; ++i) {
    const double dii = X[i];
    // alpha is read before the reduction: its barriers order every read of
    // X[i+1] before thread 0 overwrites it with the unit leading entry
    const double alpha = X[i + 1];
    const double xn2 = NT == 64 ? wave_sum(part) : block_sum(part, red);
    double beta, t, scl;
    if (xn2 == 0.0) {
      t = 0.0; beta = alpha; scl = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xn2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scl = 1.0 / (alpha - beta);
    }
    for (int j = i + 2 + tid; j < N; j += NT) X[j] *= scl;
    if (tid == 0) X[i + 1] = 1.0;
    __syncthreads();
    double *pb = pbuf + (int64_t)(i & 1) * N;
    double *rb = rowbuf + (int64_t)(i & 1) * N;
    // owned rows r >= i+1: pending rank-2 update, then p = tau M v
    const int lr0 = (i + 1 - g + G - 1) / G > 0 ? (i + 1 - g + G - 1) / G : 0;
    for (int lr = lr0 + w; g + lr * G < N; lr += nw) {
      const int r = g + lr * G;
      double *Ar;
      if constexpr (LDS_ROWS) Ar = rows + (int64_t)lr * N;
      else Ar = A + (int64_t)r * lda;
      const double vpr = i >= 1 ? VP[r] : 0.0, wpr = i >= 1 ? WP[r] : 0.0;
      const bool pub = (r == i + 1);
      double acc = 0.0;
      for (int j = i + 1 + lane; j < N; j += 64) {
        double a = Ar[j];
        if (i >= 1) {
          a -= vpr * WP[j] + wpr * VP[j];
          Ar[j] = a;
        }
        if (pub) st_coh(&rb[j], a);
        acc += a * X[j];
      }
      acc = wave_sum(acc);
      if (lane == 0) st_coh(&pb[r], t * acc);
    }
    flag_barrier(flags, epoch0 + (unsigned)i + 1u);
    if (g == i % G) {   // row i of M is finished: keep the reflector there
      for (int j = i + 1 + tid; j < N; j += NT) A[(int64_t)i * lda + j] = X[j];
      if (tid == 0) { d[i] = dii; e[i] = beta; tau[i] = t; }
    }
    // w = p - (tau/2)(p.v) v, and the next row: published row minus update i
    double *Xn = VP;
    double part2 = 0.0;
    for (int j = i + 1 + tid; j < N; j += NT) {
      const double pj = ld_coh(&pb[j]);
      const double rj = ld_coh(&rb[j]);
      WP[j] = pj;
      Xn[j] = rj;
      part2 += pj * X[j];
    }
    const double pv = NT == 64 ? wave_sum(part2) : block_sum(part2, red);
    const double aw = -0.5 * t * pv;
    for (int j = i + 1 + tid; j < N; j += NT) WP[j] += aw * X[j];
    __syncthreads();
    const double wi1 = WP[i + 1];
    part = 0.0;
    for (int j = i + 1 + tid; j < N; j += NT) {
      const double xn = Xn[j] - (WP[j] + wi1 * X[j]);   // X[i+1] = 1
      Xn[j] = xn;
      if (j >= i + 3) part += xn * xn;
    }
    __syncthreads();
    VP = X;
    X = Xn;
  }
  if (g == 0 && tid == 0) {
    d[N - 2] = X[N - 2];
    e[N - 2] = X[N - 1];
  }
  if (g == (N - 1) % G && tid == 0) {
    double a;
    if constexpr (LDS_ROWS) a = rows[(int64_t)((N - 1 - g) / G) * N + N - 1];
    else a = A[(int64_t)(N - 1) * lda + N - 1];
    d[N - 1] = a - 2.0 * VP[N - 1] * WP[N - 1];
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
    // e^2 / q through the hardware reciprocal refined by one Newton step
    // (relative error ~1e-16, the size of a rounding error in e^2)
    double r = __builtin_amdgcn_rcp(q);
    r = r * fma(-q, r, 2.0);
    q = d[i] - x - (ei * ei) * r;
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
      double di = d[0] - lj;            // current diagonal entry of row i
      double ui = N > 1 ? e[0] : 0.0;   // current super-diagonal entry of row i
      for (int i = 0; i < N - 1; ++i) {
        const double sub = e[i];
        double dn = d[i + 1] - lj;
        double un = i < N - 2 ? e[i + 1] : 0.0;
        if (fabs(di) >= fabs(sub)) {
          const double piv = fabs(di) < tiny ? copysign(tiny, di) : di;
          const double fact = sub / piv;
          rdd[i] = 1.0 / piv;
          dl[i] = fact;
          du[i] = ui;
          du2[i] = 0.0;
          swp[i] = 0;
          dn -= fact * ui;
        } else {
          const double fact = di / sub;
          rdd[i] = 1.0 / sub;
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
      }
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
// One wave per vector, 8 vectors per block.  Reflectors are applied four at a
// time: with u_0..u_3 = v_i .. v_{i-3}, x <- x - sum_m c_m u_m where
// c_m = tau_m (u_m.x - sum_{l<m} c_l u_m.u_l), so one reduction round (4 dot
// products with x and the 6 products among the u) serves four reflectors.
// The block stages each group of four reflectors in LDS once for all its
// waves, loading the next group while the current one is applied.  Lane l
// holds x[c] for c = l + 64 m (m < R) in registers.
constexpr int BT_WAVES = 8;
template <int R>
__global__ void __launch_bounds__(64 * BT_WAVES)
k_backtransform_blk(int N, int k, const double *__restrict__ A, int64_t lda,
                    const double *__restrict__ tau, double *__restrict__ Fv,
                    const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double ub[];   // 2 buffers x 4 reflectors x N
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int j = blockIdx.x * BT_WAVES + w;
  const bool active = j < k;
  double x[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int c = lane + 64 * m;
    x[m] = (active && c < N) ? Fv[(int64_t)j * N + c] : 0.0;
  }
  const int ngroups = (N - 2 + 3) / 4;   // reflectors N-3 .. 0 in groups of 4
  // group g holds reflectors i0 - q, q = 0..3, with i0 = N - 3 - 4 g
  constexpr int NTH = 64 * BT_WAVES;
  constexpr int PER = (4 * 64 * R + NTH - 1) / NTH;   // staged values per thread
  auto fetch = [&](int grp, double *pre) {
    const int i0 = N - 3 - 4 * grp;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = tid + p * NTH;
      double v = 0.0;
      if (e < 4 * N) {
        const int q = e / N, c = e % N, i = i0 - q;
        if (i >= 0 && c > i) v = A[(int64_t)i * lda + c];
      }
      pre[p] = v;
    }
  };
  auto stash = [&](const double *pre, double *dst) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = tid + p * NTH;
      if (e < 4 * N) dst[e] = pre[p];
    }
  };
  double pre[PER];
  fetch(0, pre);
  stash(pre, ub);
  __syncthreads();
  for (int grp = 0; grp < ngroups; ++grp) {
    double *cur = ub + (size_t)(grp & 1) * 4 * N;
    double *nxt = ub + (size_t)((grp + 1) & 1) * 4 * N;
    const bool more = grp + 1 < ngroups;
    if (more) fetch(grp + 1, pre);
    const int i0 = N - 3 - 4 * grp;
    double t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = (i0 - q >= 0) ? tau[i0 - q] : 0.0;
    double a[4] = {0, 0, 0, 0}, g10 = 0, g20 = 0, g21 = 0, g30 = 0, g31 = 0, g32 = 0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int c = lane + 64 * m;
      if (c < N) {
        const double u0 = cur[c], u1 = cur[N + c], u2 = cur[2 * N + c], u3 = cur[3 * N + c];
        a[0] += u0 * x[m]; a[1] += u1 * x[m]; a[2] += u2 * x[m]; a[3] += u3 * x[m];
        g10 += u1 * u0; g20 += u2 * u0; g21 += u2 * u1;
        g30 += u3 * u0; g31 += u3 * u1; g32 += u3 * u2;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a[0] += __shfl_xor(a[0], o, 64); a[1] += __shfl_xor(a[1], o, 64);
      a[2] += __shfl_xor(a[2], o, 64); a[3] += __shfl_xor(a[3], o, 64);
      g10 += __shfl_xor(g10, o, 64); g20 += __shfl_xor(g20, o, 64);
      g21 += __shfl_xor(g21, o, 64); g30 += __shfl_xor(g30, o, 64);
      g31 += __shfl_xor(g31, o, 64); g32 += __shfl_xor(g32, o, 64);
    }
    const double c0 = t[0] * a[0];
    const double c1 = t[1] * (a[1] - c0 * g10);
    const double c2 = t[2] * (a[2] - c0 * g20 - c1 * g21);
    const double c3 = t[3] * (a[3] - c0 * g30 - c1 * g31 - c2 * g32);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int c = lane + 64 * m;
      if (c < N)
        x[m] -= c0 * cur[c] + c1 * cur[N + c] + c2 * cur[2 * N + c] + c3 * cur[3 * N + c];
    }
    if (more) stash(pre, nxt);
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int c = lane + 64 * m;
      if (c < N) Fv[(int64_t)j * N + c] = x[m];
    }
  }
}

// Register variant for N <= 64 R: one wave per vector (one block each),
// reflectors applied two at a time (u_0 = v_i, u_1 = v_{i-1}:
// c_0 = tau_0 u_0.x, c_1 = tau_1 (u_1.x - c_0 u_1.u_0), x -= c_0 u_0 + c_1 u_1),
// the next pair loaded into registers while the current one is applied.
template <int R>
__global__ void __launch_bounds__(64)
k_backtransform_pair(int N, int k, const double *__restrict__ A, int64_t lda,
                     const double *__restrict__ tau, double *__restrict__ Fv,
                     const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x;
  const int j = blockIdx.x;
  double x[R], u0[R], u1[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int c = lane + 64 * m;
    x[m] = c < N ? Fv[(int64_t)j * N + c] : 0.0;
  }
  auto fetch = [&](int i, double *u) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int c = lane + 64 * m;
      u[m] = (i >= 0 && c > i && c < N) ? A[(int64_t)i * lda + c] : 0.0;
    }
  };
  int i = N - 3;
  fetch(i, u0);
  fetch(i - 1, u1);
  for (; i >= 0; i -= 2) {
    double v0[R], v1[R];
#pragma unroll
    for (int m = 0; m < R; ++m) { v0[m] = u0[m]; v1[m] = u1[m]; }
    const double t0 = tau[i];
    const double t1 = i >= 1 ? tau[i - 1] : 0.0;
    if (i >= 2) {
      fetch(i - 2, u0);
      fetch(i - 3, u1);
    }
    double a0 = 0.0, a1 = 0.0, g = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      a0 += v0[m] * x[m];
      a1 += v1[m] * x[m];
      g += v1[m] * v0[m];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
      g += __shfl_xor(g, o, 64);
    }
    const double c0 = t0 * a0;
    const double c1 = t1 * (a1 - c0 * g);
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] -= c0 * v0[m] + c1 * v1[m];
  }
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int c = lane + 64 * m;
    if (c < N) Fv[(int64_t)j * N + c] = x[m];
  }
}

// General-N variant with the vector in LDS.
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

__global__ void k_zero_u32(unsigned *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

namespace svl {

int eig_max_n() { return 6144; }

size_t eig_work_doubles(int64_t N, int k) {
  // d, e, tau (3N) + pbuf, rowbuf (4N) + inverse-iteration scratch (7N per
  // eigenvalue, used when the factors do not fit in LDS)
  return (size_t)(7 * N + 7 * N * (int64_t)k + 64);
}

// Work layout: d, e, tau (3N), pbuf, rowbuf (4N), inverse-iteration scratch.
// flags: TRI_MAX_BLOCKS * FLAG_STRIDE unsigned, zero-initialised once; *epoch
// is advanced past the epochs this launch uses.
int eig_tridiag(hipStream_t st, int64_t N64, double *A, double *work, unsigned *flags,
                unsigned *epoch, const SvDevInfo *info) {
  const int N = (int)N64;
  if (N64 > eig_max_n() || N < 1) return -1;
  double *d = work, *e = d + N, *tau = e + N, *pbuf = tau + N, *rowbuf = pbuf + 2 * N;
  static int ncu = 0;
  static bool once = false;
  if (!once) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 1;
    if (ncu > TRI_MAX_BLOCKS) ncu = TRI_MAX_BLOCKS;
    const int lim = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag<true, 64>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag<false, 64>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag<true, 256>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag<false, 256>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_stein<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_backtransform),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipGetLastError();
    once = true;
  }
  // launch shape: block width NT (64 or 256 threads) and block count G; the
  // defaults come from a sweep on MI355X, SVLCOV_TRI_THREADS / _BLOCKS
  // override them for tuning
  bool wide = true;
  int G = N / 4;
  if (const char *ev = getenv("SVLCOV_TRI_THREADS")) wide = atoi(ev) != 64;
  if (const char *ev = getenv("SVLCOV_TRI_BLOCKS")) G = atoi(ev);
  const int NT = wide ? 256 : 64;
  if (G < 1) G = 1;
  if (G > ncu) G = ncu;
  const int rmax = (N + G - 1) / G;
  const size_t base_sh = (size_t)3 * N * sizeof(double);
  const size_t rows_sh = (size_t)rmax * N * sizeof(double);
  const bool lds_rows = base_sh + rows_sh <= (size_t)150 * 1024;
  const size_t sh = lds_rows ? base_sh + rows_sh : base_sh;
  const void *fn;
  if (wide) fn = lds_rows ? reinterpret_cast<const void *>(k_tridiag<true, 256>)
                          : reinterpret_cast<const void *>(k_tridiag<false, 256>);
  else fn = lds_rows ? reinterpret_cast<const void *>(k_tridiag<true, 64>)
                     : reinterpret_cast<const void *>(k_tridiag<false, 64>);
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, sh);
  (void)hipGetLastError();
  if (nb < 1) return -2;
  if (G > nb * ncu) G = nb * ncu;
  if (*epoch > 0xF0000000u) {   // keep epochs monotonic: restart from zero
    hipLaunchKernelGGL(k_zero_u32, dim3(16), dim3(256), 0, st, flags,
                       (size_t)TRI_MAX_BLOCKS * FLAG_STRIDE);
    *epoch = 0;
  }
  unsigned e0 = *epoch;
  *epoch += (unsigned)N + 1u;
  int64_t lda = N64;
  void *args[] = {(void *)&N, (void *)&A, (void *)&lda, (void *)&d, (void *)&e, (void *)&tau,
                  (void *)&pbuf, (void *)&rowbuf, (void *)&flags, (void *)&e0, (void *)&info};
  hipError_t err = hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, sh, st);
  return err == hipSuccess ? 0 : -3;
}

void eig_bisect(hipStream_t st, int64_t N, int k, double *lam, double *work,
                const SvDevInfo *info) {
  const double *d = work, *e = work + N;
  hipLaunchKernelGGL(k_bisect, dim3(k), dim3(64), 0, st, (int)N, d, e, k, lam, info);
}

void eig_stein(hipStream_t st, int64_t N, int k, const double *lam, double *Fv, double *work,
               const SvDevInfo *info) {
  const double *d = work, *e = work + N;
  double *scratch = work + 7 * N;
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
  const double *tau = work + 2 * N;
  const int n = (int)N;
  if (N >= 3 && N <= 64 * 24) {
#define SV_BP(RR) hipLaunchKernelGGL((k_backtransform_pair<RR>), dim3(k), dim3(64), 0, st, n, k, A, N, tau, Fv, info)
    if (N <= 64 * 4) SV_BP(4);
    else if (N <= 64 * 8) SV_BP(8);
    else if (N <= 64 * 12) SV_BP(12);
    else if (N <= 64 * 16) SV_BP(16);
    else if (N <= 64 * 20) SV_BP(20);
    else SV_BP(24);
#undef SV_BP
    return;
  }
  if (N >= 3 && N <= 64 * 32) {
    static bool once = false;
    if (!once) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_backtransform_blk<32>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      once = true;
    }
    const unsigned blocks = (unsigned)((k + BT_WAVES - 1) / BT_WAVES);
    const size_t sh = (size_t)8 * N * sizeof(double);
    hipLaunchKernelGGL((k_backtransform_blk<32>), dim3(blocks), dim3(64 * BT_WAVES), sh, st, n, k,
                       A, N, tau, Fv, info);
    return;
  }
  int wpb = (int)((150 * 1024) / ((size_t)N * sizeof(double)));
  if (wpb > 4) wpb = 4;
  if (wpb < 1) wpb = 1;
  hipLaunchKernelGGL(k_backtransform, dim3((k + wpb - 1) / wpb), dim3(64 * wpb),
                     (size_t)wpb * N * sizeof(double), st, n, k, A, N, tau, Fv, info);
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
