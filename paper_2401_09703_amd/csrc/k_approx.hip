// Kernels of the -GKL and -RPI variants (the paper's appendix on approximating
// the augmented space).  Both work in the coefficient space of the update: a
// vector of the augmented space is q = Z y with y in R^s, so every product
// with Z or Z^T reduces to the residual Gram G = Z^T Z = E E^T - (EV)(EV)^T
// (Lemma 3), the s x s FP64 matrix the exact path also forms.
//   GKL  q_i = Z y_i with y_i = (p_i - beta_{i-1} y_{i-1}) / alpha_i,
//        alpha_i^2 = y^T G y, Z^T q_i = G y_i, the next p from G y_i - alpha_i p_i
//        orthogonalised against all previous p.
//   RPI  P <- orth(P); X = G P (the rows of P are coefficient vectors);
//        Q = Z P L^{-T} from the Cholesky factor L of P^T G P; Z^T Q = X L^{-T}.
#include "common.hpp"
#include "kernels.hpp"
#include "svlcov.h"

using namespace svk;

namespace {

constexpr int AP_NT = 1024;   // single-block kernels
using svl::AP_LMAX;

// The strict upper triangle of G receives the lower one (s x s, stride ld).
// Block (tj, ti) with tj <= ti reads tile (ti, tj) of the lower part and
// writes its transpose into the strict upper part; no tile is both read and
// written by different blocks.
__global__ void __launch_bounds__(256)
k_sym_lower(int64_t s, double *__restrict__ G, int64_t ld, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = ti * 32 + r, j = tj * 32 + tx;
    t[r][tx] = (i < s && j < s) ? G[i * ld + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = tj * 32 + r, j = ti * 32 + tx;   // destination, j > i
    if (i < s && j < s && j > i) G[i * ld + j] = t[tx][r];
  }
}

// Y[j] = G X[j] for the NV rows of X (each s long): one wave per row of G,
// which is read once for all NV vectors.
template <int NV>
__global__ void __launch_bounds__(256)
k_symv_multi(int64_t s, const double *__restrict__ G, int64_t ld, const double *__restrict__ X,
             double *__restrict__ Y, const int32_t *__restrict__ brk,
             const SvDevInfo *__restrict__ info) {
  if (info->status || (brk && *brk)) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= s) return;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const double *g = G + r * ld;
  for (int64_t c0 = 0; c0 < s; c0 += 256) {
    double gv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = c0 + u * 64 + lane;
      gv[u] = c < s ? g[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = c0 + u * 64 + lane;
      if (c < s) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += gv[u] * X[(int64_t)j * s + c];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) Y[(int64_t)j * s + r] = v;
  }
}

__device__ __forceinline__ double blk_dot(const double *a, const double *b, int64_t s,
                                          double *red) {
  double v = 0.0;
  for (int64_t e = threadIdx.x; e < s; e += blockDim.x) v += a[e] * b[e];
  return block_sum(v, red);
}

// GKL start: p_1 = start / ||start|| (all ones when start is NULL), y_1 = p_1;
// the other rows of P (l + 1 of them) and of Y (l), alpha, beta are zeroed.
__global__ void __launch_bounds__(AP_NT)
k_gkl_init(int64_t s, int l, const double *__restrict__ start, double *__restrict__ Pv,
           double *__restrict__ Yc, double *__restrict__ ab, int32_t *__restrict__ brk,
           SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double red[AP_NT / 64];
  double v = 0.0;
  for (int64_t e = threadIdx.x; e < s; e += blockDim.x) {
    const double x = start ? start[e] : 1.0;
    v += x * x;
  }
  const double nrm2 = block_sum(v, red);
  if (!(nrm2 > 0.0) || !isfinite(nrm2)) {
    if (threadIdx.x == 0) atomicCAS(&info->status, 0, (int)SVLCOV_E_INVALID);
    return;
  }
  const double inv = 1.0 / sqrt(nrm2);
  for (int64_t e = threadIdx.x; e < s; e += blockDim.x) {
    const double p = (start ? start[e] : 1.0) * inv;
    Pv[e] = p;
    Yc[e] = p;
  }
  for (int64_t e = s + threadIdx.x; e < (int64_t)(l + 1) * s; e += blockDim.x) Pv[e] = 0.0;
  for (int64_t e = s + threadIdx.x; e < (int64_t)l * s; e += blockDim.x) Yc[e] = 0.0;
  for (int e = threadIdx.x; e < 2 * AP_LMAX; e += blockDim.x) ab[e] = 0.0;
  if (threadIdx.x == 0) *brk = 0;
}

// One GKL step after g = G y_i (y_i unnormalised in Yc[i]).  Breakdown (a
// squared coefficient at or below rtol * info->scale, the largest squared row
// norm of E: the pivot rule of the Cholesky) stops the process; the rows not
// yet written stay zero.
__global__ void __launch_bounds__(AP_NT)
k_gkl_step(int64_t s, int i, int l, double *__restrict__ Pv, double *__restrict__ Yc,
           double *__restrict__ g, double *__restrict__ ab, int32_t *__restrict__ brk,
           double rtol, const SvDevInfo *__restrict__ info) {
  if (info->status || *brk) return;
  __shared__ double red[AP_NT / 64];
  __shared__ double cj[AP_LMAX + 1];
  const double thr = sqrt(rtol * fmax(info->scale, 0.0));
  double *y = Yc + (int64_t)i * s;
  const double a2 = blk_dot(y, g, s, red);
  const double a = sqrt(fmax(a2, 0.0));
  if (!(a > thr)) {
    for (int64_t e = threadIdx.x; e < s; e += blockDim.x) y[e] = 0.0;
    if (threadIdx.x == 0) *brk = 1;
    return;
  }
  const double ia = 1.0 / a;
  const double *pi = Pv + (int64_t)i * s;
  double *pn = Pv + (int64_t)(i + 1) * s;
  for (int64_t e = threadIdx.x; e < s; e += blockDim.x) {
    y[e] *= ia;
    pn[e] = g[e] * ia - a * pi[e];
  }
  __syncthreads();
  // two passes of classical Gram-Schmidt against p_1 .. p_i; the i + 1 dot
  // products of a pass are reduced together (per-wave sums in LDS, one
  // barrier, then one thread per product sums the waves)
  __shared__ double wred[AP_NT / 64][AP_LMAX + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j <= i; ++j) {
      const double *pj = Pv + (int64_t)j * s;
      double v = 0.0;
      for (int64_t e = threadIdx.x; e < s; e += blockDim.x) v += pj[e] * pn[e];
      v = wave_sum(v);
      if (lane == 0) wred[wv][j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x <= i) {
      double c = 0.0;
      for (int q = 0; q < AP_NT / 64; ++q) c += wred[q][threadIdx.x];
      cj[threadIdx.x] = c;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < s; e += blockDim.x) {
      double v = pn[e];
      for (int j = 0; j <= i; ++j) v -= cj[j] * Pv[(int64_t)j * s + e];
      pn[e] = v;
    }
    __syncthreads();
  }
  const double b = sqrt(fmax(blk_dot(pn, pn, s, red), 0.0));
  if (threadIdx.x == 0) ab[i] = a;
  if (!(b > thr)) {
    for (int64_t e = threadIdx.x; e < s; e += blockDim.x) pn[e] = 0.0;
    if (threadIdx.x == 0) *brk = 1;
    return;
  }
  const double ib = 1.0 / b;
  double *yn = Yc + (int64_t)(i + 1) * s;
  for (int64_t e = threadIdx.x; e < s; e += blockDim.x) {
    const double p = pn[e] * ib;
    pn[e] = p;
    if (i + 1 < l) yn[e] = p - b * y[e];
  }
  if (threadIdx.x == 0) ab[AP_LMAX + i] = b;
}

// K block of the augmented side: K[row0 + t][col0 + i] = alpha_i p_i[t] +
// beta_i p_{i+1}[t]  (P = P_{l+1} H^T).
__global__ void k_gkl_pblock(int64_t s, int l, const double *__restrict__ Pv,
                             const double *__restrict__ ab, double *__restrict__ Kout,
                             int64_t ldk, int64_t row0, int64_t col0,
                             const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * l) return;
  const int64_t t = e / l;
  const int i = (int)(e % l);
  Kout[(row0 + t) * ldk + col0 + i] =
      ab[i] * Pv[(int64_t)i * s + t] + ab[AP_LMAX + i] * Pv[(int64_t)(i + 1) * s + t];
}

// K block from rows: K[row0 + t][col0 + i] = X[i][t].
__global__ void k_rows_to_block(int64_t s, int l, const double *__restrict__ X,
                                double *__restrict__ Kout, int64_t ldk, int64_t row0,
                                int64_t col0, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * l) return;
  const int64_t t = e / l;
  const int i = (int)(e % l);
  Kout[(row0 + t) * ldk + col0 + i] = X[(int64_t)i * s + t];
}

// Kout ((K+s) x (K+l)) = [[diag(sig), 0], [Cp, 0]]; the augmented block is
// written afterwards.
__global__ void k_build_K_approx(int K, int64_t s, int l, const double *__restrict__ sig,
                                 const double *__restrict__ Cp, double *__restrict__ Kout,
                                 const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t N2 = K + l;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(K + s) * N2) return;
  const int64_t r = e / N2, c = e % N2;
  double v = 0.0;
  if (r < K) v = (r == c) ? sig[r] : 0.0;
  else if (c < K) v = Cp[(r - K) * K + c];
  Kout[e] = v;
}

// Cholesky with diagonal pivoting of the l x l Gram A (l <= AP_LMAX), pivots
// at or below rtol * info->scale (rel = 0) or rtol * max_i A_ii (rel = 1)
// dropped with everything after them.  Out (l x l) maps the rows of the Gram's vectors to orthonormal ones:
// row a < r of Out holds row a of L^{-1} scattered back through the pivot
// order; rows a >= r are zero.
__global__ void __launch_bounds__(256)
k_pchol_small(int l, const double *__restrict__ A, double *__restrict__ Out, double rtol,
              int rel, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double a[AP_LMAX][AP_LMAX + 1];
  __shared__ double tmp[AP_LMAX];
  __shared__ int perm[AP_LMAX];
  __shared__ int rank_s, piv_s;
  const int tid = threadIdx.x;
  for (int e = tid; e < l * l; e += blockDim.x) a[e / l][e % l] = A[e];
  for (int e = tid; e < l; e += blockDim.x) perm[e] = e;
  if (tid == 0) rank_s = l;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < l; ++i) dmax = fmax(dmax, a[i][i]);
  const double thr2 = rtol * (rel ? dmax : fmax(info->scale, 0.0));
  for (int j = 0; j < l; ++j) {
    if (tid == 0) {
      int p = j;
      for (int i = j + 1; i < l; ++i)
        if (a[i][i] > a[p][p]) p = i;
      piv_s = (a[p][p] > thr2 && a[p][p] > 0.0) ? p : -1;
      if (piv_s < 0) rank_s = j;
    }
    __syncthreads();
    const int p = piv_s;
    if (p < 0) break;
    if (p != j) {   // symmetric swap of rows / columns j and p
      for (int c = tid; c < l; c += blockDim.x) {
        const double t = a[j][c]; a[j][c] = a[p][c]; a[p][c] = t;
      }
      __syncthreads();
      for (int r = tid; r < l; r += blockDim.x) {
        const double t = a[r][j]; a[r][j] = a[r][p]; a[r][p] = t;
      }
      if (tid == 0) { const int t = perm[j]; perm[j] = perm[p]; perm[p] = t; }
      __syncthreads();
    }
    const double d = sqrt(a[j][j]);
    __syncthreads();
    for (int r = j + 1 + tid; r < l; r += blockDim.x) a[r][j] /= d;
    if (tid == 0) a[j][j] = d;
    __syncthreads();
    // the whole trailing square stays symmetric, so later symmetric swaps of
    // rows and columns see consistent values
    for (int e = tid; e < (l - j - 1) * (l - j - 1); e += blockDim.x) {
      const int r = j + 1 + e / (l - j - 1), c = j + 1 + e % (l - j - 1);
      a[r][c] -= a[r][j] * a[c][j];
    }
    __syncthreads();
  }
  __syncthreads();
  const int r = rank_s;
  // inverse of the leading r x r lower factor, in place
  tri_lower_inv_inplace(&a[0][0], AP_LMAX + 1, r, tmp);
  for (int e = tid; e < l * l; e += blockDim.x) {
    const int ra = e / l, cb = e % l;   // Out[ra][perm[cb]] = Linv[ra][cb]
    double v = 0.0;
    if (ra < r && cb < r && cb <= ra) v = a[ra][cb];
    if (cb < l) Out[ra * l + perm[cb]] = v;
  }
}

}  // namespace

namespace svl {

void sym_lower(hipStream_t st, int64_t s, double *G, int64_t ld, const SvDevInfo *info) {
  if (s <= 1) return;
  const unsigned T = (unsigned)((s + 31) / 32);
  hipLaunchKernelGGL(k_sym_lower, dim3(T, T), dim3(256), 0, st, s, G, ld, info);
}

void symv_rows(hipStream_t st, int64_t s, int nv, const double *G, int64_t ld, const double *X,
               double *Y, const int32_t *brk, const SvDevInfo *info) {
  const unsigned blocks = (unsigned)((s + 3) / 4);
  for (int j0 = 0; j0 < nv; j0 += 8) {
    const int n = nv - j0 < 8 ? nv - j0 : 8;
    const double *x = X + (int64_t)j0 * s;
    double *y = Y + (int64_t)j0 * s;
#define SV_SYMV(NN) hipLaunchKernelGGL((k_symv_multi<NN>), dim3(blocks), dim3(256), 0, st, s, G, \
                                       ld, x, y, brk, info)
    switch (n) {
      case 1: SV_SYMV(1); break;
      case 2: SV_SYMV(2); break;
      case 3: SV_SYMV(3); break;
      case 4: SV_SYMV(4); break;
      case 5: SV_SYMV(5); break;
      case 6: SV_SYMV(6); break;
      case 7: SV_SYMV(7); break;
      default: SV_SYMV(8); break;
    }
#undef SV_SYMV
  }
}

void gkl_basis(hipStream_t st, int64_t s, int l, const double *G, int64_t ld,
               const double *start, double *Pv, double *Yc, double *g, double *ab,
               int32_t *brk, double rtol, SvDevInfo *info) {
  hipLaunchKernelGGL(k_gkl_init, dim3(1), dim3(AP_NT), 0, st, s, l, start, Pv, Yc, ab, brk, info);
  for (int i = 0; i < l; ++i) {
    symv_rows(st, s, 1, G, ld, Yc + (int64_t)i * s, g, brk, info);
    hipLaunchKernelGGL(k_gkl_step, dim3(1), dim3(AP_NT), 0, st, s, i, l, Pv, Yc, g, ab, brk,
                       rtol, info);
  }
}

void gkl_pblock(hipStream_t st, int64_t s, int l, const double *Pv, const double *ab,
                double *Kout, int64_t ldk, int64_t row0, int64_t col0, const SvDevInfo *info) {
  const int64_t n = s * l;
  if (n == 0) return;
  hipLaunchKernelGGL(k_gkl_pblock, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, l,
                     Pv, ab, Kout, ldk, row0, col0, info);
}

void rows_to_block(hipStream_t st, int64_t s, int l, const double *X, double *Kout, int64_t ldk,
                   int64_t row0, int64_t col0, const SvDevInfo *info) {
  const int64_t n = s * l;
  if (n == 0) return;
  hipLaunchKernelGGL(k_rows_to_block, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, l,
                     X, Kout, ldk, row0, col0, info);
}

void build_K_approx(hipStream_t st, int K, int64_t s, int l, const double *sig, const double *Cp,
                    double *Kout, const SvDevInfo *info) {
  const int64_t n = (int64_t)(K + s) * (K + l);
  hipLaunchKernelGGL(k_build_K_approx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, s,
                     l, sig, Cp, Kout, info);
}

void pchol_small(hipStream_t st, int l, const double *A, double *Out, double rtol, int rel,
                 const SvDevInfo *info) {
  hipLaunchKernelGGL(k_pchol_small, dim3(1), dim3(256), 0, st, l, A, Out, rtol, rel, info);
}

// RPI: t rounds from P (l rows of s, overwritten).  On return Yc (l x s)
// holds the coefficient rows of Q and P the rows of Z^T Q.  X, T: l x s
// scratch; Gm2, Om: l x l scratch; ws / ws_len: split-K scratch.
void rpi_basis(hipStream_t st, int64_t s, int l, int t, const double *G, int64_t ld, double *P,
               double *Yc, double *X, double *T, double *Gm2, double *Om, double *ws,
               size_t ws_len, double rtol, const SvDevInfo *info) {
  for (int it = 0; it < t; ++it) {
    // P <- orth(P)
    gemm_f64_sk(st, false, true, l, l, s, 1.0, P, s, P, s, 0.0, Gm2, l, ws, ws_len, info);
    pchol_small(st, l, Gm2, Om, rtol, 1, info);
    gemm_f64(st, false, false, l, s, l, 1.0, Om, l, P, s, 0.0, T, s, info);
    // X = G P (rows), Gram P^T G P, its pivoted Cholesky
    symv_rows(st, s, l, G, ld, T, X, nullptr, info);
    gemm_f64_sk(st, false, true, l, l, s, 1.0, X, s, T, s, 0.0, Gm2, l, ws, ws_len, info);
    pchol_small(st, l, Gm2, Om, rtol, 0, info);
    // Yc = L^{-1} P (coefficients of Q), P = L^{-1} X (= Z^T Q)
    gemm_f64(st, false, false, l, s, l, 1.0, Om, l, T, s, 0.0, Yc, s, info);
    gemm_f64(st, false, false, l, s, l, 1.0, Om, l, X, s, 0.0, P, s, info);
  }
}

}  // namespace svl
