// The FP64 Cholesky of the residual Gram (the R of Algorithm 2, through
// Lemma 3's identity R^T R = E E^T - (E V)(E V)^T) and the triangular solve
// with its transpose (the normalisation T = R^{-1} applied to the Ritz block,
// Equation (1)), each as one cooperative launch.  Blocks exchange data through
// coherent (L2-bypassing) loads and stores and meet at flag barriers, so a
// factorisation of s = 1000 costs two launches instead of ~150.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"
#include "svlcov.h"
#include "kernels.hpp"
#include "lane.hpp"

using namespace svk;

namespace {

constexpr int NB = svl::CHOL_NB;   // 32
constexpr int CT = 256;

// Blocked right-looking Cholesky of the lower triangle of A (s x s, row
// stride ld) with pivot dropping: a pivot d_j <= tol * scale sets column j of
// L to zero.  The diagonal blocks are factored one step ahead by block 0 alone,
// which also forms their inverses (written to Linv, NB x NB per block), so the
// other blocks never wait on a factorisation.  Per block column b:
//   every block loads Linv_b; the panel rows r >= r0 are x = a Linv_b^T (a
//   product, no substitution chain): block 0 takes the NB rows of the next
//   block row, the other blocks the rest;
//   block 0 announces its panel rows, updates the next diagonal block with
//   them (A_{b+1} -= X X^T), factors it (wave 0, two lanes per row, pivots
//   by v_readlane and 1/sqrt by a Newton-refined v_rsq), inverts it (one lane
//   per column of the inverse) and stores both;
//   the other blocks wait for all panel rows and update the remaining lower
//   tiles of the trailing matrix on FP64 MFMA (16 x 16 quadrant per wave; the
//   next tile's operands are loaded while the current one is multiplied);
//   barrier.
// A dropped pivot leaves a zero column in L; its block inverse is formed with
// a unit placeholder on the diagonal and then has that row and column
// zeroed, so the solve drops the same directions.  All data exchanged between
// blocks goes through coherent loads and stores.
typedef double cv_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cv_d4 mfma64(double a, double b, cv_d4 c) {
  // A[m][k] from lane (m, k) = (l % 16, l / 16), B[k][n] from lane (k, n) =
  // (l / 16, l % 16), D[m][n] in lane (l % 16 = n, l / 16 + 4 q = m), slot q
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1 / sqrt(d) for d > 0: v_rsq_f64 refined by two Newton steps
// y <- y (3 - d y^2) / 2, each doubling the correct bits.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * (1.5 - 0.5 * d * y * y);
  y = y * (1.5 - 0.5 * d * y * y);
  return y;
}

// Arrive at / wait for a flag barrier separately (flag_barrier does both).
__device__ __forceinline__ void flag_arrive(unsigned *flags, unsigned epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&flags[blockIdx.x * FLAG_STRIDE], epoch, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

struct CholSh {
  double Li[NB][NB + 1];   // inverse of the current diagonal block
  double Xp[NB][NB + 1];   // block 0: its panel rows (the next block row)
  double Dg[NB][NB + 1];   // block 0: the next diagonal block
  double ta[NB][NB + 1];   // trailing update operands / block 0: next inverse
  double tb[NB][NB + 1];
  double row[CT / 32][NB];   // one panel row per half-wave
  double colA[NB], colB[NB];   // the two columns of a factorisation step
  double rowA[NB], rowB[NB];   // the two pivot rows of the inverse
  double piv[NB];              // the pivots d_j before the square root
  int dropped[NB];             // also set for the padding beyond nb
};

// C = D - X_a X_b^T for one NB x NB tile (X_a = ta, X_b = tb, D = dv in the
// output layout), wave w computing quadrant (w >> 1, w & 1); returns the
// lane's four results of its quadrant.
__device__ __forceinline__ cv_d4 tile_update(const double (*ta)[NB + 1],
                                             const double (*tb)[NB + 1], cv_d4 dv, int w,
                                             int lane) {
  const int li = lane & 15, lk = lane >> 4;
  const int qi = w >> 1, qj = w & 1;
  cv_d4 acc = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 4)
    acc = mfma64(ta[16 * qi + li][kk + lk], tb[16 * qj + li][kk + lk], acc);
  return dv - acc;
}

// Block 0: factor the nb x nb block in Dg in place and form the inverse of
// the factor in Ld (all NB x NB entries; zero outside the nb x nb lower part
// and on the rows and columns of dropped pivots), by wave 0 alone, two columns
// per step.  Lane (i, h) = (lane % 32, lane / 32) holds row i of the block,
// columns 16 h .. 16 h + 15, and rows 16 h .. 16 h + 15 of column i of the
// inverse, which starts as the identity and takes the same row operations as
// the block (elimination applied to [A | I] yields L^{-1}).  Per step the
// three entries of the 2 x 2 pivot block come by v_readlane and both inverse
// square roots are taken at once: with q = a11 d0 - a10^2 the second pivot
// is d1 = q / d0 and 1 / sqrt(d1) = sqrt(d0) / sqrt(q).  The two columns of
// L and the two pivot rows of the inverse then go through LDS for one rank-2
// update of both.  A dropped pivot zeroes its column of L and its row of the
// inverse.
__device__ void factor_and_invert(CholSh &sh, double (*Ld)[NB + 1], int nb, double thr,
                                  double scale, double &st_maxdrop, double &st_minkept,
                                  int &st_kept) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    const int i = lane & 31, h = lane >> 5;
    double a[16], x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      a[c] = sh.Dg[i][16 * h + c];
      x[c] = (16 * h + c == i) ? 1.0 : 0.0;
    }
    const bool scale_ok = scale > 0.0;
#pragma unroll
    for (int jp = 0; jp < NB; jp += 2) {
      if (jp < nb) {
        const int hj = jp >> 4, c0 = jp & 15, c1 = c0 + 1, lj = jp + 32 * hj;
        const bool two = jp + 1 < nb;
        const double d0 = readlane_d(a[c0], lj);
        const double a10 = readlane_d(a[c0], lj + 1);
        const double a11 = readlane_d(a[c1], lj + 1);
        const double q = a11 * d0 - a10 * a10;
        // three independent inverse square roots
        const double r0v = rsqrt_nr(fmax(d0, 1e-300));
        const double rqv = rsqrt_nr(fmax(q, 1e-300));
        const double rav = rsqrt_nr(fmax(a11, 1e-300));
        const bool drop0 = !(d0 > thr) || !scale_ok;
        const double r0 = drop0 ? 0.0 : r0v;
        const double d1 = drop0 ? a11 : q * r0 * r0;
        const bool drop1 = !(d1 > thr) || !scale_ok || !two;
        const double r1 = drop1 ? 0.0 : (drop0 ? rav : rqv * d0 * r0);
        const double l0n = a10 * r0;                 // L[jp + 1][jp]
        const double l0 = a[c0] * r0;                // L[i][jp]
        const double l1 = (a[c1] - l0 * l0n) * r1;   // L[i][jp + 1]
        if (lane == 0) {
          sh.piv[jp] = d0;
          if (two) sh.piv[jp + 1] = d1;
        }
        if (h == hj) {
          a[c0] = i > jp ? l0 : (i == jp ? d0 * r0 : 0.0);
          a[c1] = i > jp + 1 ? l1 : (i == jp + 1 ? d1 * r1 : 0.0);
          // the two columns below the pair (zero elsewhere, so finished rows
          // and columns are left unchanged by the update)
          sh.colA[i] = i > jp + 1 ? l0 : 0.0;
          sh.colB[i] = i > jp + 1 ? l1 : 0.0;
          // the pair's rows of the inverse, scaled (column i of the inverse)
          const double xa = x[c0] * r0;
          const double xb = (x[c1] - l0n * xa) * r1;
          x[c0] = xa;
          x[c1] = xb;
          sh.rowA[i] = xa;
          sh.rowB[i] = xb;
        }
        wave_sync();
        const double la = sh.colA[i], lb = sh.colB[i];
        const double xa = sh.rowA[i], xb = sh.rowB[i];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double ca = sh.colA[16 * h + c], cb = sh.colB[16 * h + c];
          a[c] -= la * ca;
          a[c] -= lb * cb;
          x[c] -= ca * xa;
          x[c] -= cb * xb;
        }
        wave_sync();
      }
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = 16 * h + c;
      sh.Dg[i][cc] = (i < nb && cc <= i) ? a[c] : 0.0;
    }
    // pivot decisions and statistics (lane j: pivot j)
    if (lane < NB) {
      const int j = lane;
      const double d = j < nb ? sh.piv[j] : 0.0;
      const bool drop = j < nb && (!(d > thr) || !scale_ok);
      sh.dropped[j] = (j >= nb || drop) ? 1 : 0;
      if (j < nb) {
        const double rel = scale_ok ? d / scale : 0.0;
        if (drop) st_maxdrop = fmax(st_maxdrop, rel);
        else { st_minkept = fmin(st_minkept, rel); ++st_kept; }
      }
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int r = 16 * h + c;   // row r, column i of the inverse
      Ld[r][i] = (r < i || sh.dropped[r] || sh.dropped[i]) ? 0.0 : x[c];
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(CT)
k_chol_coop(int64_t s, double *__restrict__ A, int64_t ld, double tol,
            SvDevInfo *__restrict__ info, int which, unsigned *__restrict__ flags,
            unsigned epoch0, double *__restrict__ Linv) {
  if (info->status) return;
  __shared__ CholSh sh;
  const int P = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double scale = which == 0 ? info->scale : info->scale2;
  const double thr = tol * scale;
  const int64_t nblk = (s + NB - 1) / NB;
  unsigned ep = epoch0;
  double st_maxdrop = -1.0, st_minkept = INFINITY;
  int st_kept = 0;
  // the blocks other than 0 share the panel rows and trailing tiles (block 0
  // joins them only when it is alone)
  const bool other = P == 1 || g >= 1;
  const int Po = P > 1 ? P - 1 : 1, go = P > 1 ? g - 1 : 0;

  // prologue: block 0 factors and inverts the first diagonal block
  if (g == 0) {
    const int nb = (int)(s < NB ? s : NB);
    for (int e = tid; e < NB * NB; e += CT) {
      const int i = e / NB, j = e % NB;
      sh.Dg[i][j] = (i < nb && j <= i) ? ld_coh(&A[i * ld + j]) : 0.0;
    }
    __syncthreads();
    factor_and_invert(sh, sh.ta, nb, thr, scale, st_maxdrop, st_minkept, st_kept);
    for (int e = tid; e < NB * NB; e += CT) {
      const int i = e / NB, j = e % NB;
      if (i < nb && j < nb) st_coh(&A[i * ld + j], sh.Dg[i][j]);
      st_coh(&Linv[e], sh.ta[i][j]);
    }
  }
  flag_barrier(flags, ++ep);

  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t b0 = b * NB;
    const int nb = (int)((s - b0) < NB ? (s - b0) : NB);
    const int64_t r0 = b0 + nb, rem = s - r0;
    const int nb1 = (int)(rem < NB ? rem : NB);   // rows of the next block row
    // block 0 fetches the next diagonal block with Linv_b
    double dgv[NB * NB / CT];
    if (g == 0) {
#pragma unroll
      for (int q = 0; q < NB * NB / CT; ++q) {
        const int e = tid + q * CT, i = e / NB, j = e % NB;
        dgv[q] = (i < nb1 && j <= i) ? ld_coh(&A[(r0 + i) * ld + r0 + j]) : 0.0;
      }
    }
    for (int e = tid; e < NB * NB; e += CT) sh.Li[e / NB][e % NB] = ld_coh(&Linv[b * NB * NB + e]);
    // panel rows: x_c = sum_{j <= c} a_j Linv[c][j] (half-wave hw, lane c)
    const int hw = tid >> 5, c = tid & 31;
    auto panel_row = [&](int64_t r, double a, bool act) -> double {
      sh.row[hw][c] = a;
      wave_sync();
      double x = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) x += sh.row[hw][j] * sh.Li[c][j];
      wave_sync();
      if (act && c < nb) st_coh(&A[r * ld + b0 + c], x);
      return x;
    };
    if (g == 0) {
      // the next block row, X = A_{b+1,b} Linv_b^T, as one MFMA tile product
      // (quadrant per wave) into tb and A
      double av[NB * NB / CT];
#pragma unroll
      for (int q = 0; q < NB * NB / CT; ++q) {
        const int e = tid + q * CT, i = e / NB, j = e % NB;
        av[q] = (i < nb1 && j < nb) ? ld_coh(&A[(r0 + i) * ld + b0 + j]) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < NB * NB / CT; ++q) {
        const int e = tid + q * CT;
        sh.Xp[e / NB][e % NB] = av[q];
      }
      __syncthreads();   // Li and the rows complete
      const int qi = w >> 1, qj = w & 1;
      const cv_d4 x = tile_update(sh.Xp, sh.Li, cv_d4{0.0, 0.0, 0.0, 0.0}, w, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * qi + lk + 4 * q, col = 16 * qj + li;
        sh.tb[row][col] = -x[q];
        if (row < nb1 && col < nb) st_coh(&A[(r0 + row) * ld + b0 + col], -x[q]);
      }
    } else {
      __syncthreads();
    }
    if (other) {
      // the remaining rows r0 + nb1 + idx, idx = 8 go + hw + 8 Po q
      for (int64_t base = (int64_t)go * (CT / 32); base < rem - nb1;
           base += (int64_t)Po * (CT / 32) * 4) {
        double av[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t idx = base + hw + (int64_t)q * Po * (CT / 32);
          av[q] = (idx < rem - nb1 && c < nb) ? ld_coh(&A[(r0 + nb1 + idx) * ld + b0 + c]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t idx = base + hw + (int64_t)q * Po * (CT / 32);
          panel_row(r0 + nb1 + idx, av[q], idx < rem - nb1);
        }
      }
    }
    if (g == 0) {
      flag_arrive(flags, ++ep);   // the next block row is stored
      if (nb1 > 0) {
        // A_{b+1} -= X X^T, factor, invert, store
#pragma unroll
        for (int q = 0; q < NB * NB / CT; ++q) {
          const int e = tid + q * CT;
          sh.Dg[e / NB][e % NB] = dgv[q];
        }
        __syncthreads();
        {
          const int qi = w >> 1, qj = w & 1;
          cv_d4 dv;
#pragma unroll
          for (int q = 0; q < 4; ++q) dv[q] = sh.Dg[16 * qi + lk + 4 * q][16 * qj + li];
          const cv_d4 r = tile_update(sh.tb, sh.tb, dv, w, lane);
          __syncthreads();
#pragma unroll
          for (int q = 0; q < 4; ++q) sh.Dg[16 * qi + lk + 4 * q][16 * qj + li] = r[q];
        }
        __syncthreads();
        factor_and_invert(sh, sh.ta, nb1, thr, scale, st_maxdrop, st_minkept, st_kept);
        for (int e = tid; e < NB * NB; e += CT) {
          const int i = e / NB, j = e % NB;
          if (i < nb1 && j < nb1) st_coh(&A[(r0 + i) * ld + r0 + j], sh.Dg[i][j]);
          st_coh(&Linv[(b + 1) * NB * NB + e], sh.ta[i][j]);
        }
      }
    } else {
      flag_barrier(flags, ++ep);   // every panel row is stored
    }
    if (other) {
      if (P == 1) flag_barrier(flags, ep);   // block 0 alone: its own stores are complete
      // trailing tiles t >= 1 of the lower triangle of rows / columns >= r0
      // (tile 0 is the next diagonal block, block 0's)
      const int64_t T = (rem + NB - 1) / NB;
      const int64_t ntiles = T * (T + 1) / 2;
      const int qi = w >> 1, qj = w & 1;
      auto coords = [&](int64_t t, int64_t &ra, int64_t &rb, bool &diag) {
        int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        const int64_t tj = t - ti * (ti + 1) / 2;
        ra = r0 + ti * NB;
        rb = r0 + tj * NB;
        diag = ti == tj;
      };
      // operands of a tile in registers: 4 entries each of X_a, X_b, D
      double pa[4], pb[4], pd[4];
      auto fetch = [&](int64_t t) {
        int64_t ra, rb;
        bool diag;
        coords(t, ra, rb, diag);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * CT, i = e / NB, p = e % NB;
          pa[q] = (ra + i < s && p < nb) ? ld_coh(&A[(ra + i) * ld + b0 + p]) : 0.0;
          pb[q] = (rb + i < s && p < nb) ? ld_coh(&A[(rb + i) * ld + b0 + p]) : 0.0;
          const int64_t oi = ra + 16 * qi + lk + 4 * q, oj = rb + 16 * qj + li;
          pd[q] = (oi < s && oj < s && (!diag || oj - rb <= oi - ra)) ? ld_coh(&A[oi * ld + oj])
                                                                    : 0.0;
        }
      };
      int64_t t = 1 + go;
      if (t < ntiles) fetch(t);
      for (; t < ntiles; t += Po) {
        int64_t ra, rb;
        bool diag;
        coords(t, ra, rb, diag);
        __syncthreads();   // the previous tile's operands are consumed
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * CT, i = e / NB, p = e % NB;
          sh.ta[i][p] = pa[q];
          sh.tb[i][p] = pb[q];
        }
        const cv_d4 dv = cv_d4{pd[0], pd[1], pd[2], pd[3]};
        __syncthreads();
        if (t + Po < ntiles) fetch(t + Po);   // in flight during the products
        if (!(diag && qi < qj)) {
          const cv_d4 r = tile_update(sh.ta, sh.tb, dv, w, lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t oi = ra + 16 * qi + lk + 4 * q, oj = rb + 16 * qj + li;
            if (oi < s && oj < s && (!diag || oj - rb <= oi - ra)) st_coh(&A[oi * ld + oj], r[q]);
          }
        }
      }
    }
    flag_barrier(flags, ++ep);
  }
  if (g == 0 && tid < 64) {
    // the pivot statistics were kept by lane 0 of block 0
    for (int o = 32; o > 0; o >>= 1) {
      st_maxdrop = fmax(st_maxdrop, __shfl_xor(st_maxdrop, o, 64));
      st_minkept = fmin(st_minkept, __shfl_xor(st_minkept, o, 64));
      st_kept += __shfl_xor(st_kept, o, 64);
    }
    if (tid == 0) {
      if (st_maxdrop > info->max_dropped) info->max_dropped = st_maxdrop;
      if (st_minkept < info->min_kept) info->min_kept = st_minkept;
      if (which == 0) info->rank += st_kept; else info->rank2 += st_kept;
    }
  }
}

// Y <- L^{-T} Y (Y is s x K row-major, K <= 128) with the factor and the
// diagonal-block inverses, by block rows from the bottom:
//   Y_b = Linv_b^T (Z_b - sum_{r > b} L_rb^T Y_r).
// Block 0 carries the sequential part one step ahead: having formed Y_b it
// applies Y_b to the next block row itself (Z_{b-1} -= L_{b,b-1}^T Y_b), forms
// Y_{b-1} and stores it, while the other blocks apply Y_b (published the step
// before) to the rows further up, one 32-row tile at a time; one grid
// barrier per block row.  Every product is on FP64 MFMA: an output tile of
// 16 x 16 per wave and step (the block row's 32 x K output is 2 K / 16 of
// them).  Dynamic LDS: Yb and Zb (32 x (K16 + 1) each, K16 = K rounded up to
// 16), the L tile and the inverse (32 x 33 each).
constexpr int TS_PAD = 1;

__device__ __forceinline__ void trsm_tile_mul(const double *__restrict__ At, int lda,
                                              const double *__restrict__ Bm, int ldb,
                                              double *__restrict__ Out, int ldo, int K16,
                                              bool subtract, int w, int lane) {
  // Out[m][n] (+)= sum_p At[p][m] * Bm[p][n], m < 32, n < K16, p < 32
  const int li = lane & 15, lk = lane >> 4;
  const int ntile = 2 * (K16 / 16);
  for (int t = w; t < ntile; t += CT / 64) {
    const int m0 = 16 * (t & 1), n0 = 16 * (t >> 1);
    cv_d4 acc = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < NB; kk += 4)
      acc = mfma64(At[(kk + lk) * lda + m0 + li], Bm[(kk + lk) * ldb + n0 + li], acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double *o = &Out[(m0 + lk + 4 * q) * ldo + n0 + li];
      *o = subtract ? *o - acc[q] : acc[q];
    }
  }
}

__global__ void __launch_bounds__(CT)
k_trsm_coop(int64_t s, int K, const double *__restrict__ L, int64_t ld,
            const double *__restrict__ Linv, double *__restrict__ Y,
            const SvDevInfo *__restrict__ info, unsigned *__restrict__ flags, unsigned epoch0) {
  if (info->status) return;
  extern __shared__ double tsm[];
  const int K16 = (K + 15) / 16 * 16, ldy = K16 + TS_PAD;
  double *Yb = tsm, *Zb = Yb + NB * ldy, *Lt = Zb + NB * ldy, *Li = Lt + NB * (NB + 1);
  const int P = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int64_t nblk = (s + NB - 1) / NB;
  unsigned ep = epoch0;
  const bool other = P == 1 || g >= 1;
  const int Po = P > 1 ? P - 1 : 1, go = P > 1 ? g - 1 : 0;
  auto rows_of = [&](int64_t blk) { return (int)((s - blk * NB) < NB ? (s - blk * NB) : NB); };
  auto load_Li = [&](int64_t blk) {
    for (int e = tid; e < NB * NB; e += CT) Li[(e / NB) * (NB + 1) + e % NB] = Linv[blk * NB * NB + e];
  };
  // Y_b = Linv_b^T Zb into Yb (Li loaded, all threads past a barrier since),
  // stored to Y (block 0)
  auto solve_block = [&](int64_t blk) {
    const int nbk = rows_of(blk);
    trsm_tile_mul(Li, NB + 1, Zb, ldy, Yb, ldy, K16, false, w, lane);
    __syncthreads();
    for (int e = tid; e < nbk * K; e += CT)
      st_coh(&Y[(blk * NB + e / K) * K + e % K], Yb[(e / K) * ldy + e % K]);
  };
  auto load_rows = [&](double *dst, int64_t blk) {
    const int nbk = rows_of(blk);
    for (int e = tid; e < NB * K16; e += CT) {
      const int i = e / K16, c = e % K16;
      dst[i * ldy + c] = (i < nbk && c < K) ? ld_coh(&Y[(blk * NB + i) * K + c]) : 0.0;
    }
  };
  // the L tile of block rows (rb) and block columns (cb): Lt[p][m] = L[rb*NB+p][cb*NB+m]
  auto load_L = [&](int64_t rb, int64_t cb) {
    const int nr = rows_of(rb), nc = rows_of(cb);
    for (int e = tid; e < NB * NB; e += CT) {
      const int p_ = e / NB, m = e % NB;
      Lt[p_ * (NB + 1) + m] = (p_ < nr && m < nc) ? L[(rb * NB + p_) * ld + cb * NB + m] : 0.0;
    }
  };

  // prologue: block 0 solves the last block row
  if (g == 0) {
    load_rows(Zb, nblk - 1);
    load_Li(nblk - 1);
    __syncthreads();
    solve_block(nblk - 1);
  }
  flag_barrier(flags, ++ep);
  for (int64_t b = nblk - 1; b >= 1; --b) {
    if (other && b >= 2) {
      // the rows of block rows 0 .. b-2 take Y_b (stored the step before;
      // block 0, alone, still holds it in Yb, so this part comes first)
      bool have = false;
      for (int64_t x = go; x <= b - 2; x += Po) {
        if (!have) {
          if (g != 0) load_rows(Yb, b);
          have = true;
        }
        load_rows(Zb, x);
        load_L(b, x);
        __syncthreads();
        trsm_tile_mul(Lt, NB + 1, Yb, ldy, Zb, ldy, K16, true, w, lane);
        __syncthreads();
        const int nx = rows_of(x);
        for (int e = tid; e < nx * K; e += CT)
          st_coh(&Y[(x * NB + e / K) * K + e % K], Zb[(e / K) * ldy + e % K]);
        __syncthreads();
      }
    }
    if (g == 0) {
      // Z_{b-1} -= L_{b,b-1}^T Y_b (Yb holds Y_b), then Y_{b-1}
      load_rows(Zb, b - 1);
      load_L(b, b - 1);
      load_Li(b - 1);
      __syncthreads();
      trsm_tile_mul(Lt, NB + 1, Yb, ldy, Zb, ldy, K16, true, w, lane);
      __syncthreads();
      solve_block(b - 1);
    }
    flag_barrier(flags, ++ep);
  }
}

// The same solve with one block per block row (up to 256 block rows) and
// point-to-point readiness flags instead of grid barriers: block x keeps its
// rows' Z_x in LDS, applies each Y_b (b > x, newest last) as soon as block b
// has flagged it (L_{b,x} is loaded ahead, Y_b by coherent loads), then forms
// Y_x = Linv_x^T Z_x, stores it and raises its own flag.  Block nblk - 1
// waits for nobody and block x only for blocks above it, so every wait ends;
// a wait that exceeds its spin limit marks the update failed and the block
// stops, and its own flag is still raised so that nothing waits for it.
__global__ void __launch_bounds__(CT)
k_trsm_p2p(int64_t s, int K, const double *__restrict__ L, int64_t ld,
           const double *__restrict__ Linv, double *__restrict__ Y, SvDevInfo *__restrict__ info,
           unsigned *__restrict__ flags, unsigned epoch) {
  if (info->status) return;
  extern __shared__ double tsm[];
  const int K16 = (K + 15) / 16 * 16, ldy = K16 + TS_PAD;
  double *Yb = tsm, *Zb = Yb + NB * ldy, *Lt = Zb + NB * ldy, *Li = Lt + NB * (NB + 1);
  __shared__ int bad;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t nblk = (s + NB - 1) / NB, x = blockIdx.x;
  auto rows_of = [&](int64_t blk) { return (int)((s - blk * NB) < NB ? (s - blk * NB) : NB); };
  const int nx = rows_of(x);
  if (tid == 0) bad = 0;
  for (int e = tid; e < NB * K16; e += CT) {
    const int i = e / K16, c = e % K16;
    Zb[i * ldy + c] = (i < nx && c < K) ? Y[(x * NB + i) * K + c] : 0.0;
  }
  for (int e = tid; e < NB * NB; e += CT) Li[(e / NB) * (NB + 1) + e % NB] = Linv[x * NB * NB + e];
  for (int64_t b = nblk - 1; b > x; --b) {
    const int nr = rows_of(b);
    __syncthreads();   // the previous product has consumed Lt and Yb
    for (int e = tid; e < NB * NB; e += CT) {
      const int p_ = e / NB, m = e % NB;
      Lt[p_ * (NB + 1) + m] = (p_ < nr && m < nx) ? L[(b * NB + p_) * ld + x * NB + m] : 0.0;
    }
    if (tid == 0) {
      unsigned spins = 0;
      while (__hip_atomic_load(&flags[b * FLAG_STRIDE], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 26)) { bad = 1; break; }
      }
    }
    __syncthreads();
    if (bad) break;
    for (int e = tid; e < NB * K16; e += CT) {
      const int i = e / K16, c = e % K16;
      Yb[i * ldy + c] = (i < nr && c < K) ? ld_coh(&Y[(b * NB + i) * K + c]) : 0.0;
    }
    __syncthreads();
    trsm_tile_mul(Lt, NB + 1, Yb, ldy, Zb, ldy, K16, true, w, lane);
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) {
      atomicCAS(&info->status, 0, (int)SVLCOV_E_DEVICE);
      __hip_atomic_store(&flags[x * FLAG_STRIDE], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  trsm_tile_mul(Li, NB + 1, Zb, ldy, Yb, ldy, K16, false, w, lane);
  __syncthreads();
  for (int e = tid; e < nx * K; e += CT)
    st_coh(&Y[(x * NB + e / K) * K + e % K], Yb[(e / K) * ldy + e % K]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0)
    __hip_atomic_store(&flags[x * FLAG_STRIDE], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_set_status(SvDevInfo *info, int code) {
  if (atomicCAS(&info->status, 0, code) == 0) info->failed_seq = -1;
}

__global__ void k_zero_flags(unsigned *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// blocks wanted for an s x s factor: one per ROWS_PER_BLOCK rows
// (SVLCOV_COOP_ROWS overrides it for tuning sweeps)
int coop_want(int64_t s) {
  int rows = 4;
  if (const char *ev = getenv("SVLCOV_COOP_ROWS")) rows = atoi(ev);
  if (rows < 1) rows = 1;
  return (int)((s + rows - 1) / rows);
}

int coop_blocks(const void *fn, int want) {
  static const int ncu = [] {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 1;
  }();
  // resident blocks per CU of each kernel, queried once (the query costs
  // host time on every update otherwise)
  static std::mutex mu;
  static std::vector<std::pair<const void *, int>> seen;
  int nb = -1;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &e : seen)
      if (e.first == fn) nb = e.second;
  }
  if (nb < 0) {
    nb = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, CT, 0);
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(mu);
    seen.emplace_back(fn, nb);
  }
  int lim = nb * ncu;
  if (lim > svl::TRI_MAX_BLOCKS) lim = svl::TRI_MAX_BLOCKS;
  if (want > lim) want = lim;
  return want < 1 ? 1 : want;
}

}  // namespace

namespace svl {

void set_status(hipStream_t st, SvDevInfo *info, int code) {
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(1), 0, st, info, code);
}

void zero_words(hipStream_t st, unsigned *p, size_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_flags, dim3(16), dim3(256), 0, st, p, n);
}

unsigned take_epochs(hipStream_t st, unsigned *flags, unsigned *epoch, unsigned count) {
  if (*epoch > 0xF0000000u - count) {   // keep epochs monotonic: restart from zero
    hipLaunchKernelGGL(k_zero_flags, dim3(16), dim3(256), 0, st, flags, TRI_FLAG_WORDS);
    *epoch = 0;
  }
  const unsigned e0 = *epoch;
  *epoch += count + 1u;
  return e0;
}

int cholesky_coop(hipStream_t st, int64_t s, double *G, int64_t ld, double *Linv, double tol,
                  SvDevInfo *info, int which, unsigned *flags, unsigned *epoch, int max_blocks) {
  if (s <= 0) return 0;
  const int64_t nblk = (s + NB - 1) / NB;
  int want = coop_want(s);
  if (max_blocks > 0 && want > max_blocks) want = max_blocks;
  const int P = coop_blocks(reinterpret_cast<const void *>(k_chol_coop), want);
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)(2 * nblk + 1));
  void *args[] = {(void *)&s, (void *)&G, (void *)&ld, (void *)&tol, (void *)&info,
                  (void *)&which, (void *)&flags, (void *)&e0, (void *)&Linv};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_chol_coop), dim3(P), dim3(CT),
                                 args, 0, st) != hipSuccess)
    return -3;
  return 0;
}

int trsm_coop(hipStream_t st, int64_t s, int K, const double *L, int64_t ld, const double *Linv,
              double *Y, const SvDevInfo *info, unsigned *flags, unsigned *epoch) {
  if (s <= 0) return 0;
  if (K <= 0 || K > 128) return -3;
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_trsm_coop),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  const int64_t nblk = (s + NB - 1) / NB;
  const int K16 = (K + 15) / 16 * 16;
  const size_t sh = (size_t)(2 * NB * (K16 + TS_PAD) + 2 * NB * (NB + 1)) * sizeof(double);
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once_p = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_trsm_p2p),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once_p;
  {
    // one block per block row, all resident at once (cooperative launch);
    // resident blocks per CU queried once per LDS size (K16 / 16 in 1..8)
    static std::atomic<int> nbp_of[9] = {};
    static const int ncu = [] {
      int dev = 0, n = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
      return n > 0 ? n : 1;
    }();
    int nbp = nbp_of[K16 / 16].load() - 1;
    if (nbp < 0) {
      nbp = 0;
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nbp, reinterpret_cast<const void *>(k_trsm_p2p), CT, sh);
      (void)hipGetLastError();
      nbp_of[K16 / 16].store(nbp + 1);
    }
    if (nblk <= svl::TRI_MAX_BLOCKS && nblk <= (int64_t)nbp * ncu) {
      unsigned e0 = take_epochs(st, flags, epoch, 1u);
      unsigned ready = e0 + 1u;
      SvDevInfo *inf = const_cast<SvDevInfo *>(info);
      void *args[] = {(void *)&s, (void *)&K, (void *)&L, (void *)&ld, (void *)&Linv,
                      (void *)&Y, (void *)&inf, (void *)&flags, (void *)&ready};
      return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_trsm_p2p),
                                        dim3((unsigned)nblk), dim3(CT), args, sh, st) == hipSuccess
                 ? 0 : -3;
    }
  }
  // block 0 and one block per remaining block row at most
  int want = (int)std::min<int64_t>(nblk, 256);
  int nb = 0, ncu = 0, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(k_trsm_coop),
                                                     CT, sh);
  (void)hipGetLastError();
  const int lim = std::max(1, std::min(nb * std::max(ncu, 1), svl::TRI_MAX_BLOCKS));
  const int P = std::max(1, std::min(want, lim));
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)nblk + 1u);
  void *args[] = {(void *)&s, (void *)&K, (void *)&L, (void *)&ld, (void *)&Linv,
                  (void *)&Y, (void *)&info, (void *)&flags, (void *)&e0};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_trsm_coop), dim3(P),
                                    dim3(CT), args, sh, st) == hipSuccess ? 0 : -3;
}

}  // namespace svl
