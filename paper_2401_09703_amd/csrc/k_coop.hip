// The FP64 Cholesky of the residual Gram (the R of Algorithm 2, through
// Lemma 3's identity R^T R = E E^T - (E V)(E V)^T) and the triangular solve
// with its transpose (the normalisation T = R^{-1} applied to the Ritz block,
// Equation (1)), each as one cooperative launch.  Blocks exchange data through
// coherent (L2-bypassing) loads and stores and meet at flag barriers, so a
// factorisation of s = 1000 costs two launches instead of ~150.
#include <cstdlib>

#include "common.hpp"
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
// diagonal-block inverses, by block rows from the bottom.  Per block row b
// every block forms Y_b = Linv_b^T Z_b redundantly; the rows above are
// updated, Z_r -= L[b rows, r]^T Y_b, spread over the blocks (their current
// values loaded before the block's barrier); one grid barrier; block 0 stores
// Y_b.
__global__ void __launch_bounds__(CT)
k_trsm_coop(int64_t s, int K, const double *__restrict__ L, int64_t ld,
            const double *__restrict__ Linv, double *__restrict__ Y,
            const SvDevInfo *__restrict__ info, unsigned *__restrict__ flags, unsigned epoch0) {
  if (info->status) return;
  __shared__ double Zb[NB][129];
  __shared__ double Yb[NB][129];
  __shared__ double Li[NB][NB + 1];
  __shared__ double lc[CT / 64][NB];
  const int P = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int64_t nblk = (s + NB - 1) / NB;
  unsigned ep = epoch0;
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t b0 = b * NB;
    const int nb = (int)((s - b0) < NB ? (s - b0) : NB);
    for (int e = tid; e < NB * NB; e += CT) Li[e / NB][e % NB] = Linv[b * NB * NB + e];
    for (int e = tid; e < NB * K; e += CT) {
      const int i = e / K, c = e % K;
      Zb[i][c] = i < nb ? ld_coh(&Y[(b0 + i) * K + c]) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < NB * K; e += CT) {
      const int i = e / K, c = e % K;
      double v = 0.0;   // rows p >= nb of Li, Zb are zero
#pragma unroll
      for (int p = 0; p < NB; ++p) v += Li[p][i] * Zb[p][c];
      Yb[i][c] = v;
    }
    // rows r < b0: 4 rows per pass (one wave each), lanes over the K columns
    for (int64_t base = (int64_t)g * (CT / 64); base < b0; base += (int64_t)P * (CT / 64)) {
      const int64_t r = base + w;
      const bool act = r < b0;
      double z0 = 0.0, z1 = 0.0;
      if (act) {
        if (lane < NB) lc[w][lane] = lane < nb ? L[(b0 + lane) * ld + r] : 0.0;
        if (lane < K) z0 = ld_coh(&Y[r * K + lane]);
        if (lane + 64 < K) z1 = ld_coh(&Y[r * K + lane + 64]);
      }
      __syncthreads();
      if (act) {
        double a0 = 0.0, a1 = 0.0;
        const int c0 = lane < K ? lane : 0, c1 = lane + 64 < K ? lane + 64 : 0;
#pragma unroll
        for (int p = 0; p < NB; ++p) {   // lc[w][p] = 0 for p >= nb
          const double l = lc[w][p];
          a0 += l * Yb[p][c0];
          a1 += l * Yb[p][c1];
        }
        if (lane < K) st_coh(&Y[r * K + lane], z0 - a0);
        if (lane + 64 < K) st_coh(&Y[r * K + lane + 64], z1 - a1);
      }
      __syncthreads();
    }
    __syncthreads();
    flag_barrier(flags, ++ep);
    // every block has read Z_b: block 0 may now store Y_b over it
    if (g == 0)
      for (int e = tid; e < nb * K; e += CT) st_coh(&Y[(b0 + e / K) * K + e % K], Yb[e / K][e % K]);
    __syncthreads();
  }
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
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 1;
  }
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, CT, 0);
  (void)hipGetLastError();
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
                  SvDevInfo *info, int which, unsigned *flags, unsigned *epoch) {
  if (s <= 0) return 0;
  const int64_t nblk = (s + NB - 1) / NB;
  const int P = coop_blocks(reinterpret_cast<const void *>(k_chol_coop), coop_want(s));
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
  const int64_t nblk = (s + NB - 1) / NB;
  const int P = coop_blocks(reinterpret_cast<const void *>(k_trsm_coop), coop_want(s));
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)nblk);
  void *args[] = {(void *)&s, (void *)&K, (void *)&L, (void *)&ld, (void *)&Linv,
                  (void *)&Y, (void *)&info, (void *)&flags, (void *)&e0};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_trsm_coop), dim3(P),
                                    dim3(CT), args, 0, st) == hipSuccess ? 0 : -3;
}

}  // namespace svl
