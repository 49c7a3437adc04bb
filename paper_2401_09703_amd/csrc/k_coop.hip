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
// L to zero.  Per block column (NB = 32):
//   (1) every block loads the diagonal block and factors it (wave 0, rows
//       in registers; the other waves wait);
//   (2) the panel rows are spread over the blocks, two rows per wave: a row
//       is solved against the diagonal factor by forward substitution with
//       one lane per column;
//   barrier; block 0 stores the diagonal factor;
//   (3) the lower trailing tiles are spread over the blocks; each tile's
//       operands and destination are loaded together, then updated;
//   barrier.
// All data exchanged between blocks goes through coherent loads and stores.
// The inverses of the diagonal blocks are formed by k_chol_blkinv at the
// start of the triangular solve, off this kernel's sequential path.
__global__ void __launch_bounds__(CT)
k_chol_coop(int64_t s, double *__restrict__ A, int64_t ld, double tol,
            SvDevInfo *__restrict__ info, int which, unsigned *__restrict__ flags,
            unsigned epoch0) {
  if (info->status) return;
  __shared__ double Ld[NB][NB + 1];
  __shared__ double rinv[NB];     // 1 / L_jj, 0 for a dropped pivot
  __shared__ double colj[NB];     // scaled column of the diagonal factor
  __shared__ double ta[NB][NB + 1];
  __shared__ double tb[NB][NB + 1];
  const int P = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const double scale = which == 0 ? info->scale : info->scale2;
  const double thr = tol * scale;
  const int64_t nblk = (s + NB - 1) / NB;
  unsigned ep = epoch0;
  double st_maxdrop = -1.0, st_minkept = INFINITY;
  int st_kept = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t b0 = b * NB;
    const int nb = (int)((s - b0) < NB ? (s - b0) : NB);
    const int64_t r0 = b0 + nb;
    // (1) diagonal block
    for (int e = tid; e < NB * NB; e += CT) {
      const int i = e / NB, j = e % NB;
      Ld[i][j] = (i < nb && j <= i) ? ld_coh(&A[(b0 + i) * ld + b0 + j]) : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // wave 0 factors the block right-looking with row i in lane i's
      // registers: per column the pivot comes from lane j (v_readlane), the
      // scaled column is shared through LDS, and the trailing update is a
      // fully unrolled register loop
      const int i = lane & 31;
      double a[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) a[c] = Ld[i][c];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          const double d = readlane_d(a[j], j);
          const bool drop = !(d > thr) || !(scale > 0.0);
          const double rd = drop ? 0.0 : sqrt(d);
          const double ri = drop ? 0.0 : 1.0 / rd;
          if (lane == 0) {
            rinv[j] = ri;
            const double rel = scale > 0.0 ? d / scale : 0.0;
            if (drop) st_maxdrop = fmax(st_maxdrop, rel);
            else { st_minkept = fmin(st_minkept, rel); ++st_kept; }
          }
          const double lij = i > j ? a[j] * ri : (i == j ? rd : 0.0);
          a[j] = lij;
          if (lane < NB) colj[i] = i > j ? lij : 0.0;
          wave_sync();
#pragma unroll
          for (int c = j + 1; c < NB; ++c) a[c] -= lij * colj[c];
          wave_sync();
        }
      }
      if (lane < NB)
#pragma unroll
        for (int c = 0; c < NB; ++c) Ld[i][c] = c <= i ? a[c] : 0.0;
    }
    __syncthreads();
    // (2) panel rows r >= r0: row r = r0 + h + 8 (g + P q) for the half-wave
    // h of this block; lane c of the half-wave owns column c
    {
      const int hw = tid >> 5, c = tid & 31;   // 8 half-waves per block
      for (int64_t base = (int64_t)g * (CT / 32); base < s - r0; base += (int64_t)P * (CT / 32)) {
        const int64_t r = r0 + base + hw;
        const bool act = r < s;
        double acc = (act && c < nb) ? ld_coh(&A[r * ld + b0 + c]) : 0.0;
        double x = 0.0;
        // the pivot reciprocals and this lane's row of the factor in
        // registers, then a fully unrolled substitution
        double ri[NB], lr[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) { ri[j] = rinv[j]; lr[j] = Ld[c][j]; }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if (j < nb) {
            const double xj = __shfl(acc * ri[j], (lane & 32) + j, 64);
            if (c == j) x = xj;
            if (c > j) acc -= lr[j] * xj;
          }
        }
        if (act && c < nb) st_coh(&A[r * ld + b0 + c], x);
      }
    }
    flag_barrier(flags, ++ep);
    // every block has read the diagonal block: block 0 may now overwrite it
    // with its factor (nothing reads it again in this launch)
    if (g == 0) {
      for (int e = tid; e < nb * nb; e += CT) {
        const int i = e / nb, j = e % nb;
        st_coh(&A[(b0 + i) * ld + b0 + j], j <= i ? Ld[i][j] : 0.0);
      }
    }
    // (3) trailing update of the lower tiles of rows/columns >= r0
    const int64_t T = (s - r0 + NB - 1) / NB;
    const int64_t ntiles = T * (T + 1) / 2;
    for (int64_t t = g; t < ntiles; t += P) {
      int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      while (ti * (ti + 1) / 2 > t) --ti;
      const int64_t tj = t - ti * (ti + 1) / 2;
      const int64_t ra = r0 + ti * NB, rb = r0 + tj * NB;
      constexpr int PER = NB * NB / CT;   // destination elements per thread
      double dv[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * CT, i = e / NB, j = e % NB;
        dv[q] = (ra + i < s && rb + j < s && (ti != tj || j <= i))
                    ? ld_coh(&A[(ra + i) * ld + rb + j]) : 0.0;
      }
      for (int e = tid; e < NB * NB; e += CT) {
        const int i = e / NB, p = e % NB;
        ta[i][p] = (ra + i < s && p < nb) ? ld_coh(&A[(ra + i) * ld + b0 + p]) : 0.0;
        tb[i][p] = (rb + i < s && p < nb) ? ld_coh(&A[(rb + i) * ld + b0 + p]) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * CT, i = e / NB, j = e % NB;
        if (ra + i < s && rb + j < s && (ti != tj || j <= i)) {
          double acc = 0.0;   // entries p >= nb of ta, tb are zero
#pragma unroll
          for (int p = 0; p < NB; ++p) acc += ta[i][p] * tb[j][p];
          st_coh(&A[(ra + i) * ld + rb + j], dv[q] - acc);
        }
      }
      __syncthreads();
    }
    flag_barrier(flags, ++ep);
  }
  if (g == 0 && tid < 64) {
    // the pivot statistics were kept by the lane of each column
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

// Inverse of every NB x NB diagonal block of the factor (one wave per block):
// unit placeholders on dropped pivots (zero diagonal), then their rows and
// columns zeroed.
__global__ void __launch_bounds__(64)
k_chol_blkinv(int64_t s, const double *__restrict__ L, int64_t ld, double *__restrict__ Linv,
              const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double Li[NB][NB + 1];
  __shared__ double tmp[NB];
  __shared__ int dropped[NB];
  const int64_t b = blockIdx.x, b0 = b * NB;
  const int nb = (int)((s - b0) < NB ? (s - b0) : NB);
  const int tid = threadIdx.x;
  if (tid < NB) dropped[tid] = tid < nb ? (L[(b0 + tid) * ld + b0 + tid] == 0.0) : 1;
  wave_sync();
  for (int e = tid; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    double v = (i < nb && j <= i) ? L[(b0 + i) * ld + b0 + j] : 0.0;
    if (i == j && dropped[i]) v = 1.0;
    Li[i][j] = v;
  }
  wave_sync();
  tri_lower_inv_wave(&Li[0][0], NB + 1, NB, tmp);
  for (int e = tid; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    const bool z = j > i || dropped[i] || dropped[j];
    Linv[b * NB * NB + e] = z ? 0.0 : Li[i][j];
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

int cholesky_coop(hipStream_t st, int64_t s, double *G, int64_t ld, double tol,
                  SvDevInfo *info, int which, unsigned *flags, unsigned *epoch) {
  if (s <= 0) return 0;
  const int64_t nblk = (s + NB - 1) / NB;
  const int P = coop_blocks(reinterpret_cast<const void *>(k_chol_coop), coop_want(s));
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)(2 * nblk));
  void *args[] = {(void *)&s, (void *)&G, (void *)&ld, (void *)&tol,
                  (void *)&info, (void *)&which, (void *)&flags, (void *)&e0};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_chol_coop), dim3(P), dim3(CT),
                                 args, 0, st) != hipSuccess)
    return -3;
  return 0;
}

int trsm_coop(hipStream_t st, int64_t s, int K, const double *L, int64_t ld, double *Linv,
              double *Y, const SvDevInfo *info, unsigned *flags, unsigned *epoch) {
  if (s <= 0) return 0;
  const int64_t nblk = (s + NB - 1) / NB;
  hipLaunchKernelGGL(k_chol_blkinv, dim3((unsigned)nblk), dim3(64), 0, st, s, L, ld, Linv, info);
  const int P = coop_blocks(reinterpret_cast<const void *>(k_trsm_coop), coop_want(s));
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)nblk);
  void *args[] = {(void *)&s, (void *)&K, (void *)&L, (void *)&ld, (void *)&Linv,
                  (void *)&Y, (void *)&info, (void *)&flags, (void *)&e0};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_trsm_coop), dim3(P),
                                    dim3(CT), args, 0, st) == hipSuccess ? 0 : -3;
}

}  // namespace svl
