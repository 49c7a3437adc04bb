// Kernels of the initial truncated SVD of a sparse matrix (the randomised
// range finder with power iterations of Halko, Martinsson and Tropp, which
// the paper's introduction points to for computing the starting factors):
// the transpose of the CSR by a stable radix sort of the column ids, the
// Cholesky factor of a panel's Gram with column dropping and the inverse of
// the factor, the random completion of dropped columns and the scaling of the
// right vectors by 1 / sigma.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

// ------------------------------------------------------------- CSR transpose
// A stable LSD radix sort of the nonzeros by column id, 8 bits per pass, the
// payload being the nonzero's position in A; the CSR order of A is by row,
// so stability leaves the rows ascending within every column of the result.
constexpr int RS_NT = 256;               // threads per tile
constexpr int RS_ITEMS = 16;             // items per thread
constexpr int RS_TILE = RS_NT * RS_ITEMS;
constexpr int RS_DIG = 256;

// rid[p] = row of nonzero p (one wave per row).
__global__ void __launch_bounds__(256)
k_row_ids(int64_t rows, int64_t nnz, const int64_t *__restrict__ rp, int32_t *__restrict__ rid,
          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < rows;
       i += (int64_t)gridDim.x * 4) {
    const int64_t p0 = rp[i], p1 = rp[i + 1] < nnz ? rp[i + 1] : nnz;
    for (int64_t p = p0 + lane; p < p1; p += 64) rid[p] = (int32_t)i;
  }
}

// hist[d * tiles + t] = number of keys of tile t whose digit is d.
__global__ void __launch_bounds__(RS_NT)
k_radix_hist(int64_t nnz, const uint32_t *__restrict__ keys, int shift, int64_t tiles,
             uint32_t *__restrict__ hist, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t h[RS_DIG];
  const int tid = threadIdx.x;
  const int64_t t = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t idx = t * RS_TILE + (int64_t)r * RS_NT + tid;
    if (idx < nnz) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * tiles + t] = h[tid];
}

// Exclusive prefix sum of n counts in place, by one block of 1024 threads:
// each thread sums a contiguous chunk, the chunk sums are scanned in LDS, and
// every thread rewrites its chunk.
__global__ void __launch_bounds__(1024)
k_scan_excl(int64_t n, uint32_t *__restrict__ a, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b = (int64_t)tid * chunk, e = b + chunk < n ? b + chunk : n;
  uint32_t sum = 0;
  for (int64_t i = b; i < e; ++i) sum += a[i];
  s[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // Hillis-Steele inclusive scan
    const uint32_t v = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  uint32_t run = s[tid] - sum;
  for (int64_t i = b; i < e; ++i) {
    const uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
}

// One stable pass: every key of tile t goes to off[digit][t] plus the number
// of keys of the same digit before it in the tile.  Items are taken in rounds
// of RS_NT consecutive positions; within a round a key's rank among its wave
// comes from ballots over the digit's bits, the counts of the earlier waves
// from LDS.  Payload NULL stands for the identity (the position itself).
__global__ void __launch_bounds__(RS_NT)
k_radix_scatter(int64_t nnz, const uint32_t *__restrict__ kin, const uint32_t *__restrict__ pin,
                int shift, int64_t tiles, const uint32_t *__restrict__ off,
                uint32_t *__restrict__ kout, uint32_t *__restrict__ pout,
                const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t base[RS_DIG];
  __shared__ uint32_t cnt[2][RS_NT / 64][RS_DIG];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t t = blockIdx.x;
  base[tid] = off[(int64_t)tid * tiles + t];
  for (int q = 0; q < 2; ++q)
    for (int v = 0; v < RS_NT / 64; ++v) cnt[q][v][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int par = r & 1;
    const int64_t idx = t * RS_TILE + (int64_t)r * RS_NT + tid;
    const bool valid = idx < nnz;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t pay = valid ? (pin ? pin[idx] : (uint32_t)idx) : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    if (valid && below == 0) cnt[par][w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pre = base[d] + below;
      for (int v = 0; v < w; ++v) pre += cnt[par][v][d];
      kout[pre] = key;
      pout[pre] = pay;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int v = 0; v < RS_NT / 64; ++v) {
      tot += cnt[par][v][tid];
      cnt[par][v][tid] = 0;
    }
    base[tid] += tot;
  }
}

// rpT[j] = first position of the sorted keys whose key is >= j (j <= n).
__global__ void k_col_bounds(int64_t nnz, int64_t n, const uint32_t *__restrict__ keys,
                             int64_t *__restrict__ rpT, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = q > 0 ? (int64_t)keys[q - 1] : -1;
    int64_t cur = q < nnz ? (int64_t)keys[q] : n;
    if (cur > n) cur = n;
    for (int64_t j = prev + 1; j <= cur; ++j) rpT[j] = q;
  }
}

// Column ids and values of the transpose from the sorted payload.
__global__ void k_gather_T(int64_t nnz, const uint32_t *__restrict__ perm,
                           const int32_t *__restrict__ rid, const void *__restrict__ val,
                           int vdtype, int32_t *__restrict__ ciT, double *__restrict__ vT,
                           const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = perm[q];
    ciT[q] = rid[p];
    vT[q] = vdtype == 1 ? ((const double *)val)[p] : (double)((const float *)val)[p];
  }
}

// ------------------------------------------------- panel orthonormalisation
// Cholesky factor of the L x L Gram G (L <= 128) with column dropping, and
// Out = L^{-1} with the rows of dropped columns zero, by one block of 256
// threads.  Column j is dropped when its pivot (the squared norm of what is
// left of the panel's column j after the earlier kept columns are taken out)
// is at or below rtol times the largest diagonal entry of G; a dropped column
// leaves the trailing matrix untouched.  complete[j] = 1 marks the dropped
// columns.  Right-looking on the unscaled columns, one barrier per column;
// the inverse by forward substitution with TPC threads per column.
__global__ void __launch_bounds__(256)
k_chol_drop(int L, const double *__restrict__ G, double *__restrict__ Out,
            int32_t *__restrict__ complete, double rtol, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double Ls[];   // L x (L+1): L below the diagonal, X^T above
  const int LD = L + 1;
  double *dg = Ls + L * LD;        // L: pivots, then the diagonal of X
  int *dr = (int *)(dg + L);       // L: dropped flags
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int e = tid; e < L * L; e += 256) {
    const int i = e / L, j = e % L;
    if (j <= i) Ls[i * LD + j] = G[e];
    if (i == j) mx = fmax(mx, G[e]);
  }
  mx = block_max(mx, red);
  const double thr = rtol * mx;
  __syncthreads();
  for (int j = 0; j < L; ++j) {
    const double d = Ls[j * LD + j];
    const bool drop = !(d > thr);
    if (!drop) {
      const double invd = 1.0 / d;
      for (int i = j + 1 + (tid >> 6); i < L; i += 4) {
        const double lij = Ls[i * LD + j] * invd;
        for (int c = j + 1 + (tid & 63); c <= i; c += 64) Ls[i * LD + c] -= lij * Ls[c * LD + j];
      }
    }
    if (tid == 0) dr[j] = drop ? 1 : 0;
    __syncthreads();
  }
  for (int j = tid; j < L; j += 256) dg[j] = dr[j] ? 1.0 : sqrt(Ls[j * LD + j]);
  __syncthreads();
  for (int i = tid >> 6; i < L; i += 4)
    for (int j = tid & 63; j <= i; j += 64)
      Ls[i * LD + j] = (j < i) ? (dr[j] ? 0.0 : Ls[i * LD + j] / dg[j]) : dg[i];
  __syncthreads();
  // X = L^{-1}: column c = tid / TPC; its TPC lanes (one aligned group of a
  // wave) split the terms p of x_i = (delta_ic - sum_{c<=p<i} L[i][p] x_p) /
  // L[i][i].  X[p][c] lives at Ls[c][p] (p > c) or dg[c] (p = c).
  int TPC = 1;
  while (TPC < 64 && TPC * 2 * L <= 256) TPC *= 2;
  const int c = tid / TPC, q = tid % TPC;
  for (int i = 0; i < L; ++i) {
    double acc = 0.0;
    if (c < L && i > c)
      for (int p = c + q; p < i; p += TPC) acc += Ls[i * LD + p] * (p == c ? dg[c] : Ls[c * LD + p]);
    for (int o = 1; o < TPC; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (c < L && q == 0 && i >= c) {
      const double x = ((i == c ? 1.0 : 0.0) - acc) / Ls[i * LD + i];
      if (i == c) dg[c] = x;
      else Ls[c * LD + i] = x;
    }
    wave_sync();
  }
  __syncthreads();
  for (int e = tid; e < L * L; e += 256) {
    const int r = e / L, cc = e % L;
    double v = cc < r ? Ls[cc * LD + r] : (cc == r ? dg[r] : 0.0);
    Out[e] = dr[r] ? 0.0 : v;
  }
  for (int j = tid; j < L; j += 256) complete[j] = dr[j];
}

// Columns c of the R x L panel X with complete[c] set receive pseudo-random
// entries of variance 1 / R (uniform on [-sqrt(3/R), sqrt(3/R)]).
__global__ void k_fill_cols(int64_t R, int L, double *__restrict__ X,
                            const int32_t *__restrict__ complete, uint64_t seed,
                            const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ int32_t fl[128];
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    fl[c] = complete[c];
    if (fl[c]) any = 1;
  }
  __syncthreads();
  if (!any) return;
  const double sc = sqrt(3.0 / (double)R);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < R * L;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % L);
    if (fl[c])
      X[e] = sc * hash_unit(seed * 0x9E3779B97F4A7C15ull + (uint64_t)e * 0xD1B54A32D192ED03ull);
  }
}

// sigma_c = sqrt(max(lambda_c, 0)); column c of the R x k panel X is scaled by
// 1 / sigma_c, or zeroed when sigma_c <= tol * sigma_0 (left for completion).
__global__ void k_inv_sigma_cols(int64_t R, int k, const double *__restrict__ lam,
                                 double *__restrict__ sig, double *__restrict__ X, double tol,
                                 const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double inv[128];
  const double s0 = sqrt(fmax(lam[0], 0.0));
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    const double s = sqrt(fmax(lam[c], 0.0));
    inv[c] = (s > tol * s0 && s > 0.0) ? 1.0 / s : 0.0;
    if (blockIdx.x == 0) sig[c] = s;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < R * k;
       e += (int64_t)gridDim.x * blockDim.x)
    X[e] *= inv[e % k];
}

// status = E_NUMERIC when any of x[0..n) is not finite (grid-stride).
__global__ void k_check_finite_wide(int64_t n, const double *__restrict__ x, SvDevInfo *info) {
  if (info->status) return;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicCAS(&info->status, 0, 4);
}

template <typename F>
void allow_big_lds(F *f) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

unsigned grid_for(int64_t work, int64_t per_block, int64_t cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

namespace svl {

size_t csr_transpose_bytes(int64_t nnz, int64_t n) {
  const int64_t tiles = (nnz + RS_TILE - 1) / RS_TILE;
  return (size_t)nnz * (4 * sizeof(uint32_t) + sizeof(int32_t)) +
         (size_t)(tiles > 0 ? tiles : 1) * RS_DIG * sizeof(uint32_t) + 1024;
}

void csr_transpose(hipStream_t st, int64_t rows, int64_t cols, int64_t nnz, const int64_t *rp,
                   const int32_t *ci, const void *v, int vdt, int64_t *rpT, int32_t *ciT,
                   double *vT, void *scratch, const SvDevInfo *info) {
  const int64_t tiles = (nnz + RS_TILE - 1) / RS_TILE;
  char *p = (char *)scratch;
  uint32_t *ka = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *kb = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *pa = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *pb = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  int32_t *rid = (int32_t *)p; p += (size_t)nnz * sizeof(int32_t);
  uint32_t *hist = (uint32_t *)p;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(rows, 4, 1 << 20)), dim3(256), 0, st, rows, nnz,
                       rp, rid, info);
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < cols) ++bits;
    const int passes = (bits + 7) / 8;
    const uint32_t *kin = (const uint32_t *)ci;
    const uint32_t *pin = nullptr;
    for (int ps = 0; ps < passes; ++ps) {
      uint32_t *kout = (ps & 1) ? kb : ka;
      uint32_t *pout = (ps & 1) ? pb : pa;
      hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)tiles), dim3(RS_NT), 0, st, nnz, kin,
                         8 * ps, tiles, hist, info);
      hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, tiles * RS_DIG, hist, info);
      hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(RS_NT), 0, st, nnz, kin, pin,
                         8 * ps, tiles, hist, kout, pout, info);
      kin = kout;
      pin = pout;
    }
    hipLaunchKernelGGL(k_gather_T, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, st, nnz, pin,
                       rid, v, vdt, ciT, vT, info);
    hipLaunchKernelGGL(k_col_bounds, dim3(grid_for(nnz + 1, 256, 8192)), dim3(256), 0, st, nnz,
                       cols, kin, rpT, info);
  } else {
    hipLaunchKernelGGL(k_col_bounds, dim3(1), dim3(256), 0, st, (int64_t)0, cols,
                       (const uint32_t *)nullptr, rpT, info);
  }
}

void check_finite_wide(hipStream_t st, int64_t n, const double *x, SvDevInfo *info) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_finite_wide, dim3(grid_for(n, 256 * 8, 2048)), dim3(256), 0, st, n,
                     x, info);
}

void chol_drop(hipStream_t st, int L, const double *G, double *Out, int32_t *complete,
               double rtol, const SvDevInfo *info) {
  static bool once = false;
  if (!once) {
    allow_big_lds(k_chol_drop);
    (void)hipGetLastError();
    once = true;
  }
  const size_t sh = (size_t)L * (L + 2) * sizeof(double) + (size_t)L * sizeof(int);
  hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(256), sh, st, L, G, Out, complete, rtol, info);
}

void fill_cols(hipStream_t st, int64_t R, int L, double *X, const int32_t *complete,
               uint64_t seed, const SvDevInfo *info) {
  hipLaunchKernelGGL(k_fill_cols, dim3(grid_for(R * L, 256, 4096)), dim3(256), 0, st, R, L, X,
                     complete, seed, info);
}

void inv_sigma_cols(hipStream_t st, int64_t R, int k, const double *lam, double *sig, double *X,
                    double tol, const SvDevInfo *info) {
  hipLaunchKernelGGL(k_inv_sigma_cols, dim3(grid_for(R * k, 256, 4096)), dim3(256), 0, st, R, k,
                     lam, sig, X, tol, info);
}

// Orthonormal basis of the columns of the R x L panel X (R >= L), written to
// Y; X is overwritten.  Three passes of Cholesky QR with column dropping: the
// first keeps the columns that are independent to within rtol (squared,
// relative to the largest column) and replaces the others by random columns,
// the second restores orthogonality to rounding for kept columns of
// condition number up to ~1/sqrt(u), the third does so for the random ones.
// Without dropping the columns keep their order: column j of Y spans the
// first j + 1 columns of X.
void orth_cols(hipStream_t st, int64_t R, int L, double *X, double *Y, double *G, double *Out,
               int32_t *complete, double *ws, size_t ws_len, uint64_t seed, double rtol,
               const SvDevInfo *info) {
  for (int pass = 0; pass < 3; ++pass) {
    double *src = (pass & 1) ? Y : X;
    double *dst = (pass & 1) ? X : Y;
    gemm_f64_sk(st, true, false, L, L, R, 1.0, src, L, src, L, 0.0, G, L, ws, ws_len, info);
    chol_drop(st, L, G, Out, complete, rtol, info);
    gemm_f64(st, false, true, R, L, L, 1.0, src, L, Out, L, 0.0, dst, L, info);
    fill_cols(st, R, L, dst, complete, seed * 3 + (uint64_t)pass, info);
  }
}

}  // namespace svl
