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
#include "k_rsvd.hpp"

using namespace svk;

namespace {

// A gated pass does nothing unless the flag *need (written by k_orth_gate
// before it) is set; need == NULL runs it always.  Every thread reads the same
// word, so the decision is uniform across the block.
__device__ __forceinline__ bool skip_pass(const int32_t *__restrict__ need) {
  return need && *need == 0;
}

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

// Exclusive prefix sum of n counts in place, in three launches: the sums of
// tiles of SC_TILE counts, the scan of those sums (one block), and the scan
// of every tile in LDS plus its offset.  All loads and stores are coalesced.
constexpr int SC_NT = 256, SC_PER = 8, SC_TILE = SC_NT * SC_PER;

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *sh, uint32_t *total) {
  // Hillis-Steele over the block's SC_NT values; sh holds SC_NT entries
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < SC_NT; o <<= 1) {
    const uint32_t x = tid >= o ? sh[tid - o] : 0u;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  const uint32_t incl = sh[tid];
  *total = sh[SC_NT - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(SC_NT)
k_scan_sums(int64_t n, const uint32_t *__restrict__ a, uint32_t *__restrict__ bsum,
            const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t sh[SC_NT];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  uint32_t s = 0;
  for (int u = 0; u < SC_PER; ++u) {
    const int64_t i = base + (int64_t)u * SC_NT + threadIdx.x;
    if (i < n) s += a[i];
  }
  uint32_t tot;
  (void)block_excl_scan_u32(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SC_NT)
k_scan_bsum(int64_t nb, uint32_t *__restrict__ bsum, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t sh[SC_NT];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SC_NT) {
    const int64_t i = b0 + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan_u32(v, sh, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(SC_NT)
k_scan_apply(int64_t n, uint32_t *__restrict__ a, const uint32_t *__restrict__ bsum,
             const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ uint32_t tile[SC_TILE];
  __shared__ uint32_t sh[SC_NT];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  for (int u = 0; u < SC_PER; ++u) {
    const int64_t i = base + (int64_t)u * SC_NT + tid;
    tile[u * SC_NT + tid] = i < n ? a[i] : 0u;
  }
  __syncthreads();
  uint32_t loc[SC_PER], s = 0;
  for (int u = 0; u < SC_PER; ++u) {   // thread tid owns counts [tid SC_PER, (tid+1) SC_PER)
    loc[u] = s;
    s += tile[tid * SC_PER + u];
  }
  uint32_t tot;
  const uint32_t off = block_excl_scan_u32(s, sh, &tot) + bsum[blockIdx.x];
  for (int u = 0; u < SC_PER; ++u) tile[tid * SC_PER + u] = off + loc[u];
  __syncthreads();
  for (int u = 0; u < SC_PER; ++u) {
    const int64_t i = base + (int64_t)u * SC_NT + tid;
    if (i < n) a[i] = tile[u * SC_NT + tid];
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
// Out = L^{-1} for the Cholesky factor L of the L x L Gram G (L <= 128), with
// column dropping, by one block of CD_NT threads.  Symmetric elimination of G
// applied to the identity beside it: after column j is eliminated, row i > j
// of the augmented part holds row i of (unit lower L)^{-1} as far as it is
// known, so at the end Out[i] = Aug[i] / sqrt(d_i) with d_i the pivots.
// Column j is dropped when its pivot (the squared norm of what is left of the
// panel's column j after the earlier kept columns are taken out) is at or
// below rtol times the largest diagonal entry of G: it eliminates nothing,
// and its row of Out is zero (complete[j] = 1).  One array of L x (L+1): the
// trailing part of G in the lower triangle with the diagonal, the strict lower
// part of Aug transposed into the strict upper triangle (Aug[i][c] at
// S[c][i], the unit diagonal implicit).  Per column the update of the
// trailing lower triangle (c > j) and of the augmented rows (c <= j) read
// only column j of G and row j of Aug, which no thread writes in that step,
// so one barrier per column suffices.
constexpr int CD_NT = 1024;
constexpr int CD_RW = (128 + CD_NT / 64 - 1) / (CD_NT / 64);   // rows per wave and column

__global__ void __launch_bounds__(CD_NT)
k_chol_drop(int L, const double *__restrict__ G, double *__restrict__ Out,
            int32_t *__restrict__ complete, double rtol, const SvDevInfo *__restrict__ info,
            const int32_t *__restrict__ need) {
  if (info->status) return;
  if (skip_pass(need)) {   // Out = I and nothing to complete: the product copies the panel
    for (int e = threadIdx.x; e < L * L; e += blockDim.x) Out[e] = (e / L == e % L) ? 1.0 : 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) complete[j] = 0;
    return;
  }
  extern __shared__ double S[];
  const int LD = L + 1;
  double *dg = S + L * LD;         // pivots
  int *dr = (int *)(dg + L);       // dropped flags
  __shared__ double red[CD_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NW = CD_NT / 64;
  double mx = 0.0;
  for (int e = tid; e < L * L; e += CD_NT) {
    const int i = e / L, c = e % L;
    S[i * LD + c] = (c <= i) ? G[e] : 0.0;   // Aug starts as the identity
    if (i == c) mx = fmax(mx, G[e]);
  }
  mx = block_max(mx, red);
  const double thr = rtol * mx;
  __syncthreads();
  for (int j = 0; j < L; ++j) {
    const double d = S[j * LD + j];
    const bool drop = !(d > thr);
    if (!drop) {
      // column j of G below the diagonal and row j of Aug (c < j): the two
      // entries this lane needs, then the wave's row multipliers, all loaded
      // before the first update
      const double invd = 1.0 / d;
      const int c0 = lane, c1 = lane + 64;
      const double a0 = c0 < L ? S[c0 * LD + j] : 0.0;
      const double a1 = c1 < L ? S[c1 * LD + j] : 0.0;
      double li[CD_RW];
#pragma unroll
      for (int t = 0; t < CD_RW; ++t) {
        const int i = j + 1 + w + NW * t;
        li[t] = i < L ? S[i * LD + j] * invd : 0.0;
      }
      // the targets of this lane: (row i_t, column c0 / c1) in the trailing
      // lower triangle (c > j), Aug[i_t][c] at S[c][i_t] (c < j), or
      // Aug[i_t][j] (c = j, overwritten); all loaded before any store
      int o0[CD_RW], o1[CD_RW];
      double v0[CD_RW], v1[CD_RW];
#pragma unroll
      for (int t = 0; t < CD_RW; ++t) {
        const int i = j + 1 + w + NW * t;
        o0[t] = -1;
        o1[t] = -1;
        if (i < L && c0 <= i) o0[t] = c0 > j ? i * LD + c0 : (c0 < j ? c0 * LD + i : j * LD + i);
        if (i < L && c1 <= i) o1[t] = c1 > j ? i * LD + c1 : (c1 < j ? c1 * LD + i : j * LD + i);
        v0[t] = (o0[t] >= 0 && c0 != j) ? S[o0[t]] : 0.0;
        v1[t] = (o1[t] >= 0 && c1 != j) ? S[o1[t]] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < CD_RW; ++t) {
        if (o0[t] >= 0) S[o0[t]] = c0 == j ? -li[t] : v0[t] - li[t] * a0;
        if (o1[t] >= 0) S[o1[t]] = c1 == j ? -li[t] : v1[t] - li[t] * a1;
      }
    }
    if (tid == 0) {
      dg[j] = d;
      dr[j] = drop ? 1 : 0;
    }
    __syncthreads();
  }
  for (int e = tid; e < L * L; e += CD_NT) {
    const int i = e / L, c = e % L;
    double v = 0.0;
    if (!dr[i] && c <= i) v = (c == i ? 1.0 : S[c * LD + i]) / sqrt(dg[i]);
    Out[e] = v;
  }
  for (int j = tid; j < L; j += CD_NT) complete[j] = dr[j];
}

// -------------------------------------------- tall-skinny FP64 MFMA products
// v_mfma_f64_16x16x4: A 16 x 4 with lane l holding A[l % 16][l / 16], B 4 x 16
// with lane l holding B[l / 16][l % 16], D 16 x 16 with lane l holding
// D[l / 16 + 4 q][l % 16] in element q (rows interleaved, unlike the FP32
// 16 x 16 x 4 form).
typedef double rv_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rv_d4 mfma_f64(double a, double b, rv_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial Grams of an R x L panel Y (L = 16 LT): block z sums Y_r^T Y_r over
// its rows r in [z rpb, (z+1) rpb), for the NT = LT (LT+1)/2 lower 16 x 16
// tiles only (tile t = ti (ti+1)/2 + tj, ti >= tj), into part[z][t][16][16].
// Rows are staged TG_KC at a time in LDS (the next chunk is loaded into
// registers while the current one is multiplied); wave w owns the tiles t
// with t mod 4 = w, and every lane's operands for all tiles of a step of four
// rows are the LT values Y[r][16 t + l % 16], r = step + l / 16.
constexpr int TG_KC = 32;

template <int L>
__global__ void __launch_bounds__(256)
k_ts_gram(int64_t R, int64_t rpb, const double *__restrict__ Y, double *__restrict__ part,
          const SvDevInfo *__restrict__ info, const int32_t *__restrict__ need) {
  if (info->status || skip_pass(need)) return;
  constexpr int LT = L / 16;
  constexpr int NT = LT * (LT + 1) / 2;
  constexpr int TW = (NT + 3) / 4;
  constexpr int LDY = L + 8;
  constexpr int PER = TG_KC * L / 2 / 256;   // 16-byte loads per thread and chunk
  __shared__ double Ys[TG_KC * LDY];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  rv_d4 acc[TW];
#pragma unroll
  for (int u = 0; u < TW; ++u) acc[u] = rv_d4{0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = r0 + rpb < R ? r0 + rpb : R;
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 nx[PER > 0 ? PER : 1];
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int h = 0; h < PER; ++h) {
      const int e = (h * 256 + tid) * 2;
      const int rr = e / L, cc = e % L;
      const int64_t r = c0 + rr;
      nx[h] = r < r1 ? *(const d2 *)(Y + r * L + cc) : d2{0.0, 0.0};
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += TG_KC) {
#pragma unroll
    for (int h = 0; h < PER; ++h) {
      const int e = (h * 256 + tid) * 2;
      *(d2 *)(Ys + (e / L) * LDY + e % L) = nx[h];
    }
    __syncthreads();
    if (c0 + TG_KC < r1) fetch(c0 + TG_KC);
#pragma unroll
    for (int kk = 0; kk < TG_KC; kk += 4) {
      double a[LT];
#pragma unroll
      for (int t = 0; t < LT; ++t) a[t] = Ys[(kk + lk) * LDY + t * 16 + li];
#pragma unroll
      for (int ti = 0; ti < LT; ++ti)
#pragma unroll
        for (int tj = 0; tj <= ti; ++tj) {
          const int t = ti * (ti + 1) / 2 + tj;
          if ((t & 3) == w) acc[t >> 2] = mfma_f64(a[ti], a[tj], acc[t >> 2]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < TW; ++u) {
    const int t = 4 * u + w;
    if (t < NT)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        part[((int64_t)blockIdx.x * NT + t) * 256 + (lk + 4 * q) * 16 + li] = acc[u][q];
  }
}

// part2[s][e] = sum over z = s, s + S, s + 2S, ... < Z of part[z][e]
// (e < NE); then G from the S slabs, both triangles (fixed order: identical
// inputs give identical bits).
__global__ void k_gram_reduce1(int Z, int S, int64_t NE, const double *__restrict__ part,
                               double *__restrict__ part2, const SvDevInfo *__restrict__ info,
                               const int32_t *__restrict__ need) {
  if (info->status || skip_pass(need)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= NE) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int u = 0;
  for (int z = s; z < Z; z += S, ++u) acc[u & 3] += part[(int64_t)z * NE + e];
  part2[(int64_t)s * NE + e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__global__ void k_gram_reduce2(int L, int S, const double *__restrict__ part2,
                               double *__restrict__ G, const SvDevInfo *__restrict__ info,
                               const int32_t *__restrict__ need) {
  if (info->status || skip_pass(need)) return;
  const int LT = L / 16, NT = LT * (LT + 1) / 2;
  const int64_t NE = (int64_t)NT * 256;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NE) return;
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += part2[(int64_t)s * NE + e];
  const int t = (int)(e >> 8), x = (int)(e & 255);
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int i = ti * 16 + (x >> 4), j = tj * 16 + (x & 15);
  G[i * L + j] = v;
  G[j * L + i] = v;
}

// Y = X Out^T for the R x L panel X and the lower-triangular L x L Out
// (L = 16 LT): block = 64 rows, wave w its rows 16 w .. 16 w + 15 for all LT
// column tiles.  The inner index runs in chunks of 16 staged in LDS (the
// chunk of X and of Out); chunk c meets only column tiles tj >= c, since
// Out[j][k] = 0 for k > j.
template <int L>
__global__ void __launch_bounds__(256)
k_ts_mul_lt(int64_t R, const double *__restrict__ X, const double *__restrict__ Out,
            double *__restrict__ Y, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int LT = L / 16;
  constexpr int LD = 16 + 1;
  __shared__ double Xs[64 * LD];
  __shared__ double Os[L * LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  rv_d4 acc[LT];
#pragma unroll
  for (int t = 0; t < LT; ++t) acc[t] = rv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < LT; ++c) {
    const int kc = 16 * c;
    for (int e = tid; e < 64 * 16; e += 256) {
      const int rr = e >> 4, cc = e & 15;
      const int64_t r = r0 + rr;
      Xs[rr * LD + cc] = r < R ? X[r * L + kc + cc] : 0.0;
    }
    for (int e = tid; e < L * 16; e += 256) {
      const int j = e >> 4, cc = e & 15;
      Os[j * LD + cc] = Out[j * L + kc + cc];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const double a = Xs[(w * 16 + li) * LD + kk + lk];
#pragma unroll
      for (int tj = c; tj < LT; ++tj) acc[tj] = mfma_f64(a, Os[(tj * 16 + li) * LD + kk + lk], acc[tj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int tj = 0; tj < LT; ++tj)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + w * 16 + lk + 4 * q;
      if (r < R) Y[r * L + tj * 16 + li] = acc[tj][q];
    }
}

// The same factor and inverse for L = 16 NB (L <= 128) in 16 x 16 blocks,
// by one block of CB_NT threads, the block updates on FP64 MFMA.  Per block
// column b: wave 0 factors the diagonal block (right-looking, with the same
// dropping rule) and inverts it into X'_bb (the rows of dropped columns zero);
// the panel below becomes L_rb = A_rb X'_bb^T (which leaves the columns of
// dropped pivots zero); the trailing lower tiles take A_rc -= L_rb L_cb^T.
// Then block rows of X' = L^{-1} (dropped rows zero) follow from
// X'_ij = -X'_ii sum_{k=j}^{i-1} L_ik X'_kj.  S holds L in its lower triangle
// and X'^T strictly above the diagonal; dg the diagonal of X'.
// Lane J of each row of 16 lanes, to every lane of that row (DPP
// row_newbcast; J a constant).
template <int J>
__device__ __forceinline__ double row_bcast16(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + J, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Steps J .. 15 of the right-looking Cholesky of a 16 x 16 block held one row
// per lane in each row of 16 lanes (lane 16 g + i: row i of the reduced
// block, both triangles, in a; the same in all four rows), with the inverse
// of the factor spread over the four rows (lane 16 g + i: entries
// 4 g .. 4 g + 3 of row i in z) and the factor's columns below the diagonal
// (lr).  Column J's pivot d is dropped unless d > thr, which leaves a zero
// column of multipliers (no update), a unit diagonal and a row of the inverse
// that the caller zeroes.  Row J of the inverse is zero beyond column J, so
// the update z_ic -= l_iJ z_Jc / sqrt(d) runs over all four entries; lane J
// scales its row instead (l_JJ is 0 there).  Lane 0 records the pivot and the
// drop flag.
template <int J>
__device__ __forceinline__ void diag16_steps(double (&a)[16], double (&z)[4], double (&lr)[16],
                                             int i, double thr, double &ldiag, bool &mydrop,
                                             double *piv, int *dr, bool rec) {
  if constexpr (J < 16) {
    const double d = row_bcast16<J>(a[J]);
    const bool drop = !(d > thr);
    const double sd = drop ? 1.0 : sqrt(d);
    const double r = 1.0 / sd;
    const double li = (i > J && !drop) ? a[J] * r : 0.0;
    const double sc = i == J ? r : 1.0;
    lr[J] = li;
    if (i == J) {
      ldiag = sd;
      mydrop = drop;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) z[q] = fma(-li, row_bcast16<J>(z[q]) * r, z[q] * sc);
#pragma unroll
    for (int c = J + 1; c < 16; ++c) a[c] -= li * (row_bcast16<J>(a[c]) * r);
    if (rec) {
      dr[J] = drop ? 1 : 0;
      piv[J] = d;
    }
    diag16_steps<J + 1>(a, z, lr, i, thr, ldiag, mydrop, piv, dr, rec);
  }
}

constexpr int CB_NT = 512;
constexpr int CB_NW = CB_NT / 64;

__global__ void __launch_bounds__(CB_NT)
k_chol_drop_blk(int L, const double *__restrict__ G, double *__restrict__ Out,
                int32_t *__restrict__ complete, double rtol, const SvDevInfo *__restrict__ info,
                const int32_t *__restrict__ need) {
  if (info->status) return;
  if (skip_pass(need)) {   // Out = I and nothing to complete: the product copies the panel
    for (int e = threadIdx.x; e < L * L; e += blockDim.x) Out[e] = (e / L == e % L) ? 1.0 : 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) complete[j] = 0;
    return;
  }
  extern __shared__ double S[];
  const int LD = L + 1, NB = L / 16;
  double *dg = S + L * LD;              // diagonal of X'
  double *piv = dg + L;                 // pivots
  double *wsc = piv + L;                // CB_NW scratch tiles of 16 x 17
  int *dr = (int *)(wsc + CB_NW * 16 * 17);
  __shared__ double red[CB_NW];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double mx = 0.0;
  for (int e0 = 0; e0 < L * L; e0 += 4 * CB_NT) {   // four loads in flight per thread
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * CB_NT + tid;
      v[u] = e < L * L ? G[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * CB_NT + tid;
      if (e < L * L) {
        const int i = e / L, c = e % L;
        S[i * LD + c] = (c <= i) ? v[u] : 0.0;
        if (i == c) mx = fmax(mx, v[u]);
      }
    }
  }
  mx = block_max(mx, red);
  const double thr = rtol * mx;
  __syncthreads();
  for (int b = 0; b < NB; ++b) {
    const int o = 16 * b;
    if (w == 0) {
      // the diagonal block by wave 0: lane 16 g + i holds row i of the
      // reduced block (both triangles, so that l_cj = A[j][c] / sqrt(A[j][j])
      // is lane j's own entry c) and entries 4 g .. 4 g + 3 of row i of its
      // inverse in registers; per column j lane j's entries reach the other
      // lanes of its row of 16 by a row broadcast (no LDS round trip, no wave
      // barrier).
      const int i = lane & 15, g = lane >> 4;
      double a[16], z[4], lr[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        a[c] = c <= i ? S[(o + i) * LD + o + c] : S[(o + c) * LD + o + i];
        lr[c] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) z[q] = 4 * g + q == i ? 1.0 : 0.0;
      double ldiag = 1.0;
      bool mydrop = false;
      diag16_steps<0>(a, z, lr, i, thr, ldiag, mydrop, piv + o, dr + o, lane == 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {   // X'^T above the diagonal, the diagonal of X'
        const int c = 4 * g + q;
        if (c < i) S[(o + c) * LD + o + i] = mydrop ? 0.0 : z[q];
        else if (c == i) dg[o + i] = mydrop ? 0.0 : z[q];
      }
      if (g == 0) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < i) S[(o + i) * LD + o + c] = lr[c];   // L below the diagonal
          else if (c == i) S[(o + i) * LD + o + i] = ldiag;
        }
      }
    }
    __syncthreads();
    // L_rb = A_rb X'_bb^T: B[k][n] = X'_bb[n][k]
    for (int rb = b + 1 + w; rb < NB; rb += CB_NW) {
      double av[4], bv[4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + lk, n = li;
        av[s4] = S[(16 * rb + li) * LD + o + k];
        bv[s4] = (k == n) ? dg[o + n] : (k < n ? S[(o + k) * LD + o + n] : 0.0);
      }
      rv_d4 acc = rv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) acc = mfma_f64(av[s4], bv[s4], acc);
      wave_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) S[(16 * rb + lk + 4 * q) * LD + o + li] = acc[q];
    }
    __syncthreads();
    // A_rc -= L_rb L_cb^T for b < c <= r
    {
      int t = 0;
      for (int r = b + 1; r < NB; ++r)
        for (int c = b + 1; c <= r; ++c, ++t) {
          if (t % CB_NW != w) continue;
          rv_d4 acc;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = S[(16 * r + lk + 4 * q) * LD + 16 * c + li];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int k = 4 * s4 + lk;
            acc = mfma_f64(-S[(16 * r + li) * LD + o + k], S[(16 * c + li) * LD + o + k], acc);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) S[(16 * r + lk + 4 * q) * LD + 16 * c + li] = acc[q];
        }
    }
    __syncthreads();
  }
  // block rows of X' below the diagonal
  double *wt = wsc + w * 16 * 17;
  for (int i = 1; i < NB; ++i) {
    for (int j = w; j < i; j += CB_NW) {
      rv_d4 T = rv_d4{0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; ++k) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int q = 4 * s4 + lk, n = li;
          const double a = S[(16 * i + li) * LD + 16 * k + q];
          double bq;
          if (k == j) bq = q == n ? dg[16 * j + q] : (q > n ? S[(16 * j + n) * LD + 16 * j + q] : 0.0);
          else bq = S[(16 * j + n) * LD + 16 * k + q];
          T = mfma_f64(a, bq, T);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) wt[(lk + 4 * q) * 17 + li] = T[q];
      wave_sync();
      rv_d4 X = rv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kq = 4 * s4 + lk;
        const double xi = li == kq ? dg[16 * i + li]
                                   : (li > kq ? S[(16 * i + kq) * LD + 16 * i + li] : 0.0);
        X = mfma_f64(-xi, wt[kq * 17 + li], X);
      }
      wave_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) S[(16 * j + li) * LD + 16 * i + lk + 4 * q] = X[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < L * L; e += CB_NT) {
    const int i = e / L, c = e % L;
    Out[e] = c > i ? 0.0 : (c == i ? dg[i] : S[c * LD + i]);
  }
  for (int j = tid; j < L; j += CB_NT) complete[j] = dr[j];
}

// Columns c of the R x L panel X with complete[c] set receive pseudo-random
// entries of variance 1 / R (uniform on [-sqrt(3/R), sqrt(3/R)]).
__global__ void k_fill_cols(int64_t R, int L, double *__restrict__ X,
                            const int32_t *__restrict__ complete, uint64_t seed,
                            const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ int32_t fl[128];
  bool mine = false;
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    fl[c] = complete[c];
    mine |= fl[c] != 0;
  }
  if (!__syncthreads_or(mine)) return;
  const double sc = sqrt(3.0 / (double)R);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < R * L;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % L);
    if (fl[c])
      X[e] = sc * hash_unit(seed * 0x9E3779B97F4A7C15ull + (uint64_t)e * 0xD1B54A32D192ED03ull);
  }
}

// *need = 1 unless the Gram G of the panel that a Cholesky QR pass has just
// orthonormalised was within tau of the identity after column scaling
// (|G_ic| <= tau sqrt(G_ii G_cc) for every i != c) and that pass completed
// no column.  Then the panel's condition number was at most
// sqrt((1 + (L-1) tau) / (1 - (L-1) tau)), and one pass already left it
// orthonormal to a small multiple of the unit roundoff: a second pass would
// change nothing but rounding.
__global__ void __launch_bounds__(1024)
k_orth_gate(int L, const double *__restrict__ G, const int32_t *__restrict__ complete,
            double tau, int32_t *__restrict__ need, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double dg[];   // sqrt(G_ii), L entries
  bool more = false;
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    dg[j] = sqrt(G[j * L + j]);
    more |= complete[j] != 0;
  }
  __syncthreads();
  // eight independent entries in flight per thread
  const int n = L * L;
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * (int)blockDim.x) {
    double g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      g[u] = e < n ? G[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      const int i = e / L, c = e - (e / L) * L;
      if (e < n && c < i) more |= !(fabs(g[u]) <= tau * (dg[i] * dg[c]));
    }
  }
  more = __syncthreads_or(more);
  if (threadIdx.x == 0) *need = more ? 1 : 0;
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

// ------------------------------------------ deterministic sparse row update
// base[c, :] += sum_i E[i, c] M[i, :] without floating-point atomics: the
// nonzeros are sorted by column (the stable radix sort above, so rows stay
// ascending within a column), every distinct column gets one wave, and the
// wave sums its rows in that order, so the result does not depend on
// scheduling.

__global__ void k_zero_count(uint32_t *__restrict__ count, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  *count = 0u;
}

// heads[count++] = q for every q that starts a run of equal keys (the order
// of the list is free: each run is summed by its own wave).
__global__ void k_seg_heads(int64_t nnz, const uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ heads, uint32_t *__restrict__ count,
                            const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * blockDim.x)
    if (q == 0 || keys[q] != keys[q - 1]) heads[atomicAdd(count, 1u)] = (uint32_t)q;
}

// Runs longer than SEG_LONG nonzeros (the hot columns of a power-law
// update: thousands of rows in one column) go to k_scatter_long.
constexpr int64_t SEG_LONG = 256;

template <typename T, int K>
__global__ void __launch_bounds__(256)
k_scatter_seg(int64_t nnz, const uint32_t *__restrict__ keys, const uint32_t *__restrict__ perm,
              const uint32_t *__restrict__ heads, const uint32_t *__restrict__ count,
              const int32_t *__restrict__ rid, const void *__restrict__ val, int vdtype,
              const double *__restrict__ M, T *__restrict__ base,
              const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  const int lane = threadIdx.x & 63;
  const uint32_t nseg = *count;
  for (int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); sg < (int64_t)nseg;
       sg += (int64_t)gridDim.x * 4) {
    const uint32_t q0 = heads[sg], key = keys[q0];
    if ((int64_t)q0 + SEG_LONG < nnz && keys[q0 + SEG_LONG] == key) continue;   // k_scatter_long's
    double acc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) acc[u] = 0.0;
    // SU nonzeros of the segment at a time: their indices, values and rows
    // of M are loaded together (a hot column's segment is thousands long,
    // and one load chain per nonzero made it the kernel's whole time), then
    // added in segment order as before
    constexpr int SU = 32;
    for (uint32_t q = q0;; q += SU) {
      bool in[SU];
      uint32_t pp[SU];
#pragma unroll
      for (int b = 0; b < SU; ++b) {
        const uint32_t qq = q + b;
        in[b] = qq < (uint32_t)nnz && keys[qq] == key;
        pp[b] = in[b] ? perm[qq] : 0u;
      }
      double vb[SU], mb[SU][CPL];
#pragma unroll
      for (int b = 0; b < SU; ++b) {
        vb[b] = !in[b] ? 0.0
                       : vdtype == 1 ? ((const double *)val)[pp[b]]
                                     : (double)((const float *)val)[pp[b]];
        const int64_t i = in[b] ? rid[pp[b]] : 0;
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          mb[b][u] = in[b] && lane + 64 * u < K ? M[i * K + lane + 64 * u] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < SU; ++b)
        if (in[b])
#pragma unroll
          for (int u = 0; u < CPL; ++u)
            if (lane + 64 * u < K) acc[u] += vb[b] * mb[b][u];
      if (!in[SU - 1]) break;
    }
    T *dst = base + (int64_t)key * K;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (lane + 64 * u < K) dst[lane + 64 * u] = (T)((double)dst[lane + 64 * u] + acc[u]);
  }
}

// The runs longer than SEG_LONG, one block of LW waves each: the run's end by
// binary search over the sorted keys, wave w sums the w-th of LW contiguous
// pieces in row order (SU nonzeros' loads at a time, as k_scatter_seg), and
// the LW partial sums are added in wave order, so the result is again fixed
// by the input alone.  Blocks stride over the list of runs LW at a time, each
// wave testing one run (three dependent loads) and listing the long ones in
// LDS; the block then takes the listed runs one after another (their order
// does not matter: every run writes its own base row).
constexpr int LW = 8;   // two waves per SIMD: 256 registers a lane for the batch of loads

template <typename T, int K>
__global__ void __launch_bounds__(LW * 64)
k_scatter_long(int64_t nnz, const uint32_t *__restrict__ keys, const uint32_t *__restrict__ perm,
               const uint32_t *__restrict__ heads, const uint32_t *__restrict__ count,
               const int32_t *__restrict__ rid, const void *__restrict__ val, int vdtype,
               const double *__restrict__ M, T *__restrict__ base,
               const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  __shared__ double part[LW][K];
  __shared__ uint32_t lq[LW];
  __shared__ int nl;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t nseg = *count;
  for (int64_t sg0 = (int64_t)blockIdx.x * LW; sg0 < (int64_t)nseg;
       sg0 += (int64_t)gridDim.x * LW) {
    if (threadIdx.x == 0) nl = 0;
    __syncthreads();
    if (lane == 0 && sg0 + w < (int64_t)nseg) {
      const uint32_t q = heads[sg0 + w];
      if ((int64_t)q + SEG_LONG < nnz && keys[q + SEG_LONG] == keys[q]) lq[atomicAdd(&nl, 1)] = q;
    }
    __syncthreads();
    const int nlong = nl;
    for (int t = 0; t < nlong; ++t) {
      const uint32_t q0 = lq[t], key = keys[q0];
      // keys[lo] == key, keys[hi] != key (or hi == nnz): the run ends at hi
      int64_t lo = (int64_t)q0 + SEG_LONG, hi = nnz;
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key) lo = mid; else hi = mid;
      }
      const int64_t len = hi - (int64_t)q0, per = (len + LW - 1) / LW;
      const int64_t a = (int64_t)q0 + w * per;
      const int64_t b = a + per < hi ? a + per : hi;
      double acc[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) acc[u] = 0.0;
      constexpr int SU = 32;
      for (int64_t q = a; q < b; q += SU) {
        bool in[SU];
        uint32_t pp[SU];
#pragma unroll
        for (int e = 0; e < SU; ++e) {
          in[e] = q + e < b;
          pp[e] = in[e] ? perm[q + e] : 0u;
        }
        double vb[SU], mb[SU][CPL];
#pragma unroll
        for (int e = 0; e < SU; ++e) {
          vb[e] = !in[e] ? 0.0
                         : vdtype == 1 ? ((const double *)val)[pp[e]]
                                       : (double)((const float *)val)[pp[e]];
          const int64_t i = in[e] ? rid[pp[e]] : 0;
#pragma unroll
          for (int u = 0; u < CPL; ++u)
            mb[e][u] = in[e] && lane + 64 * u < K ? M[i * K + lane + 64 * u] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < SU; ++e)
          if (in[e])
#pragma unroll
            for (int u = 0; u < CPL; ++u)
              if (lane + 64 * u < K) acc[u] += vb[e] * mb[e][u];
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < K) part[w][lane + 64 * u] = acc[u];
      __syncthreads();
      if (w == 0) {
        T *dst = base + (int64_t)key * K;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const int c = lane + 64 * u;
          if (c < K) {
            double tot = 0.0;
            for (int ww = 0; ww < LW; ++ww) tot += part[ww][c];
            dst[c] = (T)((double)dst[c] + tot);
          }
        }
      }
      __syncthreads();
    }
  }
}

// The same row update for updates with few nonzeros, in one launch: block b
// owns the base rows of columns [b BW, (b+1) BW) and keeps their increments
// in LDS in the base's precision.  Thread t takes the contiguous nonzeros
// [t L, (t+1) L) of the CSR, counts its hits in the bucket, and one exclusive
// scan over the block lays the hits out in CSR order; wave 0 then adds them
// one after another, so every column sums its rows in row order whatever the
// scheduling (more hits than the buffer holds are taken in windows of
// SB_CAP).  The touched rows are then added to the base once.
constexpr int SB_NT = 512;
constexpr int SB_CAP = 1024;   // hits buffered per window
constexpr int SB_ITEMS = 64;   // nonzeros per thread: the kernel takes nnz <= SB_ITEMS SB_NT
constexpr int SB_LDS = 48 * 1024;   // bytes of increments per block

template <typename T, int K>
__global__ void __launch_bounds__(SB_NT)
k_scatter_bucket(int64_t s, int64_t cols, const int64_t *__restrict__ rp,
                 const int32_t *__restrict__ ci, const int32_t *__restrict__ rid,
                 const void *__restrict__ val, int vdtype, const double *__restrict__ M,
                 T *__restrict__ base, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int BW = SB_LDS / (int)sizeof(T) / K;   // columns per bucket
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  __shared__ T tab[BW * K];
  __shared__ int touched[BW];
  __shared__ int32_t mcol[SB_CAP], mrow[SB_CAP];
  __shared__ double mval[SB_CAP];
  __shared__ int wtot[SB_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * BW;
  const int64_t nnz = rp[s];
  const int L = (int)((nnz + SB_NT - 1) / SB_NT);
  const int64_t p0 = (int64_t)tid * L;
  for (int e = tid; e < BW * K; e += SB_NT) tab[e] = (T)0;
  for (int e = tid; e < BW; e += SB_NT) touched[e] = 0;
  // this thread's nonzeros: a bit per hit in the bucket
  uint64_t hits = 0;
#pragma unroll
  for (int r = 0; r < SB_ITEMS; ++r) {
    const int64_t p = p0 + r;
    const int32_t c = (r < L && p < nnz) ? ci[p] : -1;
    hits |= (c >= c0 && c < c0 + BW) ? (1ull << r) : 0ull;
  }
  const int mine = __popcll(hits);
  // exclusive scan of the counts: within the wave by shuffles, then the
  // wave totals
  int incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int woff = 0, total = 0;
  for (int v = 0; v < SB_NT / 64; ++v) {
    woff += v < w ? wtot[v] : 0;
    total += wtot[v];
  }
  const int first = woff + incl - mine;   // index of this thread's first hit
  for (int h0 = 0; h0 < total; h0 += SB_CAP) {
    // the hits with index in [h0, h0 + SB_CAP), in order
    int idx = first;
    for (uint64_t m = hits; m; m &= m - 1, ++idx) {
      if (idx < h0 || idx >= h0 + SB_CAP) continue;
      const int64_t p = p0 + __builtin_ctzll(m);
      const int slot = idx - h0;
      mcol[slot] = (int32_t)(ci[p] - c0);
      mrow[slot] = rid[p];
      mval[slot] = vdtype == 1 ? ((const double *)val)[p] : (double)((const float *)val)[p];
    }
    __syncthreads();
    if (w == 0) {
      const int n = total - h0 < SB_CAP ? total - h0 : SB_CAP;
      for (int q0 = 0; q0 < n; q0 += 8) {
        double mv[8][CPL];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int v = 0; v < CPL; ++v) {
            const int j = lane + 64 * v;
            mv[u][v] = (q0 + u < n && j < K) ? M[(int64_t)mrow[q0 + u] * K + j] : 0.0;
          }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (q0 + u < n) {
            const int cl = mcol[q0 + u];
            const double x = mval[q0 + u];
#pragma unroll
            for (int v = 0; v < CPL; ++v) {
              const int j = lane + 64 * v;
              if (j < K) tab[cl * K + j] = (T)((double)tab[cl * K + j] + x * mv[u][v]);
            }
            if (lane == 0) touched[cl] = 1;
          }
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < BW * K; e += SB_NT) {
    const int cl = e / K, j = e % K;
    if (touched[cl] && c0 + cl < cols) {
      T *dst = base + (c0 + cl) * K + j;
      *dst = *dst + tab[e];
    }
  }
}

}  // namespace

namespace svl {

size_t csr_transpose_bytes(int64_t nnz, int64_t n) {
  const int64_t tiles = (nnz + RS_TILE - 1) / RS_TILE;
  const int64_t nh = (tiles > 0 ? tiles : 1) * RS_DIG;
  return (size_t)nnz * (4 * sizeof(uint32_t) + sizeof(int32_t)) + (size_t)nh * sizeof(uint32_t) +
         (size_t)((nh + SC_TILE - 1) / SC_TILE + 1) * sizeof(uint32_t) + 1024;
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
  uint32_t *bsum = hist + (tiles > 0 ? tiles : 1) * RS_DIG;
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
      const int64_t nh = tiles * RS_DIG, nb = (nh + SC_TILE - 1) / SC_TILE;
      hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SC_NT), 0, st, nh, hist, bsum, info);
      hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(SC_NT), 0, st, nb, bsum, info);
      hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SC_NT), 0, st, nh, hist, bsum, info);
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

size_t scatter_det_bytes(int64_t nnz) {
  return csr_transpose_bytes(nnz, 0) + (size_t)nnz * sizeof(uint32_t) + 256;
}

template <typename T, int K>
static void scatter_bucket_launch(hipStream_t st, int64_t s, int64_t cols, int64_t nnz,
                                  const int64_t *rp, const int32_t *ci, const void *v, int vdt,
                                  const double *M, T *base, int32_t *rid, const SvDevInfo *info) {
  constexpr int BW = SB_LDS / (int)sizeof(T) / K;
  hipLaunchKernelGGL(k_row_ids, dim3(grid_for(s, 4, 1 << 20)), dim3(256), 0, st, s, nnz, rp, rid,
                     info);
  const unsigned nb = (unsigned)((cols + BW - 1) / BW);
  hipLaunchKernelGGL((k_scatter_bucket<T, K>), dim3(nb), dim3(SB_NT), 0, st, s, cols, rp, ci, rid,
                     v, vdt, M, base, info);
}

template <typename T>
void scatter_det(hipStream_t st, int K, int64_t s, int64_t cols, int64_t nnz, const int64_t *rp,
                 const int32_t *ci, const void *v, int vdt, const double *M, T *base,
                 void *scratch, const SvDevInfo *info) {
  if (s <= 0 || nnz <= 0) return;
  // few nonzeros against the column buckets: every bucket scans them all, in
  // one launch; otherwise the sort
  const int64_t bw = SB_LDS / (int64_t)sizeof(T) / K;
  const int64_t buckets = (cols + bw - 1) / bw;
  if (nnz <= (int64_t)SB_ITEMS * SB_NT && (double)nnz * (double)buckets <= (double)(1ll << 26)) {
    switch (K) {
      case 16: scatter_bucket_launch<T, 16>(st, s, cols, nnz, rp, ci, v, vdt, M, base,
                                              (int32_t *)scratch, info); break;
      case 32: scatter_bucket_launch<T, 32>(st, s, cols, nnz, rp, ci, v, vdt, M, base,
                                              (int32_t *)scratch, info); break;
      case 64: scatter_bucket_launch<T, 64>(st, s, cols, nnz, rp, ci, v, vdt, M, base,
                                              (int32_t *)scratch, info); break;
      case 128: scatter_bucket_launch<T, 128>(st, s, cols, nnz, rp, ci, v, vdt, M, base,
                                              (int32_t *)scratch, info); break;
    }
    return;
  }
  const int64_t tiles = (nnz + RS_TILE - 1) / RS_TILE;
  char *p = (char *)scratch;
  uint32_t *ka = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *kb = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *pa = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *pb = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  int32_t *rid = (int32_t *)p; p += (size_t)nnz * sizeof(int32_t);
  uint32_t *hist = (uint32_t *)p;
  const int64_t nh = (tiles > 0 ? tiles : 1) * RS_DIG;
  uint32_t *bsum = hist + nh;
  p = (char *)(bsum + (nh + SC_TILE - 1) / SC_TILE + 1);
  uint32_t *heads = (uint32_t *)p; p += (size_t)nnz * sizeof(uint32_t);
  uint32_t *count = (uint32_t *)p;
  hipLaunchKernelGGL(k_row_ids, dim3(grid_for(s, 4, 1 << 20)), dim3(256), 0, st, s, nnz, rp, rid,
                     info);
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < cols) ++bits;
  const int passes = (bits + 7) / 8;
  const uint32_t *kin = (const uint32_t *)ci;
  const uint32_t *pin = nullptr;
  for (int ps = 0; ps < passes; ++ps) {
    uint32_t *kout = (ps & 1) ? kb : ka;
    uint32_t *pout = (ps & 1) ? pb : pa;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)tiles), dim3(RS_NT), 0, st, nnz, kin, 8 * ps,
                       tiles, hist, info);
    const int64_t nb = (nh + SC_TILE - 1) / SC_TILE;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SC_NT), 0, st, nh, hist, bsum, info);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(SC_NT), 0, st, nb, bsum, info);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SC_NT), 0, st, nh, hist, bsum, info);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(RS_NT), 0, st, nnz, kin, pin,
                       8 * ps, tiles, hist, kout, pout, info);
    kin = kout;
    pin = pout;
  }
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, count, info);
  hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, st, nnz, kin,
                     heads, count, info);
  const unsigned blocks = (unsigned)std::min<int64_t>((nnz + 3) / 4, 16384);
#define SV_SS(KK) hipLaunchKernelGGL((k_scatter_seg<T, KK>), dim3(blocks), dim3(256), 0, st, nnz, \
                                     kin, pin, heads, count, rid, v, vdt, M, base, info)
  switch (K) {
    case 16: SV_SS(16); break;
    case 32: SV_SS(32); break;
    case 64: SV_SS(64); break;
    case 128: SV_SS(128); break;
  }
#undef SV_SS
  if (nnz > SEG_LONG) {   // runs longer than SEG_LONG exist only then
    const unsigned lb = (unsigned)std::min<int64_t>(nnz / SEG_LONG, 1024);
#define SV_SL(KK) hipLaunchKernelGGL((k_scatter_long<T, KK>), dim3(lb), dim3(LW * 64), 0, st, nnz, \
                                     kin, pin, heads, count, rid, v, vdt, M, base, info)
    switch (K) {
      case 16: SV_SL(16); break;
      case 32: SV_SL(32); break;
      case 64: SV_SL(64); break;
      case 128: SV_SL(128); break;
    }
#undef SV_SL
  }
}
template void scatter_det<float>(hipStream_t, int, int64_t, int64_t, int64_t, const int64_t *,
                                 const int32_t *, const void *, int, const double *, float *,
                                 void *, const SvDevInfo *);
template void scatter_det<double>(hipStream_t, int, int64_t, int64_t, int64_t, const int64_t *,
                                  const int32_t *, const void *, int, const double *, double *,
                                  void *, const SvDevInfo *);

void check_finite_wide(hipStream_t st, int64_t n, const double *x, SvDevInfo *info) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_finite_wide, dim3(grid_for(n, 256 * 8, 2048)), dim3(256), 0, st, n,
                     x, info);
}

// Gram of a tall panel on FP64 MFMA; ws must hold ts_gram_ws(R, L) doubles.
size_t ts_gram_ws(int64_t R, int L) {
  const int LT = L / 16, NT = LT * (LT + 1) / 2;
  const int64_t Z = std::min<int64_t>(256, std::max<int64_t>(1, (R + 127) / 128));
  return (size_t)(Z + 16) * NT * 256;
}

void ts_gram_if(hipStream_t st, int64_t R, int L, const double *Y, double *G, double *ws,
                const SvDevInfo *info, const int32_t *need) {
  const int LT = L / 16, NT = LT * (LT + 1) / 2;
  int64_t Z = std::min<int64_t>(256, std::max<int64_t>(1, (R + 127) / 128));
  int64_t rpb = (R + Z - 1) / Z;
  rpb = (rpb + TG_KC - 1) / TG_KC * TG_KC;
  Z = std::max<int64_t>(1, (R + rpb - 1) / rpb);
  const int S = (int)std::min<int64_t>(16, Z);
  const int64_t NE = (int64_t)NT * 256;
  double *part = ws, *part2 = ws + Z * NE;
#define SV_TG(LL) hipLaunchKernelGGL((k_ts_gram<LL>), dim3((unsigned)Z), dim3(256), 0, st, R, rpb, \
                                     Y, part, info, need)
  switch (L) { case 16: SV_TG(16); break; case 32: SV_TG(32); break;
               case 64: SV_TG(64); break; case 128: SV_TG(128); break; }
#undef SV_TG
  hipLaunchKernelGGL(k_gram_reduce1, dim3((unsigned)((NE + 255) / 256), (unsigned)S), dim3(256), 0,
                     st, (int)Z, S, NE, part, part2, info, need);
  hipLaunchKernelGGL(k_gram_reduce2, dim3((unsigned)((NE + 255) / 256)), dim3(256), 0, st, L, S,
                     part2, G, info, need);
}

void ts_gram(hipStream_t st, int64_t R, int L, const double *Y, double *G, double *ws,
             const SvDevInfo *info) {
  ts_gram_if(st, R, L, Y, G, ws, info, nullptr);
}

void ts_mul_lt(hipStream_t st, int64_t R, int L, const double *X, const double *Out, double *Y,
               const SvDevInfo *info) {
  const unsigned nb = (unsigned)((R + 63) / 64);
#define SV_TM(LL) hipLaunchKernelGGL((k_ts_mul_lt<LL>), dim3(nb), dim3(256), 0, st, R, X, Out, Y, info)
  switch (L) { case 16: SV_TM(16); break; case 32: SV_TM(32); break;
               case 64: SV_TM(64); break; case 128: SV_TM(128); break; }
#undef SV_TM
}

void chol_drop_if(hipStream_t st, int L, const double *G, double *Out, int32_t *complete,
                  double rtol, const SvDevInfo *info, const int32_t *need) {
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    allow_big_lds(k_chol_drop);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once_b = [] {
    allow_big_lds(k_chol_drop_blk);
    (void)hipGetLastError();
    return true;
  }();
  (void)once_b;
  if (L % 16 == 0 && L <= 128) {
    const size_t shb = ((size_t)L * (L + 3) + (size_t)CB_NW * 16 * 17) * sizeof(double) +
                       (size_t)L * sizeof(int);
    hipLaunchKernelGGL(k_chol_drop_blk, dim3(1), dim3(CB_NT), shb, st, L, G, Out, complete, rtol,
                       info, need);
    return;
  }
  const size_t sh = (size_t)L * (L + 2) * sizeof(double) + (size_t)L * sizeof(int);
  hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(CD_NT), sh, st, L, G, Out, complete, rtol, info,
                     need);
}

void chol_drop(hipStream_t st, int L, const double *G, double *Out, int32_t *complete,
               double rtol, const SvDevInfo *info) {
  chol_drop_if(st, L, G, Out, complete, rtol, info, nullptr);
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

// Orthonormal basis of the columns of the R x L panel X (R >= L) by passes
// of Cholesky QR with column dropping, alternating between X and Y; returns
// the buffer that holds the result (Y after an odd number of passes, X after
// an even one).  Each pass keeps the columns that are independent to within
// rtol (squared, relative to the largest column) and replaces the others by
// random columns, which in R >> L dimensions are nearly orthogonal to the
// kept ones; one pass leaves a basis of condition number 1 + O(u kappa^2)
// for kept columns of condition number kappa up to ~1/sqrt(rtol), which is
// what a power iteration needs, and a second pass makes it orthonormal to
// rounding.  Without dropping the columns keep their order: column j of the
// result spans the first j + 1 columns of X.
double *orth_cols(hipStream_t st, int64_t R, int L, double *X, double *Y, int passes, double *G,
                  double *Out, int32_t *complete, double *ws, size_t ws_len, uint64_t seed,
                  double rtol, const SvDevInfo *info) {
  double *src = X, *dst = Y;
  const bool mf = (L == 16 || L == 32 || L == 64 || L == 128) && ws_len >= ts_gram_ws(R, L);
  for (int pass = 0; pass < passes; ++pass) {
    if (mf) ts_gram(st, R, L, src, G, ws, info);
    else gemm_f64_sk(st, true, false, L, L, R, 1.0, src, L, src, L, 0.0, G, L, ws, ws_len, info);
    chol_drop(st, L, G, Out, complete, rtol, info);
    if (mf) ts_mul_lt(st, R, L, src, Out, dst, info);
    else gemm_f64(st, false, true, R, L, L, 1.0, src, L, Out, L, 0.0, dst, L, info);
    fill_cols(st, R, L, dst, complete, seed * 3 + (uint64_t)pass, info);
    double *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// orth_cols with two passes, the second gated on k_orth_gate: it runs only
// when the first pass completed a column or its input was not orthonormal to
// within ORTH_GATE_TAU, and otherwise the product copies the panel (the gated
// Cholesky writes Out = I), so the result is in X either way.  For the
// factors of the initial SVD (U = Q F and V = W F diag(1/sigma)) the input is
// orthonormal to rounding unless some column had to be completed.
double *orth_cols_cond(hipStream_t st, int64_t R, int L, double *X, double *Y, double *G,
                       double *Out, int32_t *complete, int32_t *need, double *ws, size_t ws_len,
                       uint64_t seed, double rtol, const SvDevInfo *info, double gate_tau) {
  const bool mf = (L == 16 || L == 32 || L == 64 || L == 128) && ws_len >= ts_gram_ws(R, L);
  double *src = X, *dst = Y;
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t *gate = pass == 0 ? nullptr : need;
    if (mf) ts_gram_if(st, R, L, src, G, ws, info, gate);
    else gemm_f64_sk(st, true, false, L, L, R, 1.0, src, L, src, L, 0.0, G, L, ws, ws_len, info);
    chol_drop_if(st, L, G, Out, complete, rtol, info, gate);
    if (pass == 0)
      hipLaunchKernelGGL(k_orth_gate, dim3(1), dim3(1024), (size_t)L * sizeof(double), st, L, G,
                         complete, gate_tau, need, info);
    if (mf) ts_mul_lt(st, R, L, src, Out, dst, info);
    else gemm_f64(st, false, true, R, L, L, 1.0, src, L, Out, L, 0.0, dst, L, info);
    fill_cols(st, R, L, dst, complete, seed * 3 + (uint64_t)pass, info);
    double *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace svl
