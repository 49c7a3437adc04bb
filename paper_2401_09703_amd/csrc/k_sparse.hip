// Sparse kernels of one update: input validation, the projection of the
// update onto the tall factor (SpMM with the k x k factor as epilogue), the
// sparse Gram E E^T, and the two writes into the tall factors (the sparse row
// update and the appended rows).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

__device__ __forceinline__ void fail(SvDevInfo *info, int code, int seq) {
  if (atomicCAS(&info->status, 0, code) == 0) info->failed_seq = seq;
}

// Canonical-CSR check (0-based, monotone row_ptr, strictly increasing
// in-range column ids per row, finite values), one wave per row with the
// row's entries spread over the lanes (each lane compares its entry with the
// one before it).  Every access is bounded by the declared nnz, so a
// malformed row_ptr cannot push reads out of range.  Within a row a
// structural error is reported before a non-finite value.
__global__ void __launch_bounds__(256)
k_validate_csr(int64_t rows, int64_t cols, int64_t nnz, const int64_t *__restrict__ row_ptr,
               const int32_t *__restrict__ col_idx, const void *__restrict__ val, int vdtype,
               SvDevInfo *info, int seq) {
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (row_ptr[0] != 0 || row_ptr[rows] != nnz) fail(info, 1, seq);
  }
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < rows;
       i += (int64_t)gridDim.x * 4) {
    const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
    if (p0 < 0 || p1 < p0 || p1 > nnz) {
      if (lane == 0) fail(info, 1, seq);
      continue;
    }
    bool bad_s = false, bad_v = false;
    for (int64_t p = p0 + lane; p < p1; p += 64) {
      const int32_t c = col_idx[p];
      const int32_t prev = p > p0 ? col_idx[p - 1] : -1;
      bad_s |= c <= prev || c >= cols;
      const double v = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
      bad_v |= !isfinite(v);
    }
    const bool any_s = __ballot(bad_s) != 0, any_v = __ballot(bad_v) != 0;
    if (lane == 0 && (any_s || any_v)) fail(info, any_s ? 1 : 4, seq);
  }
}

// Row kernels take one block of SP_NW waves per row of E: the waves take
// interleaved chunks of 64 nonzeros, each chunk loaded coalesced (one nonzero
// per lane) and then broadcast lane by lane with shuffles, so that a lane
// keeps SP_U independent gathers of base rows in flight.  Long (hub) rows are
// thus spread over SP_NW waves and never wait on one load per nonzero.
constexpr int SP_NW = 4;
constexpr int SP_U = 8;

__device__ __forceinline__ double ldv(const void *val, int vdtype, int64_t p) {
  return vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
}

// Row i of P = E * base (K columns, accumulated in A: T, or FP64 for FP32
// storage where the caller needs C' to FP64 rounding), C'[i] = P[i] W (FP64,
// W is K x K FP64) and ||e_i||^2, by one block of SP_NW waves.  For K <= 64 a
// wave splits into 64/K groups of K lanes that take alternate nonzeros of a
// chunk; for K = 128 each lane owns two columns.  red (SP_NW x K), ptot (K)
// and nred (SP_NW) are LDS scratch of the caller.
template <typename T, typename A, int K>
__device__ __forceinline__ void
spmm_row(int64_t i, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
         const void *__restrict__ val, int vdtype, const T *__restrict__ base,
         const double *__restrict__ W, double *__restrict__ Cp64, float *__restrict__ Cp32,
         double *__restrict__ rownorm2, double *red, double *ptot, double *nred) {
  constexpr int G = K <= 64 ? 64 / K : 1;
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / (64 / G), c = lane % (64 / G);
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  A acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = (A)0;
  double nrm = 0.0;
  for (int64_t cb = p0 + 64 * w; cb < p1; cb += 64 * SP_NW) {
    const int n = (int)((p1 - cb) < 64 ? (p1 - cb) : 64);
    int32_t mc = 0;
    double mvd = 0.0;
    if (lane < n) {
      mc = col_idx[cb + lane];
      mvd = ldv(val, vdtype, cb + lane);
    }
    nrm += mvd * mvd;
    const A mv = (A)mvd;
    // lanes >= n carry column 0 and value 0: their gathers are valid and add 0
    for (int j0 = 0; j0 < n; j0 += SP_U * G) {
      int32_t cc[SP_U];
      A vv[SP_U];
#pragma unroll
      for (int u = 0; u < SP_U; ++u) {
        const int jj = j0 + u * G + g;
        cc[u] = __shfl(mc, jj, 64);
        vv[u] = __shfl(mv, jj, 64);
      }
      T bb[SP_U][CPL];
#pragma unroll
      for (int u = 0; u < SP_U; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) bb[u][q] = base[(int64_t)cc[u] * K + c + 64 * q];
#pragma unroll
      for (int u = 0; u < SP_U; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] += vv[u] * (A)bb[u][q];
    }
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int o = K; o < 64; o <<= 1) acc[0] += __shfl_xor(acc[0], o, 64);
  }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) red[w * K + c + 64 * q] = (double)acc[q];
  }
  nrm = wave_sum(nrm);
  if (lane == 0) nred[w] = nrm;
  __syncthreads();
  for (int t = threadIdx.x; t < K; t += 64 * SP_NW) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < SP_NW; ++q) sum += red[q * K + t];
    ptot[t] = sum;
  }
  __syncthreads();
  // epilogue: C'[i, col] = sum_l P[i, l] W[l, col]
  for (int col = threadIdx.x; col < K; col += 64 * SP_NW) {
    double out = 0.0;
#pragma unroll 8
    for (int l = 0; l < K; ++l) out += ptot[l] * W[l * K + col];
    Cp64[i * K + col] = out;
    if (Cp32) Cp32[i * K + col] = (float)out;
  }
  if (threadIdx.x == 0) {
    double tn = 0.0;
    for (int q = 0; q < SP_NW; ++q) tn += nred[q];
    rownorm2[i] = tn;
  }
}

// The projection of one update: one block per row of E.
template <typename T, typename A, int K>
__global__ void __launch_bounds__(64 * SP_NW)
k_spmm_w(int64_t s, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
         const void *__restrict__ val, int vdtype, const T *__restrict__ base,
         const double *__restrict__ W, double *__restrict__ Cp64, float *__restrict__ Cp32,
         double *__restrict__ rownorm2, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double red[SP_NW * K];
  __shared__ double ptot[K];
  __shared__ double nred[SP_NW];
  spmm_row<T, A, K>((int64_t)blockIdx.x, row_ptr, col_idx, val, vdtype, base, W, Cp64, Cp32,
                 rownorm2, red, ptot, nred);
}

// 16-byte vectors of the base storage type: one gather per lane moves four
// FP32 or two FP64 columns of a base row.
typedef float sv_f4 __attribute__((ext_vector_type(4)));
typedef double sv_d2 __attribute__((ext_vector_type(2)));
template <typename T> struct Wide;
template <> struct Wide<float> { typedef sv_f4 V; static constexpr int E = 4; };
template <> struct Wide<double> { typedef sv_d2 V; static constexpr int E = 2; };

// Row i of P = E * base accumulated by one wave (T accumulate).  A base row of
// K columns is read by LPR = K/E lanes with one 16-byte load each, so one
// load instruction gathers G = 64/LPR rows (G nonzeros of E) and a lane keeps
// U such loads in flight; loads past the row's last nonzero are skipped (a
// uniform branch).  Lanes of group 0 end with P[i][c..c+E) in out (LDS);
// *nrm_out receives ||e_i||^2.
template <typename T, int K, int U>
__device__ __forceinline__ void
wave_row_project(int64_t i, const int64_t *__restrict__ row_ptr,
                 const int32_t *__restrict__ col_idx, const void *__restrict__ val, int vdtype,
                 const T *__restrict__ base, double *out, double *nrm_out) {
  typedef typename Wide<T>::V V;
  constexpr int E = Wide<T>::E;
  constexpr int LPR = K / E;                   // lanes per base row
  constexpr int G = 64 / LPR;                  // base rows per load
  constexpr int NB = U * G;                    // nonzeros per batch of loads
  constexpr int CH = NB > 64 ? NB / 64 : 1;    // CSR entries held per lane
  constexpr int CW = 64 * CH;                  // nonzeros per CSR chunk
  static_assert(LPR >= 1 && LPR <= 64 && (NB % 64 == 0 || 64 % NB == 0), "tile shape");
  const int lane = threadIdx.x & 63;
  const int g = lane / LPR, c = (lane % LPR) * E;
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  V acc = (V)(T)0;
  double nrm = 0.0;
  for (int64_t cb = p0; cb < p1; cb += CW) {
    const int n = (int)((p1 - cb) < CW ? (p1 - cb) : CW);
    int32_t mc[CH];
    T mv[CH];
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int p = h * 64 + lane;
      mc[h] = 0;
      mv[h] = (T)0;
      if (p < n) {
        mc[h] = col_idx[cb + p];
        const double x = ldv(val, vdtype, cb + p);
        nrm += x * x;
        mv[h] = (T)x;
      }
    }
    // one pass when NB >= CW, else CW / NB passes over the chunk
    for (int j0 = 0; j0 < n; j0 += NB) {
      V bb[U];
      T vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int h = (u * G) / 64;              // j0 == 0 whenever CH > 1
        const int jj = (j0 + u * G + g) & 63;
        const int32_t col = __shfl(mc[h], jj, 64);
        vv[u] = __shfl(mv[h], jj, 64);
        bb[u] = (V)(T)0;
        if (j0 + u * G < n) bb[u] = *(const V *)(base + (int64_t)col * K + c);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += vv[u] * bb[u];
    }
  }
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] += __shfl_xor(acc[e], o, 64);
  if (g == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) out[c + e] = (double)acc[e];
  }
  nrm = wave_sum(nrm);
  if (lane == 0) *nrm_out = nrm;
}

// The projections of many updates of one rank, storage type and tile shape
// in one launch (a batch of mixed ones is one launch per group, so each
// launch keeps the registers of its own shape and its occupancy).  Block b
// takes tile t = order[b], a tile of RB consecutive rows of the request whose
// tiles start at row0 <= t: each wave accumulates whole rows of P (one row at
// a time, 16-byte gathers, U in flight per lane), the tile's rows of P meet
// in LDS, and C' = P W is formed for the tile with each element of W read
// once (from L2) by the thread that owns its column and part of the inner
// index.  (U, RB) is chosen per launch from the tuning table by storage
// type, rank and the bin of the launch's mean nonzeros per row.
constexpr int SV_XCDS = 8;   // MI355X: workgroup b runs on XCD b mod 8

template <typename T, int K, int U, int RB>
__global__ void __launch_bounds__(64 * SP_NW)
k_spmm_batch(int n, const svl::ProjDesc *__restrict__ descs, const int32_t *__restrict__ order) {
  constexpr int Q = 64 * SP_NW / K;   // parts of the inner index in C' = P W
  constexpr int LQ = K / Q;
  __shared__ double Pt[RB][K];
  __shared__ double Pp[Q][RB][K];
  __shared__ double nr[RB];
  const int64_t t = order[blockIdx.x];
  if (t < 0) return;
  int lo = 0, hi = n - 1;   // last request with row0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].row0 <= t) lo = mid; else hi = mid - 1;
  }
  const svl::ProjDesc &d = descs[lo];
  if (d.info && d.info->status) return;
  const int64_t i0 = (t - d.row0) * RB;
  const int rows = (int)((d.s - i0) < RB ? (d.s - i0) : RB);
  if (rows <= 0) return;
  const int tid = threadIdx.x, w = tid >> 6;
  for (int rr = w; rr < rows; rr += SP_NW)
    wave_row_project<T, K, U>(i0 + rr, d.row_ptr, d.col_idx, d.val, d.vdtype, (const T *)d.base,
                           Pt[rr], &nr[rr]);
  for (int rr = rows + w; rr < RB; rr += SP_NW)   // rows past the end stay finite
    for (int c = tid & 63; c < K; c += 64) Pt[rr][c] = 0.0;
  __syncthreads();
  // thread (part, col): the part's LQ inner indices for all rows of the tile,
  // so every element of W is read once per tile
  {
    const int col = tid % K, part = tid / K;
    double o[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) o[r] = 0.0;
    constexpr int UB = LQ < 16 ? LQ : 16;   // W loads in flight per thread
#pragma unroll 1
    for (int u0 = 0; u0 < LQ; u0 += UB) {
      double wv[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) wv[u] = d.W[(part * LQ + u0 + u) * K + col];
#pragma unroll
      for (int u = 0; u < UB; ++u)
#pragma unroll
        for (int r = 0; r < RB; ++r) o[r] += Pt[r][part * LQ + u0 + u] * wv[u];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) Pp[part][r][col] = o[r];
  }
  __syncthreads();
  for (int e = tid; e < rows * K; e += 64 * SP_NW) {
    const int rr = e / K, col = e % K;
    double o = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) o += Pp[q][rr][col];
    d.Cp64[(i0 + rr) * K + col] = o;
    if (d.Cp32) d.Cp32[(i0 + rr) * K + col] = (float)o;
  }
  if (tid < rows) d.rown[i0 + tid] = nr[tid];
}

// row id of every nonzero (the CSR row pointers expanded)
__global__ void k_row_ids(int64_t s, const int64_t *__restrict__ row_ptr,
                          int32_t *__restrict__ rid, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= s) return;
  for (int64_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) rid[p] = (int32_t)i;
}

// Dense updates (s >= 512, density >= GRAM_DENSE_MIN, long rows): S = E E^T as a sum
// of D D^T over column blocks D of E made dense in workspace, since the
// sparse kernel's cost grows with the product of the rows' lengths.
constexpr double GRAM_DENSE_MIN = 0.02;

// cur[i] = row_ptr[i]: the first nonzero of row i not yet made dense.
__global__ void k_row_cursor(int64_t s, const int64_t *__restrict__ row_ptr,
                             int64_t *__restrict__ cur, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < s) cur[i] = row_ptr[i];
}

__global__ void k_fill_zero(int64_t n, double *__restrict__ x, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

// Row i's nonzeros with columns in [c0, c0 + nb) into D[i][col - c0]; they
// follow cur[i] (columns are sorted), which moves past them.  One wave per row.
__global__ void k_densify(int64_t s, const int64_t *__restrict__ row_ptr,
                          const int32_t *__restrict__ col_idx, const void *__restrict__ val,
                          int vdtype, int64_t c0, int64_t nb, int64_t *__restrict__ cur,
                          double *__restrict__ D, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= s) return;
  const int64_t end = row_ptr[i + 1];
  int64_t p = cur[i];
  while (p < end) {
    const int64_t q = p + lane;
    const bool in = q < end && (int64_t)col_idx[q] < c0 + nb;
    if (in) D[i * nb + ((int64_t)col_idx[q] - c0)] = ldv(val, vdtype, q);
    const int taken = __popcll(__ballot(in));   // an in-range prefix of the chunk
    p += taken;
    if (taken < 64) break;
  }
  if (lane == 0) cur[i] = p;
}

constexpr int GRAM_LDS_CAP = 4096;      // nonzeros of the pivot row kept in LDS

// S = E E^T (FP64, full s x s).  Block b handles rows i = b and s-1-b (folded
// so that every block does about s/2 row pairs).  Row i is staged in LDS; the
// nonzeros of rows 0..i are contiguous in the CSR, so the block streams them
// with coalesced loads (one nonzero per thread), finds each column in row i
// by binary search, and accumulates the products per row j in LDS.  The sums
// are kept in 64-bit fixed point with 2^61 standing for scale = max_i
// ||e_i||^2 (every |S_ij| is at most that, by Cauchy-Schwarz): integer
// additions commute, so S is bitwise the same whatever order the atomics
// land in, and each product is rounded to 2^-62 scale, far below the
// Cholesky's pivot floor (>= 1e-13 scale).
__global__ void __launch_bounds__(256)
k_sparse_gram(int64_t s, const int64_t *__restrict__ row_ptr,
              const int32_t *__restrict__ col_idx, const int32_t *__restrict__ rid,
              const void *__restrict__ val, int vdtype, double *__restrict__ S,
              int64_t lds, const SvDevInfo *__restrict__ info, int which) {
  if (info->status) return;
  __shared__ int32_t sc[GRAM_LDS_CAP];
  __shared__ double sv[GRAM_LDS_CAP];
  extern __shared__ unsigned long long acc[];   // s fixed-point sums
  const double scale = which == 0 ? info->scale : info->scale2;
  const double fx = scale > 0.0 ? 2305843009213693952.0 / scale : 0.0;   // 2^61 / scale
  const double unfx = scale > 0.0 ? scale / 2305843009213693952.0 : 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t i = pass == 0 ? (int64_t)blockIdx.x : s - 1 - (int64_t)blockIdx.x;
    if (pass == 1 && i <= (int64_t)blockIdx.x) break;
    if (i < 0 || i >= s) continue;
    const int64_t q0 = row_ptr[i], q1 = row_ptr[i + 1];
    const int64_t ni = q1 - q0;
    const bool in_lds = ni <= GRAM_LDS_CAP;
    __syncthreads();
    if (in_lds) {
      for (int64_t t = threadIdx.x; t < ni; t += blockDim.x) {
        sc[t] = col_idx[q0 + t];
        sv[t] = ldv(val, vdtype, q0 + t);
      }
    }
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x) acc[j] = 0ull;
    __syncthreads();
    const int32_t *ci = in_lds ? sc : col_idx + q0;
    if (ni > 0) {
      // GU column indices per thread are loaded together before any search,
      // so that a block has GU loads in flight per thread, not one
      constexpr int GU = 8;
      for (int64_t p0 = threadIdx.x; p0 < q1; p0 += (int64_t)GU * blockDim.x) {
        int32_t cs[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
          const int64_t p = p0 + (int64_t)u * blockDim.x;
          cs[u] = p < q1 ? col_idx[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
          const int64_t p = p0 + (int64_t)u * blockDim.x;
          const int32_t c = cs[u];
          if (c < 0) continue;
          int64_t lo = 0, hi = ni;   // first position with ci[pos] >= c
          while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ci[mid] < c) lo = mid + 1; else hi = mid;
          }
          if (lo < ni && ci[lo] == c) {
            const double vi = in_lds ? sv[lo] : ldv(val, vdtype, q0 + lo);
            const long long q = __double2ll_rn(vi * ldv(val, vdtype, p) * fx);
            atomicAdd(&acc[rid[p]], (unsigned long long)q);
          }
        }
      }
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x) {
      const double a = (double)(long long)acc[j] * unfx;
      S[i * lds + j] = a;
      S[j * lds + i] = a;
    }
  }
}

// base[col] += sum_i E[i, col] * M[i]  (the sparse row update of the tall
// factor, Equation (1) second term), with FP atomics; nonzeros are taken in
// coalesced chunks as in k_spmm_w.
template <typename T, int K>
__global__ void __launch_bounds__(64 * SP_NW)
k_scatter(int64_t s, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
          const void *__restrict__ val, int vdtype, const double *__restrict__ M,
          T *__restrict__ base, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int G = K <= 64 ? 64 / K : 1;
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = blockIdx.x;
  const int g = lane / (64 / G), c = lane % (64 / G);
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  double mrow[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) mrow[q] = M[i * K + c + 64 * q];
  for (int64_t cb = p0 + 64 * w; cb < p1; cb += 64 * SP_NW) {
    const int n = (int)((p1 - cb) < 64 ? (p1 - cb) : 64);
    int32_t mc = 0;
    double mv = 0.0;
    if (lane < n) {
      mc = col_idx[cb + lane];
      mv = ldv(val, vdtype, cb + lane);
    }
    // the loop is uniform over the wave so that every source lane of the
    // shuffles is active (a shuffle from an inactive lane reads zero)
    for (int j0 = 0; j0 < n; j0 += G) {
      const int jj = j0 + g;
      const int32_t cc = __shfl(mc, jj, 64);
      const double vv = __shfl(mv, jj, 64);
      if (jj < n) {
        T *dst = base + (int64_t)cc * K + c;
#pragma unroll
        for (int q = 0; q < CPL; ++q) atomicAdd(dst + 64 * q, (T)(vv * mrow[q]));
      }
    }
  }
}

// out[i] = X[i, :] * Winv, or X[i, :] when the k x k factor was reset to the
// identity, with X[i][l] = src[i * rs + l * cs].  Used for the appended rows of
// the tall factor (X = F[k:], Equation (1)) and for the sparse-update rows
// (X = T G[k:]).
template <typename T, int K>
__global__ void k_append(int64_t s, const double *__restrict__ src, int64_t rs, int64_t cs,
                         const double *__restrict__ Winv,
                         const int32_t *__restrict__ reset_flag,
                         T *__restrict__ out, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= s) return;
  const bool reset = reset_flag != nullptr && *reset_flag != 0;
  for (int j = lane; j < K; j += 64) {
    double acc = 0.0;
    if (reset) {
      acc = src[i * rs + (int64_t)j * cs];
    } else {
      for (int l = 0; l < K; ++l) acc += src[i * rs + (int64_t)l * cs] * Winv[l * K + j];
    }
    out[i * K + j] = (T)acc;
  }
}

// Y = A X for a CSR A (rows x cols) and a dense FP64 X (cols x L, row-major):
// one wave per row of A, its nonzeros gathered as in the projection (16-byte
// loads of rows of X, U of them in flight per lane); the lanes of group 0
// store the row of Y.
template <int L, int U>
__global__ void __launch_bounds__(256)
k_csr_dense(int64_t rows, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
            const void *__restrict__ val, int vdtype, const double *__restrict__ X,
            double *__restrict__ Y, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double nr[4];
  const int w = threadIdx.x >> 6;
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < rows; i += (int64_t)gridDim.x * 4)
    wave_row_project<double, L, U>(i, rp, ci, val, vdtype, X, Y + i * L, &nr[w]);
}

}  // namespace

// ---------------------------------------------------------------- launchers
namespace svl {

void validate_csr(hipStream_t st, int64_t rows, int64_t cols, int64_t nnz,
                  const int64_t *rp, const int32_t *ci, const void *v, int vdt,
                  SvDevInfo *info, int seq) {
  int64_t blocks = (rows + 3) / 4;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)blocks), dim3(256), 0, st,
                     rows, cols, nnz, rp, ci, v, vdt, info, seq);
}

template <typename T>
void spmm_w(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
            const void *v, int vdt, const T *base, const double *W, double *Cp64,
            float *Cp32, double *rownorm2, const SvDevInfo *info, bool acc64) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)s;
#define SV_SPMM(AA, KK) hipLaunchKernelGGL((k_spmm_w<T, AA, KK>), dim3(blocks), dim3(64 * SP_NW), 0, \
                                           st, s, rp, ci, v, vdt, base, W, Cp64, Cp32, rownorm2, info)
#define SV_SPMM_K(AA) \
  switch (K) {        \
    case 16: SV_SPMM(AA, 16); break; \
    case 32: SV_SPMM(AA, 32); break; \
    case 64: SV_SPMM(AA, 64); break; \
    case 128: SV_SPMM(AA, 128); break; \
  }
  if (acc64 || sizeof(T) == sizeof(double)) {
    SV_SPMM_K(double)
  } else {
    SV_SPMM_K(T)
  }
#undef SV_SPMM_K
#undef SV_SPMM
}
template void spmm_w<float>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                            const void *, int, const float *, const double *, double *,
                            float *, double *, const SvDevInfo *, bool);
template void spmm_w<double>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                             const void *, int, const double *, const double *, double *,
                             float *, double *, const SvDevInfo *, bool);

// Tile shapes of the fused projection: (16-byte loads in flight per lane,
// rows per tile).  Variant 0 is the default.
struct PbShape { int u, rb; };
constexpr PbShape PB_SHAPES[] = {{8, 8}, {4, 8}, {16, 8}, {8, 16}, {4, 16}, {8, 4}};
constexpr int PB_NSHAPES = (int)(sizeof(PB_SHAPES) / sizeof(PB_SHAPES[0]));

// Tuning table: variant per (FP64 storage, rank index log2(K/16), row bin),
// process-wide; written by the tuner through the C ABI, read per batch.
std::atomic<int> g_pb_tune[2][4][PB_ROW_BINS];

int k_index(int K) { return K <= 16 ? 0 : K <= 32 ? 1 : K <= 64 ? 2 : 3; }

int spmm_batch_rows_per_block() { return PB_SHAPES[0].rb; }
int spmm_variant_count() { return PB_NSHAPES; }
bool spmm_variant_shape(int v, int *u, int *rb) {
  if (v < 0 || v >= PB_NSHAPES) return false;
  *u = PB_SHAPES[v].u;
  *rb = PB_SHAPES[v].rb;
  return true;
}
int spmm_row_bin(int64_t nnz, int64_t s) {
  const double m = s > 0 ? (double)nnz / (double)s : 0.0;
  return m < 16.0 ? 0 : m < 64.0 ? 1 : m < 256.0 ? 2 : 3;
}
bool spmm_tune_set(int fp64, int K, int bin, int v) {
  if ((fp64 != 0 && fp64 != 1) || (K != 16 && K != 32 && K != 64 && K != 128) || bin < 0 ||
      bin >= PB_ROW_BINS || v < 0 || v >= PB_NSHAPES)
    return false;
  g_pb_tune[fp64][k_index(K)][bin].store(v, std::memory_order_relaxed);
  return true;
}
int spmm_tune_get(int fp64, int K, int bin) {
  if ((fp64 != 0 && fp64 != 1) || (K != 16 && K != 32 && K != 64 && K != 128) || bin < 0 ||
      bin >= PB_ROW_BINS)
    return -1;
  return g_pb_tune[fp64][k_index(K)][bin].load(std::memory_order_relaxed);
}

void ProjBatch::pack(void *host) const {
  char *p = (char *)host;
  std::memcpy(p, d.data(), d.size() * sizeof(ProjDesc));
  std::memcpy(p + d.size() * sizeof(ProjDesc), order.data(), order.size() * sizeof(int32_t));
}

ProjBatch spmm_batch_prepare(std::vector<ProjDesc> d) {
  // XCD-affine by default; SVLCOV_PROJ_ORDER=rr deals the tiles round-robin
  static const bool xcd_affine = [] {
    const char *e = std::getenv("SVLCOV_PROJ_ORDER");
    return !(e && std::strcmp(e, "rr") == 0);
  }();
  // one launch per (storage type, rank); its tile shape is the tuned one for
  // the group's mean nonzeros per row (kept in pad), so mixed row lengths do
  // not split a launch
  std::stable_sort(d.begin(), d.end(), [](const ProjDesc &a, const ProjDesc &b) {
    return a.fp64 != b.fp64 ? a.fp64 < b.fp64 : a.K < b.K;
  });
  ProjBatch out;
  size_t g0 = 0;
  while (g0 < d.size()) {
    size_t g1 = g0 + 1;
    while (g1 < d.size() && d[g1].fp64 == d[g0].fp64 && d[g1].K == d[g0].K) ++g1;
    int64_t gnnz = 0, gs = 0;
    for (size_t q = g0; q < g1; ++q) { gnnz += d[q].nnz; gs += d[q].s; }
    const int v = spmm_tune_get(d[g0].fp64, d[g0].K, spmm_row_bin(gnnz, gs));
    for (size_t q = g0; q < g1; ++q) d[q].pad = v < 0 ? 0 : v;
    const int RB = PB_SHAPES[d[g0].pad].rb;
    int64_t tiles = 0;
    for (size_t q = g0; q < g1; ++q) {
      d[q].row0 = tiles;
      tiles += (d[q].s + RB - 1) / RB;
    }
    if (!xcd_affine) {   // tiles in request order, dealt round-robin over the XCDs
      out.g_desc.push_back(g0);
      out.g_order.push_back(out.order.size());
      for (int64_t u = 0; u < tiles; ++u) out.order.push_back((int32_t)u);
      g0 = g1;
      continue;
    }
    // estimated cost of one tile of request q: its gathered elements plus the
    // K x K of W, in units of one gathered element
    const int K = d[g0].K;
    std::vector<double> tc(g1 - g0);
    double total_cost = 0.0;
    for (size_t q = g0; q < g1; ++q) {
      const int64_t nt = (d[q].s + RB - 1) / RB;
      tc[q - g0] = nt > 0 ? (double)d[q].nnz / (double)nt * K + (double)K * K : 0.0;
      total_cost += tc[q - g0] * (double)nt;
    }
    // chunks of at most a quarter of one XCD's share, costliest first, each
    // to the least loaded XCD (longest-processing-time rule)
    const double cap = total_cost / (4.0 * SV_XCDS);
    struct Chunk { int64_t t0, n; double cost; };
    std::vector<Chunk> ch;
    for (size_t q = g0; q < g1; ++q) {
      const int64_t nt = (d[q].s + RB - 1) / RB;
      const double c1 = tc[q - g0];
      const int64_t pieces = std::max<int64_t>(
          1, std::min<int64_t>(nt, (int64_t)std::ceil(c1 * (double)nt / std::max(cap, 1.0))));
      for (int64_t c = 0; c < pieces; ++c) {
        const int64_t a = nt * c / pieces, b = nt * (c + 1) / pieces;
        if (b > a) ch.push_back({d[q].row0 + a, b - a, c1 * (double)(b - a)});
      }
    }
    std::stable_sort(ch.begin(), ch.end(),
                     [](const Chunk &a, const Chunk &b) { return a.cost > b.cost; });
    std::vector<std::vector<int32_t>> lists(SV_XCDS);
    std::vector<double> load(SV_XCDS, 0.0);
    for (const Chunk &c : ch) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (int64_t u = 0; u < c.n; ++u) lists[x].push_back((int32_t)(c.t0 + u));
      load[x] += c.cost;
    }
    size_t len = 0;
    for (int x = 0; x < SV_XCDS; ++x) len = std::max(len, lists[x].size());
    out.g_desc.push_back(g0);
    out.g_order.push_back(out.order.size());
    const size_t base = out.order.size();
    out.order.resize(base + len * SV_XCDS, -1);
    for (int x = 0; x < SV_XCDS; ++x)
      for (size_t l = 0; l < lists[x].size(); ++l) out.order[base + l * SV_XCDS + x] = lists[x][l];
    g0 = g1;
  }
  out.g_desc.push_back(d.size());
  out.g_order.push_back(out.order.size());
  out.d = std::move(d);
  return out;
}

template <typename T, int K>
void launch_pb(hipStream_t st, int v, unsigned blocks, int n, const ProjDesc *dd,
               const int32_t *oo) {
#define SV_PBV(UU, RR) hipLaunchKernelGGL((k_spmm_batch<T, K, UU, RR>), dim3(blocks), \
                                          dim3(64 * SP_NW), 0, st, n, dd, oo)
  switch (v) {
    case 1: SV_PBV(4, 8); break;
    case 2: SV_PBV(16, 8); break;
    case 3: SV_PBV(8, 16); break;
    case 4: SV_PBV(4, 16); break;
    case 5: SV_PBV(8, 4); break;
    default: SV_PBV(8, 8); break;
  }
#undef SV_PBV
}

void spmm_batch(hipStream_t st, const ProjBatch &b, const void *blob_dev) {
  static_assert(PB_NSHAPES == 6, "launch_pb covers every tile shape");
  const ProjDesc *descs = (const ProjDesc *)blob_dev;
  const int32_t *order = (const int32_t *)((const char *)blob_dev + b.d.size() * sizeof(ProjDesc));
  for (size_t g = 0; g + 1 < b.g_desc.size(); ++g) {
    const size_t q0 = b.g_desc[g], o0 = b.g_order[g];
    const size_t blocks = b.g_order[g + 1] - o0;
    const int n = (int)(b.g_desc[g + 1] - q0);
    if (blocks == 0 || n == 0) continue;
    const ProjDesc *dd = descs + q0;
    const int32_t *oo = order + o0;
    const int v = b.d[q0].pad;
    const unsigned nb = (unsigned)blocks;
    if (b.d[q0].fp64) {
      switch (b.d[q0].K) {
        case 16: launch_pb<double, 16>(st, v, nb, n, dd, oo); break;
        case 32: launch_pb<double, 32>(st, v, nb, n, dd, oo); break;
        case 64: launch_pb<double, 64>(st, v, nb, n, dd, oo); break;
        default: launch_pb<double, 128>(st, v, nb, n, dd, oo); break;
      }
    } else {
      switch (b.d[q0].K) {
        case 16: launch_pb<float, 16>(st, v, nb, n, dd, oo); break;
        case 32: launch_pb<float, 32>(st, v, nb, n, dd, oo); break;
        case 64: launch_pb<float, 64>(st, v, nb, n, dd, oo); break;
        default: launch_pb<float, 128>(st, v, nb, n, dd, oo); break;
      }
    }
  }
}

// the update paths are exercised up to this many rows of E per update
constexpr int GRAM_MAX_ROWS = 8192;
int gram_max_rows() { return GRAM_MAX_ROWS; }

int64_t gram_dense_block(int64_t s, int64_t cols, int64_t nnz, size_t dws_len) {
  if (s <= 0 || cols <= 0 || dws_len == 0) return 0;
  const double dens = (double)nnz / ((double)s * (double)cols);
  // a small s gives the block products too few output tiles to fill the chip
  if (s < 512 || dens < GRAM_DENSE_MIN || nnz / s < 1024) return 0;
  const size_t avail = dws_len > (size_t)s ? dws_len - (size_t)s : 0;   // s cursors first
  int64_t nb = (int64_t)(avail / (size_t)s);
  nb = std::min<int64_t>(nb, 8192) / 64 * 64;
  if (nb < 256) return 0;
  return std::min<int64_t>(nb, (cols + 63) / 64 * 64);
}

void sparse_gram(hipStream_t st, int64_t s, int64_t cols, int64_t nnz, const int64_t *rp,
                 const int32_t *ci, const void *v, int vdt, int32_t *rid, double *S, int64_t lds,
                 double *dws, size_t dws_len, const SvDevInfo *info, int which) {
  if (s <= 0) return;
  const int64_t nb = gram_dense_block(s, cols, nnz, dws_len);
  if (nb > 0) {   // a dense update: S = sum over column blocks of D D^T
    int64_t *cur = (int64_t *)dws;
    double *D = dws + s;
    const unsigned rb = (unsigned)((s + 3) / 4);
    hipLaunchKernelGGL(k_row_cursor, dim3(rb), dim3(256), 0, st, s, rp, cur, info);
    for (int64_t c0 = 0; c0 < cols; c0 += nb) {
      const int64_t nbl = std::min<int64_t>(nb, cols - c0);
      const int64_t cnt = s * nb;
      hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 16384)),
                         dim3(256), 0, st, cnt, D, info);
      hipLaunchKernelGGL(k_densify, dim3(rb), dim3(256), 0, st, s, rp, ci, v, vdt, c0, nb, cur, D,
                         info);
      gemm_f64(st, false, true, s, s, nbl, 1.0, D, nb, D, nb, c0 == 0 ? 0.0 : 1.0, S, lds, info);
    }
    return;
  }
  hipLaunchKernelGGL(k_row_ids, dim3((unsigned)((s + 3) / 4)), dim3(256), 0, st, s, rp, rid,
                     info);
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_sparse_gram),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 112 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  const unsigned blocks = (unsigned)((s + 1) / 2);
  hipLaunchKernelGGL(k_sparse_gram, dim3(blocks), dim3(256),
                     (size_t)s * sizeof(unsigned long long), st, s, rp, ci, rid, v, vdt, S, lds,
                     info, which);
}

template <typename T>
void scatter(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
             const void *v, int vdt, const double *M, T *base, const SvDevInfo *info) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)s;
#define SV_SC(KK) hipLaunchKernelGGL((k_scatter<T, KK>), dim3(blocks), dim3(64 * SP_NW), 0, st, \
                                     s, rp, ci, v, vdt, M, base, info)
  switch (K) {
    case 16: SV_SC(16); break;
    case 32: SV_SC(32); break;
    case 64: SV_SC(64); break;
    case 128: SV_SC(128); break;
  }
#undef SV_SC
}
template void scatter<float>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                             const void *, int, const double *, float *, const SvDevInfo *);
template void scatter<double>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                              const void *, int, const double *, double *, const SvDevInfo *);

template <typename T>
void append_rows(hipStream_t st, int K, int64_t s, const double *src, int64_t rs, int64_t cs,
                 const double *Winv, const int32_t *reset_flag, T *out,
                 const SvDevInfo *info) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)((s + 3) / 4);
#define SV_AP(KK) hipLaunchKernelGGL((k_append<T, KK>), dim3(blocks), dim3(256), 0, st, \
                                     s, src, rs, cs, Winv, reset_flag, out, info)
  switch (K) {
    case 16: SV_AP(16); break;
    case 32: SV_AP(32); break;
    case 64: SV_AP(64); break;
    case 128: SV_AP(128); break;
  }
#undef SV_AP
}
template void append_rows<float>(hipStream_t, int, int64_t, const double *, int64_t, int64_t,
                                 const double *, const int32_t *, float *, const SvDevInfo *);
template void append_rows<double>(hipStream_t, int, int64_t, const double *, int64_t, int64_t,
                                  const double *, const int32_t *, double *, const SvDevInfo *);

void csr_dense(hipStream_t st, int L, int64_t rows, const int64_t *rp, const int32_t *ci,
               const void *v, int vdt, const double *X, double *Y, const SvDevInfo *info) {
  if (rows <= 0) return;
  const int64_t nb = (rows + 3) / 4;
  const unsigned grid = (unsigned)(nb < (1 << 30) ? nb : (1 << 30));
#define SV_CD(LL) hipLaunchKernelGGL((k_csr_dense<LL, 8>), dim3(grid), dim3(256), 0, st, rows, rp, \
                                     ci, v, vdt, X, Y, info)
  switch (L) {
    case 16: SV_CD(16); break;
    case 32: SV_CD(32); break;
    case 64: SV_CD(64); break;
    case 128: SV_CD(128); break;
  }
#undef SV_CD
}

}  // namespace svl
