// Sparse kernels of one update: input validation, the projection of the
// update onto the tall factor (SpMM with the k x k factor as epilogue), the
// sparse Gram E E^T, and the two writes into the tall factors (the sparse row
// update and the appended rows).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

__device__ __forceinline__ void fail(SvDevInfo *info, int code, int seq) {
  if (atomicCAS(&info->status, 0, code) == 0) info->failed_seq = seq;
}

// Canonical-CSR check (0-based, monotone row_ptr, strictly increasing
// in-range column ids per row, finite values).  Every access is bounded by
// the declared nnz, so a malformed row_ptr cannot push reads out of range.
__global__ void k_validate_csr(int64_t rows, int64_t cols, int64_t nnz,
                               const int64_t *__restrict__ row_ptr,
                               const int32_t *__restrict__ col_idx,
                               const void *__restrict__ val, int vdtype,
                               SvDevInfo *info, int seq) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    if (row_ptr[0] != 0 || row_ptr[rows] != nnz) fail(info, 1, seq);
  }
  for (int64_t i = tid; i < rows; i += stride) {
    const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
    if (p0 < 0 || p1 < p0 || p1 > nnz) { fail(info, 1, seq); continue; }
    int32_t prev = -1;
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t c = col_idx[p];
      if (c <= prev || c >= cols) { fail(info, 1, seq); break; }
      prev = c;
      const double v = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
      if (!isfinite(v)) { fail(info, 4, seq); break; }
    }
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

// Row i of P = E * base (K columns, accumulated in T), C'[i] = P[i] W (FP64,
// W is K x K FP64) and ||e_i||^2, by one block of SP_NW waves.  For K <= 64 a
// wave splits into 64/K groups of K lanes that take alternate nonzeros of a
// chunk; for K = 128 each lane owns two columns.  red (SP_NW x K), ptot (K)
// and nred (SP_NW) are LDS scratch of the caller.
template <typename T, int K>
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
  T acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = (T)0;
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
    const T mv = (T)mvd;
    // lanes >= n carry column 0 and value 0: their gathers are valid and add 0
    for (int j0 = 0; j0 < n; j0 += SP_U * G) {
      int32_t cc[SP_U];
      T vv[SP_U];
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
        for (int q = 0; q < CPL; ++q) acc[q] += vv[u] * bb[u][q];
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
template <typename T, int K>
__global__ void __launch_bounds__(64 * SP_NW)
k_spmm_w(int64_t s, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
         const void *__restrict__ val, int vdtype, const T *__restrict__ base,
         const double *__restrict__ W, double *__restrict__ Cp64, float *__restrict__ Cp32,
         double *__restrict__ rownorm2, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ double red[SP_NW * K];
  __shared__ double ptot[K];
  __shared__ double nred[SP_NW];
  spmm_row<T, K>((int64_t)blockIdx.x, row_ptr, col_idx, val, vdtype, base, W, Cp64, Cp32,
                 rownorm2, red, ptot, nred);
}

constexpr int PB_U = 16;   // gathers in flight per lane in the fused projection

// Row i of P = E * base accumulated by one wave (T accumulate); lanes c < K
// (and c + 64 for K = 128) end with P[i][c] in out[c] (LDS); *nrm receives
// ||e_i||^2 (lane 0).  Same gather scheme as spmm_row.
template <typename T, int K>
__device__ __forceinline__ void
wave_row_project(int64_t i, const int64_t *__restrict__ row_ptr,
                 const int32_t *__restrict__ col_idx, const void *__restrict__ val, int vdtype,
                 const T *__restrict__ base, double *out, double *nrm_out) {
  constexpr int G = K <= 64 ? 64 / K : 1;
  constexpr int CPL = K <= 64 ? 1 : K / 64;
  const int lane = threadIdx.x & 63;
  const int g = lane / (64 / G), c = lane % (64 / G);
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  T acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = (T)0;
  double nrm = 0.0;
  for (int64_t cb = p0; cb < p1; cb += 64) {
    const int n = (int)((p1 - cb) < 64 ? (p1 - cb) : 64);
    int32_t mc = 0;
    double mvd = 0.0;
    if (lane < n) {
      mc = col_idx[cb + lane];
      mvd = ldv(val, vdtype, cb + lane);
    }
    nrm += mvd * mvd;
    const T mv = (T)mvd;
    for (int j0 = 0; j0 < n; j0 += PB_U * G) {
      int32_t cc[PB_U];
      T vv[PB_U];
#pragma unroll
      for (int u = 0; u < PB_U; ++u) {
        const int jj = j0 + u * G + g;
        cc[u] = __shfl(mc, jj, 64);
        vv[u] = __shfl(mv, jj, 64);
      }
      T bb[PB_U][CPL];
#pragma unroll
      for (int u = 0; u < PB_U; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) bb[u][q] = base[(int64_t)cc[u] * K + c + 64 * q];
#pragma unroll
      for (int u = 0; u < PB_U; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] += vv[u] * bb[u][q];
    }
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int o = K; o < 64; o <<= 1) acc[0] += __shfl_xor(acc[0], o, 64);
  }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) out[c + 64 * q] = (double)acc[q];
  }
  nrm = wave_sum(nrm);
  if (lane == 0) *nrm_out = nrm;
}

// The projections of many updates of one rank and storage type in one
// launch (a batch of mixed ranks and types is one launch per group, so each
// launch keeps the registers of its own shape and its occupancy).  Block b
// takes a tile of PB_RB consecutive rows of request r, with row0 the prefix
// sums of the group's tile counts: each
// wave accumulates whole rows of P (one row at a time, 16 gathers in flight
// per lane), the tile's rows of P meet in LDS, and C' = P W is formed for the
// tile (W from L2; small LDS keeps many blocks resident per CU).
constexpr int PB_RB = 8;

template <typename T, int K>
__global__ void __launch_bounds__(64 * SP_NW)
k_spmm_batch(int n, const svl::ProjDesc *__restrict__ descs) {
  __shared__ double Pt[PB_RB][K];
  __shared__ double nr[PB_RB];
  const int64_t b = blockIdx.x;
  int lo = 0, hi = n - 1;   // last request with row0 <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].row0 <= b) lo = mid; else hi = mid - 1;
  }
  const svl::ProjDesc &d = descs[lo];
  if (d.info && d.info->status) return;
  const int64_t i0 = (b - d.row0) * PB_RB;
  const int rows = (int)((d.s - i0) < PB_RB ? (d.s - i0) : PB_RB);
  if (rows <= 0) return;
  const int tid = threadIdx.x, w = tid >> 6;
  for (int rr = w; rr < rows; rr += SP_NW)
    wave_row_project<T, K>(i0 + rr, d.row_ptr, d.col_idx, d.val, d.vdtype, (const T *)d.base,
                           Pt[rr], &nr[rr]);
  __syncthreads();
  for (int e = tid; e < rows * K; e += 64 * SP_NW) {
    const int rr = e / K, col = e % K;
    double o = 0.0;
#pragma unroll 8
    for (int l = 0; l < K; ++l) o += Pt[rr][l] * d.W[l * K + col];
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

constexpr int GRAM_LDS_CAP = 4096;      // nonzeros of the pivot row kept in LDS
constexpr int GRAM_ACC_CAP = 8192;      // rows j accumulated in LDS (dynamic)

// S = E E^T (FP64, full s x s).  Block b handles rows i = b and s-1-b (folded
// so that every block does about s/2 row pairs).  Row i is staged in LDS; the
// nonzeros of rows 0..i are contiguous in the CSR, so the block streams them
// with coalesced loads (one nonzero per thread), finds each column in row i
// by binary search, and accumulates the products per row j in LDS.
__global__ void __launch_bounds__(256)
k_sparse_gram(int64_t s, const int64_t *__restrict__ row_ptr,
              const int32_t *__restrict__ col_idx, const int32_t *__restrict__ rid,
              const void *__restrict__ val, int vdtype, double *__restrict__ S,
              int64_t lds, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ int32_t sc[GRAM_LDS_CAP];
  __shared__ double sv[GRAM_LDS_CAP];
  extern __shared__ double acc[];   // s doubles
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
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x) acc[j] = 0.0;
    __syncthreads();
    const int32_t *ci = in_lds ? sc : col_idx + q0;
    if (ni > 0) {
      for (int64_t p = threadIdx.x; p < q1; p += blockDim.x) {
        const int32_t c = col_idx[p];
        int64_t lo = 0, hi = ni;   // first position with ci[pos] >= c
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (ci[mid] < c) lo = mid + 1; else hi = mid;
        }
        if (lo < ni && ci[lo] == c) {
          const double vi = in_lds ? sv[lo] : ldv(val, vdtype, q0 + lo);
          atomicAdd(&acc[rid[p]], vi * ldv(val, vdtype, p));
        }
      }
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x) {
      const double a = acc[j];
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

}  // namespace

// ---------------------------------------------------------------- launchers
namespace svl {

void validate_csr(hipStream_t st, int64_t rows, int64_t cols, int64_t nnz,
                  const int64_t *rp, const int32_t *ci, const void *v, int vdt,
                  SvDevInfo *info, int seq) {
  int64_t blocks = (rows + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)blocks), dim3(256), 0, st,
                     rows, cols, nnz, rp, ci, v, vdt, info, seq);
}

template <typename T>
void spmm_w(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
            const void *v, int vdt, const T *base, const double *W, double *Cp64,
            float *Cp32, double *rownorm2, const SvDevInfo *info) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)s;
#define SV_SPMM(KK) hipLaunchKernelGGL((k_spmm_w<T, KK>), dim3(blocks), dim3(64 * SP_NW), 0, st, \
                                       s, rp, ci, v, vdt, base, W, Cp64, Cp32, rownorm2, info)
  switch (K) {
    case 16: SV_SPMM(16); break;
    case 32: SV_SPMM(32); break;
    case 64: SV_SPMM(64); break;
    case 128: SV_SPMM(128); break;
  }
#undef SV_SPMM
}
template void spmm_w<float>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                            const void *, int, const float *, const double *, double *,
                            float *, double *, const SvDevInfo *);
template void spmm_w<double>(hipStream_t, int, int64_t, const int64_t *, const int32_t *,
                             const void *, int, const double *, const double *, double *,
                             float *, double *, const SvDevInfo *);

int spmm_batch_rows_per_block() { return PB_RB; }

void spmm_batch_prepare(std::vector<ProjDesc> &d) {
  std::stable_sort(d.begin(), d.end(), [](const ProjDesc &a, const ProjDesc &b) {
    return a.fp64 != b.fp64 ? a.fp64 < b.fp64 : a.K < b.K;
  });
  int64_t tiles = 0;
  for (size_t q = 0; q < d.size(); ++q) {
    if (q > 0 && (d[q].fp64 != d[q - 1].fp64 || d[q].K != d[q - 1].K)) tiles = 0;
    d[q].row0 = tiles;
    tiles += (d[q].s + PB_RB - 1) / PB_RB;
  }
}

void spmm_batch(hipStream_t st, const std::vector<ProjDesc> &d, const ProjDesc *descs_dev) {
  size_t g0 = 0;
  while (g0 < d.size()) {
    size_t g1 = g0 + 1;
    while (g1 < d.size() && d[g1].fp64 == d[g0].fp64 && d[g1].K == d[g0].K) ++g1;
    const ProjDesc &last = d[g1 - 1];
    const int64_t tiles = last.row0 + (last.s + PB_RB - 1) / PB_RB;
    const int n = (int)(g1 - g0);
    const ProjDesc *dd = descs_dev + g0;
    if (tiles > 0) {
#define SV_PB(TT, KK) hipLaunchKernelGGL((k_spmm_batch<TT, KK>), dim3((unsigned)tiles), \
                                         dim3(64 * SP_NW), 0, st, n, dd)
      if (d[g0].fp64) {
        switch (d[g0].K) {
          case 16: SV_PB(double, 16); break;
          case 32: SV_PB(double, 32); break;
          case 64: SV_PB(double, 64); break;
          default: SV_PB(double, 128); break;
        }
      } else {
        switch (d[g0].K) {
          case 16: SV_PB(float, 16); break;
          case 32: SV_PB(float, 32); break;
          case 64: SV_PB(float, 64); break;
          default: SV_PB(float, 128); break;
        }
      }
#undef SV_PB
    }
    g0 = g1;
  }
}

int gram_max_rows() { return GRAM_ACC_CAP; }

void sparse_gram(hipStream_t st, int64_t s, const int64_t *rp, const int32_t *ci,
                 const void *v, int vdt, int32_t *rid, double *S, int64_t lds,
                 const SvDevInfo *info) {
  if (s <= 0) return;
  hipLaunchKernelGGL(k_row_ids, dim3((unsigned)((s + 3) / 4)), dim3(256), 0, st, s, rp, rid,
                     info);
  static bool once = false;
  if (!once) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_sparse_gram),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 112 * 1024);
    (void)hipGetLastError();
    once = true;
  }
  const unsigned blocks = (unsigned)((s + 1) / 2);
  hipLaunchKernelGGL(k_sparse_gram, dim3(blocks), dim3(256), (size_t)s * sizeof(double), st, s,
                     rp, ci, rid, v, vdt, S, lds, info);
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

}  // namespace svl
