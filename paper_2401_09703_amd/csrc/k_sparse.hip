// Sparse kernels of one update: input validation, the projection of the
// update onto the tall factor (SpMM with the k x k factor as epilogue), the
// sparse Gram E E^T, and the two writes into the tall factors (the sparse row
// update and the appended rows).
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

// P = E * base (s x K, accumulated in T), C' = P * W (FP64, W is K x K FP64),
// plus ||e_i||^2.  One wavefront per row of E.  For K <= 64 the wave splits
// into 64/K groups of K lanes that take every (64/K)-th nonzero; for K = 128
// each lane owns two columns.
template <typename T, int K>
__global__ void k_spmm_w(int64_t s, const int64_t *__restrict__ row_ptr,
                         const int32_t *__restrict__ col_idx,
                         const void *__restrict__ val, int vdtype,
                         const T *__restrict__ base,
                         const double *__restrict__ W,
                         double *__restrict__ Cp64, float *__restrict__ Cp32,
                         double *__restrict__ rownorm2,
                         const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= s) return;
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  double nrm = 0.0;
  for (int64_t p = p0 + lane; p < p1; p += 64) {
    const double v = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
    nrm += v * v;
  }
  nrm = wave_sum(nrm);
  if constexpr (K <= 64) {
    constexpr int G = 64 / K;
    const int g = lane / K, c = lane % K;
    T acc = 0;
    for (int64_t p = p0 + g; p < p1; p += G) {
      const int32_t col = col_idx[p];
      const T v = (T)(vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p]);
      acc += v * base[(int64_t)col * K + c];
    }
#pragma unroll
    for (int o = K; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    // epilogue: lanes 0..K-1 compute column c of C' = P W
    double out = 0.0;
#pragma unroll 8
    for (int l = 0; l < K; ++l) {
      const double pl = (double)__shfl(acc, l, 64);
      out += pl * W[l * K + c];
    }
    if (lane < K) {
      Cp64[i * K + c] = out;
      if (Cp32) Cp32[i * K + c] = (float)out;
    }
  } else {
    T a0 = 0, a1 = 0;
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t col = col_idx[p];
      const T v = (T)(vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p]);
      a0 += v * base[(int64_t)col * K + lane];
      a1 += v * base[(int64_t)col * K + 64 + lane];
    }
    double o0 = 0.0, o1 = 0.0;
#pragma unroll 8
    for (int l = 0; l < 64; ++l) {
      const double pl = (double)__shfl(a0, l, 64);
      o0 += pl * W[l * K + lane];
      o1 += pl * W[l * K + 64 + lane];
    }
#pragma unroll 8
    for (int l = 0; l < 64; ++l) {
      const double pl = (double)__shfl(a1, l, 64);
      o0 += pl * W[(64 + l) * K + lane];
      o1 += pl * W[(64 + l) * K + 64 + lane];
    }
    Cp64[i * K + lane] = o0;
    Cp64[i * K + 64 + lane] = o1;
    if (Cp32) {
      Cp32[i * K + lane] = (float)o0;
      Cp32[i * K + 64 + lane] = (float)o1;
    }
  }
  if (lane == 0) rownorm2[i] = nrm;
}

constexpr int GRAM_LDS_CAP = 4096;

// S = E E^T (FP64, full s x s).  Block b handles rows i = b and s-1-b (folded
// so that every block does about s/2 row pairs).  Row i is staged in LDS and
// every row j <= i is intersected with it by binary search; one wave per j.
__global__ void __launch_bounds__(256)
k_sparse_gram(int64_t s, const int64_t *__restrict__ row_ptr,
              const int32_t *__restrict__ col_idx,
              const void *__restrict__ val, int vdtype, double *__restrict__ S,
              int64_t lds, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  __shared__ int32_t sc[GRAM_LDS_CAP];
  __shared__ double sv[GRAM_LDS_CAP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
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
        sv[t] = vdtype ? ((const double *)val)[q0 + t] : (double)((const float *)val)[q0 + t];
      }
    }
    __syncthreads();
    const int32_t *ci = in_lds ? sc : col_idx + q0;
    for (int64_t j = w; j <= i; j += nw) {
      const int64_t p0 = row_ptr[j], p1 = row_ptr[j + 1];
      double acc = 0.0;
      if (ni > 0) {
        for (int64_t p = p0 + lane; p < p1; p += 64) {
          const int32_t c = col_idx[p];
          int64_t lo = 0, hi = ni;   // first position with ci[pos] >= c
          while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ci[mid] < c) lo = mid + 1; else hi = mid;
          }
          if (lo < ni && ci[lo] == c) {
            const double vi = in_lds ? sv[lo]
                                     : (vdtype ? ((const double *)val)[q0 + lo]
                                               : (double)((const float *)val)[q0 + lo]);
            const double vj = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
            acc += vi * vj;
          }
        }
      }
      acc = wave_sum(acc);
      if (lane == 0) {
        S[i * lds + j] = acc;
        S[j * lds + i] = acc;
      }
    }
  }
}

// base[col] += sum_i E[i, col] * M[i]  (the sparse row update of the tall
// factor, Equation (1) second term).  One wave per row of E; FP atomics.
template <typename T, int K>
__global__ void k_scatter(int64_t s, const int64_t *__restrict__ row_ptr,
                          const int32_t *__restrict__ col_idx,
                          const void *__restrict__ val, int vdtype,
                          const double *__restrict__ M, T *__restrict__ base,
                          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= s) return;
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  if constexpr (K <= 64) {
    constexpr int G = 64 / K;
    const int g = lane / K, c = lane % K;
    const double mc = M[i * K + c];
    for (int64_t p = p0 + g; p < p1; p += G) {
      const double v = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
      atomicAdd(&base[(int64_t)col_idx[p] * K + c], (T)(v * mc));
    }
  } else {
    const double m0 = M[i * K + lane], m1 = M[i * K + 64 + lane];
    for (int64_t p = p0; p < p1; ++p) {
      const double v = vdtype ? ((const double *)val)[p] : (double)((const float *)val)[p];
      T *dst = base + (int64_t)col_idx[p] * K;
      atomicAdd(dst + lane, (T)(v * m0));
      atomicAdd(dst + 64 + lane, (T)(v * m1));
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
  const unsigned blocks = (unsigned)((s + 3) / 4);
#define SV_SPMM(KK) hipLaunchKernelGGL((k_spmm_w<T, KK>), dim3(blocks), dim3(256), 0, st, \
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

void sparse_gram(hipStream_t st, int64_t s, const int64_t *rp, const int32_t *ci,
                 const void *v, int vdt, double *S, int64_t lds, const SvDevInfo *info) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)((s + 1) / 2);
  hipLaunchKernelGGL(k_sparse_gram, dim3(blocks), dim3(256), 0, st, s, rp, ci, v, vdt, S,
                     lds, info);
}

template <typename T>
void scatter(hipStream_t st, int K, int64_t s, const int64_t *rp, const int32_t *ci,
             const void *v, int vdt, const double *M, T *base, const SvDevInfo *info) {
  if (s <= 0) return;
  const unsigned blocks = (unsigned)((s + 3) / 4);
#define SV_SC(KK) hipLaunchKernelGGL((k_scatter<T, KK>), dim3(blocks), dim3(256), 0, st, \
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
