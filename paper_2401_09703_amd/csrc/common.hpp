// Shared device helpers for the gfx950 kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SV_WAVE 64

namespace svk {

// Cross-lane moves of a double through DPP (the two 32-bit halves moved
// separately); CTRL is the DPP control word.  A DPP move costs a few cycles,
// a shuffle through ds_bpermute an LDS round trip.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_dbl(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Sum over each group of four consecutive lanes, in every lane of the group.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_d<DPP_QUAD_XOR1>(v);
  v += dpp_d<DPP_QUAD_XOR2>(v);
  return v;
}

// Wave-wide sum in every lane: DPP within each row of 16 lanes, then the four
// row sums read from lanes 0, 16, 32, 48 (fixed order, so every lane and
// every call with the same inputs gets the same bits).  All 64 lanes must be
// active (every caller reduces in converged code).
__device__ __forceinline__ double wave_sum(double v) {
  v = quad_sum(v);
  v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
  v += dpp_d<DPP_ROW_MIRROR>(v);
  return (readlane_dbl(v, 0) + readlane_dbl(v, 16)) + (readlane_dbl(v, 32) + readlane_dbl(v, 48));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave-wide maximum in every lane (DPP as for wave_sum; all lanes active).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<DPP_QUAD_XOR1>(v));
  v = fmax(v, dpp_d<DPP_QUAD_XOR2>(v));
  v = fmax(v, dpp_d<DPP_ROW_HALF_MIRROR>(v));
  v = fmax(v, dpp_d<DPP_ROW_MIRROR>(v));
  return fmax(fmax(readlane_dbl(v, 0), readlane_dbl(v, 16)),
              fmax(readlane_dbl(v, 32), readlane_dbl(v, 48)));
}

// Block-wide sum; every thread returns the same value (fixed summation order,
// so identical inputs give bitwise identical results in every block).
// red must hold blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

__device__ __forceinline__ double block_max(double v, double *red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < nw; ++i) t = fmax(t, red[i]);
  return t;
}

template <typename T>
__device__ __forceinline__ double load_val(const void *p, int64_t i);
template <>
__device__ __forceinline__ double load_val<float>(const void *p, int64_t i) {
  return (double)((const float *)p)[i];
}
template <>
__device__ __forceinline__ double load_val<double>(const void *p, int64_t i) {
  return ((const double *)p)[i];
}

// Deterministic pseudo-random double in [-1, 1) from a 64-bit key
// (SplitMix64 finaliser).
__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Synchronise the lanes of one wave through LDS (no block barrier): orders
// this wave's LDS accesses before and after the call.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-level variant of tri_lower_inv_inplace (only the calling wave takes
// part; lane = threadIdx.x & 63).
__device__ inline void tri_lower_inv_wave(double *L, int ld, int n, double *tmp) {
  const int lane = threadIdx.x & 63;
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = 1.0 / L[j * ld + j];
    for (int i = j + 1 + lane; i < n; i += 64) {
      double y = 0.0;
      for (int p = j + 1; p <= i; ++p) y += L[i * ld + p] * L[p * ld + j];
      tmp[i] = -ljj * y;
    }
    wave_sync();
    for (int i = j + 1 + lane; i < n; i += 64) L[i * ld + j] = tmp[i];
    if (lane == 0) L[j * ld + j] = ljj;
    wave_sync();
  }
}

// Coherent (L2-bypassing) accesses for data that blocks of one cooperative
// launch exchange: agent-scope relaxed atomics are served at the device
// coherence point, so neither side needs an L2-wide writeback or invalidate.
__device__ __forceinline__ void st_coh(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int FLAG_STRIDE = 16;   // one flag per 64-byte line

// All-to-all arrival barrier of a cooperative launch: every block publishes
// the epoch once its coherent stores have completed, then waits until every
// block has published it.  Flags grow monotonically across launches (epochs
// are never reused), so no reset is needed between barriers.
__device__ __forceinline__ void flag_barrier(unsigned *flags, unsigned epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&flags[blockIdx.x * FLAG_STRIDE], epoch, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned t = threadIdx.x; t < gridDim.x; t += blockDim.x)
    while (__hip_atomic_load(&flags[t * FLAG_STRIDE], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) < epoch)
      __builtin_amdgcn_s_sleep(1);
  __syncthreads();
}

// In-place inverse of the n x n lower-triangular matrix in LDS (row stride
// ld), column by column from the last one: column j of the inverse is
// -inv(L_jj) * inv(L22) * L[j+1:, j] with the trailing block already
// inverted.  tmp holds n doubles.  All threads of the block take part.
__device__ inline void tri_lower_inv_inplace(double *L, int ld, int n, double *tmp) {
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = 1.0 / L[j * ld + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
      double y = 0.0;
      for (int p = j + 1; p <= i; ++p) y += L[i * ld + p] * L[p * ld + j];
      tmp[i] = -ljj * y;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) L[i * ld + j] = tmp[i];
    if (threadIdx.x == 0) L[j * ld + j] = ljj;
    __syncthreads();
  }
}

}  // namespace svk

// Device status word layout (one per state).
struct SvDevInfo {
  int32_t status;       // 0 ok; else the svlcov_status of the first failure
  int32_t failed_seq;   // sequence number of the update that failed
  int32_t rank;         // kept pivots, first orthogonalisation of last update
  int32_t rank2;        // second orthogonalisation (weights) or -1
  int32_t reset_U;      // set by the condition check of the last update
  int32_t reset_V;
  int32_t pad0, pad1;
  double kappa_U, kappa_V;
  double min_kept, max_dropped;   // relative pivots of the last Cholesky
  double scale;                   // max_i ||e_i||^2 of the last Gram
  double scale2;
  int64_t resets_U, resets_V;
  int64_t updates;
};
