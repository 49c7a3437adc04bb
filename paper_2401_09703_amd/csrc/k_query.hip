// Queries and scores on the maintained factors: Query(i) of Theorem 1 for
// many rows (row i of U_base times W, O(k^2) each), and the pair score
// U[i]^T Sigma V[j] of the link-prediction and collaborative-filtering
// workloads, taken on realised factors U_base (W_U Sigma) and V_base W_V so
// that each pair is two row gathers and a k-term dot product.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

// out[r] = base[idx[r]] W (FP64 out), one wave per row, W in LDS; rows with
// an index outside [0, rows) receive NaN.
template <typename T, int K>
__global__ void __launch_bounds__(256)
k_query_rows(int64_t n, const int64_t *__restrict__ idx, int64_t rows,
             const T *__restrict__ base, const double *__restrict__ W,
             double *__restrict__ out) {
  constexpr bool WLDS = K <= 64;            // W (K x K FP64) staged when it fits
  __shared__ double Ws[WLDS ? K * K : 1];
  __shared__ double xr[4][K];
  if constexpr (WLDS) {
    for (int e = threadIdx.x; e < K * K; e += 256) Ws[e] = W[e];
    __syncthreads();
  }
  const double *Wp = WLDS ? Ws : W;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * 4 + w; r < n; r += (int64_t)gridDim.x * 4) {
    const int64_t i = idx[r];
    const bool ok = i >= 0 && i < rows;
    for (int a = lane; a < K; a += 64) xr[w][a] = ok ? (double)base[i * K + a] : 0.0;
    wave_sync();
    for (int c = lane; c < K; c += 64) {
      double acc = 0.0;
#pragma unroll 8
      for (int a = 0; a < K; ++a) acc += xr[w][a] * Wp[a * K + c];
      out[r * K + c] = ok ? acc : NAN;
    }
    wave_sync();
  }
}

// WS = W diag(sig) (K x K).
__global__ void k_scale_cols(int K, const double *__restrict__ W, const double *__restrict__ sig,
                             double *__restrict__ WS) {
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) WS[e] = W[e] * sig[e % K];
}

typedef float sq_f4 __attribute__((ext_vector_type(4)));
typedef double sq_d2 __attribute__((ext_vector_type(2)));
template <typename T> struct QWide;
template <> struct QWide<float> { typedef sq_f4 V; static constexpr int E = 4; };
template <> struct QWide<double> { typedef sq_d2 V; static constexpr int E = 2; };

// score[p] = Ut[i_p] . Vt[j_p] (and the max with Ut[j_p] . Vt[i_p] when both):
// a row of K elements is LPR lanes with one 16-byte load each, so a wave
// scores 64 / LPR pairs at a time, QU of them per lane group in flight.
constexpr int QU = 4;

template <typename T, int K, bool BOTH>
__global__ void __launch_bounds__(256)
k_score_pairs(int64_t n, const int64_t *__restrict__ I, const int64_t *__restrict__ J,
              int64_t m, int64_t nn, const T *__restrict__ Ut, const T *__restrict__ Vt,
              double *__restrict__ out) {
  typedef typename QWide<T>::V V;
  constexpr int E = QWide<T>::E;
  constexpr int LPR = K / E;          // lanes per row
  constexpr int G = 64 / LPR;         // pairs per wave and step
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / LPR, c = (lane % LPR) * E;
  const int64_t per_step = (int64_t)G * QU;
  const int64_t wave_id = (int64_t)blockIdx.x * 4 + w, waves = (int64_t)gridDim.x * 4;
  for (int64_t p0 = wave_id * per_step; p0 < n; p0 += waves * per_step) {
    int64_t pi[QU], pj[QU];
    bool ok[QU];
    V a[QU], b[QU], a2[QU], b2[QU];
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      const int64_t p = p0 + (int64_t)u * G + g;
      const bool in = p < n;
      const int64_t i = in ? I[p] : 0, j = in ? J[p] : 0;
      ok[u] = in && i >= 0 && j >= 0 && i < m && j < nn &&
              (!BOTH || (j < m && i < nn));
      pi[u] = ok[u] ? i : 0;
      pj[u] = ok[u] ? j : 0;
    }
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      a[u] = *(const V *)(Ut + pi[u] * K + c);
      b[u] = *(const V *)(Vt + pj[u] * K + c);
      if constexpr (BOTH) {
        a2[u] = *(const V *)(Ut + pj[u] * K + c);
        b2[u] = *(const V *)(Vt + pi[u] * K + c);
      }
    }
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        s1 += (double)a[u][e] * (double)b[u][e];
        if constexpr (BOTH) s2 += (double)a2[u][e] * (double)b2[u][e];
      }
#pragma unroll
      for (int o = 1; o < LPR; o <<= 1) {
        s1 += __shfl_xor(s1, o, 64);
        if constexpr (BOTH) s2 += __shfl_xor(s2, o, 64);
      }
      const int64_t p = p0 + (int64_t)u * G + g;
      if (lane % LPR == 0 && p < n) out[p] = ok[u] ? (BOTH ? fmax(s1, s2) : s1) : NAN;
    }
  }
}

}  // namespace

namespace svl {

template <typename T>
void query_rows(hipStream_t st, int K, int64_t n, const int64_t *idx, int64_t rows,
                const T *base, const double *W, double *out) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 3) / 4, 4096);
#define SV_Q(KK) hipLaunchKernelGGL((k_query_rows<T, KK>), dim3(grid), dim3(256), 0, st, n, idx, \
                                    rows, base, W, out)
  switch (K) {
    case 16: SV_Q(16); break;
    case 32: SV_Q(32); break;
    case 64: SV_Q(64); break;
    default: SV_Q(128); break;
  }
#undef SV_Q
}
template void query_rows<float>(hipStream_t, int, int64_t, const int64_t *, int64_t,
                                const float *, const double *, double *);
template void query_rows<double>(hipStream_t, int, int64_t, const int64_t *, int64_t,
                                 const double *, const double *, double *);

void scale_cols(hipStream_t st, int K, const double *W, const double *sig, double *WS) {
  hipLaunchKernelGGL(k_scale_cols, dim3(1), dim3(256), 0, st, K, W, sig, WS);
}

template <typename T>
void score_pairs(hipStream_t st, int K, int64_t n, const int64_t *I, const int64_t *J, int both,
                 int64_t m, int64_t nn, const T *Ut, const T *Vt, double *out) {
  if (n <= 0) return;
  constexpr int E = sizeof(T) == 4 ? 4 : 2;
  const int64_t per_block = (int64_t)4 * (64 / (K / E)) * QU;
  const unsigned grid = (unsigned)std::min<int64_t>((n + per_block - 1) / per_block, 8192);
#define SV_S(KK, BB) hipLaunchKernelGGL((k_score_pairs<T, KK, BB>), dim3(grid), dim3(256), 0, st, \
                                        n, I, J, m, nn, Ut, Vt, out)
  switch (K) {
    case 16: if (both) SV_S(16, true); else SV_S(16, false); break;
    case 32: if (both) SV_S(32, true); else SV_S(32, false); break;
    case 64: if (both) SV_S(64, true); else SV_S(64, false); break;
    default: if (both) SV_S(128, true); else SV_S(128, false); break;
  }
#undef SV_S
}
template void score_pairs<float>(hipStream_t, int, int64_t, const int64_t *, const int64_t *, int,
                                 int64_t, int64_t, const float *, const float *, double *);
template void score_pairs<double>(hipStream_t, int, int64_t, const int64_t *, const int64_t *,
                                  int, int64_t, int64_t, const double *, const double *,
                                  double *);

}  // namespace svl
