// Dense kernels of one update: FP64 GEMM on MFMA, the residual Gram on MFMA (FP32 and
// BF16x3), the FP64 Cholesky with pivot dropping and its triangular solve,
// assembly of K, the k x k inverse with a condition estimate, row
// orthonormalisation and the tall-skinny realisation GEMM.
#include "common.hpp"
#include "kernels.hpp"
#include "k_rsvd.hpp"

#include <type_traits>

using namespace svk;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

namespace {

// ------------------------------------------------------------------ FP64 GEMM
// Tile 64 x BN (BN 64, or 32 for widths 64 q + 32 such as the 96- and
// 160-column panels, where 64-wide tiles would spend a quarter or a sixth of
// the products on zero columns), stages of 64 along K.  A stage of both
// operands is loaded into registers in one go (every load of the stage in
// flight at once), stored to LDS k-major, and the next stage's loads are
// issued before this stage's products, so that a block waits for memory
// about once per stage rather than once per MFMA step.  On gfx950 an FP64
// MFMA 16x16x4 occupies its SIMD for 64 cycles (128 flops per clock per CU),
// so a product is spread over enough blocks to keep every CU's four SIMDs
// busy: the operands here are small (N x p panels, N ~ 10^3) and each
// product is only a few stages deep.
constexpr int GB_M = 64, GB_K = 64, GB_LDA = GB_K + 1;
typedef double gm_d4 __attribute__((ext_vector_type(4)));

template <int BN>
constexpr size_t gemm_lds_bytes() {
  return ((size_t)GB_K * GB_LDA + (size_t)GB_K * (BN + 1)) * sizeof(double);
}

// With part != nullptr the launch is split over K: block z sums the products
// of k in [z*kchunk, (z+1)*kchunk) and writes alpha times its partial sum to
// part[z][M][N] (beta is ignored; k_gemm_reduce finishes).
template <bool TA, bool TB, int BN>
__global__ void __launch_bounds__(256)
k_gemm_f64(int64_t M, int64_t N, int64_t Kfull, double alpha, const double *__restrict__ A,
           int64_t lda, const double *__restrict__ B, int64_t ldb, double beta,
           double *__restrict__ C, int64_t ldc, int64_t kchunk, double *__restrict__ part,
           const SvDevInfo *__restrict__ info) {
  static_assert(BN == 32 || BN == 64, "tile width");
  constexpr int LDB = BN + 1;
  constexpr int TM = BN == 64 ? 2 : 1;   // 16-row MFMA tiles per wave
  constexpr int NA = GB_M * GB_K / 256, NB = BN * GB_K / 256;   // loads per thread
  if (info && info->status) return;
  int64_t K = Kfull;
  if (part) {
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = kb + kchunk < Kfull ? kb + kchunk : Kfull;
    K = ke > kb ? ke - kb : 0;
    A += TA ? kb * lda : kb;
    B += TB ? kb : kb * ldb;
  }
  extern __shared__ double gsm[];
  double *As = gsm, *Bs = gsm + GB_K * GB_LDA;   // [k][row], [k][col]
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // the wave's block of the tile: a 32 x 32 quadrant (BN 64) or a 16 x 32
  // strip (BN 32)
  const int wm = BN == 64 ? (w >> 1) * 32 : 16 * w, wn = BN == 64 ? (w & 1) * 32 : 0;
  const int64_t m0 = (int64_t)blockIdx.y * GB_M, n0 = (int64_t)blockIdx.x * BN;
  // element e = tid + 256 t of a stage: consecutive threads take consecutive
  // addresses of the operand in memory (a row of A, a column of A^T, ...)
  auto a_ip = [&](int t, int &i, int &p) {
    const int e = tid + 256 * t;
    if (TA) { i = e & 63; p = e >> 6; } else { p = e & 63; i = e >> 6; }
  };
  auto b_jq = [&](int t, int &j, int &q) {
    const int e = tid + 256 * t;
    if (TB) { q = e & 63; j = e >> 6; } else { j = e % BN; q = e / BN; }
  };
  double ra[NA], rb[NB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      int i, p;
      a_ip(t, i, p);
      const int64_t gi = m0 + i, gp = k0 + p;
      ra[t] = (gi < M && gp < K) ? (TA ? A[gp * lda + gi] : A[gi * lda + gp]) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      int j, q;
      b_jq(t, j, q);
      const int64_t gj = n0 + j, gq = k0 + q;
      rb[t] = (gj < N && gq < K) ? (TB ? B[gj * ldb + gq] : B[gq * ldb + gj]) : 0.0;
    }
  };
  gm_d4 acc[TM][2];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = gm_d4{0.0, 0.0, 0.0, 0.0};
  if (K > 0) load(0);
  for (int64_t k0 = 0; k0 < K; k0 += GB_K) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      int i, p;
      a_ip(t, i, p);
      As[p * GB_LDA + i] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      int j, q;
      b_jq(t, j, q);
      Bs[q * LDB + j] = rb[t];
    }
    __syncthreads();
    if (k0 + GB_K < K) load(k0 + GB_K);
    // v_mfma_f64_16x16x4: A[m][k] from lane (m, k) = (l % 16, l / 16), B[k][n]
    // from lane (k, n) = (l / 16, l % 16).  A short last stage is zero
    // beyond K and runs whole: a branch per step would keep the compiler
    // from reading the next step's operands during this step's products.
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      double a[TM], b[2];
#pragma unroll
      for (int t = 0; t < TM; ++t) a[t] = As[(kk + lk) * GB_LDA + wm + 16 * t + li];
#pragma unroll
      for (int u = 0; u < 2; ++u) b[u] = Bs[(kk + lk) * LDB + wn + 16 * u + li];
#pragma unroll
      for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[m][n] of a 16 x 16 tile sits in lane n + 16 (m % 4), element m / 4
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = m0 + wm + 16 * t + lk + 4 * q;
        const int64_t gj = n0 + wn + 16 * u + li;
        if (gi >= M || gj >= N) continue;
        double v = alpha * acc[t][u][q];
        if (part) {
          part[((int64_t)blockIdx.z * M + gi) * N + gj] = v;
          continue;
        }
        if (beta != 0.0) v += beta * C[gi * ldc + gj];
        C[gi * ldc + gj] = v;
      }
}

__global__ void k_gemm_reduce(int64_t M, int64_t N, int splits, const double *__restrict__ part,
                              double beta, double *__restrict__ C, int64_t ldc,
                              const SvDevInfo *__restrict__ info) {
  if (info && info->status) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e % N;
  double v = 0.0;
  for (int z = 0; z < splits; ++z) v += part[(int64_t)z * M * N + e];
  if (beta != 0.0) v += beta * C[i * ldc + j];
  C[i * ldc + j] = v;
}

// ------------------------------------------------- residual Gram on MFMA
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

// Tile 64 x 64 of the lower triangle; 4 waves, each a 32 x 32 quadrant made
// of 2 x 2 MFMA 16 x 16 blocks.  LDS holds the two 64-row panels of C.
template <int MODE>
__global__ void __launch_bounds__(256)
k_gram_lowp(int64_t s, int K, const float *__restrict__ C, double *__restrict__ G,
            int64_t ldg, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  constexpr int KP = 128 + 8;  // padded row length (elements)
  extern __shared__ unsigned char smem[];
  // decode lower-triangular tile pair (ti >= tj)
  const int64_t t = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t r0 = ti * 64, c0 = tj * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (MODE == 1) {
    float *As = (float *)smem;
    float *Bs = As + 64 * KP;
    for (int e = tid; e < 64 * K; e += 256) {
      const int rr = e / K, cc = e % K;
      As[rr * KP + cc] = (r0 + rr < s) ? C[(r0 + rr) * K + cc] : 0.f;
      Bs[rr * KP + cc] = (c0 + rr < s) ? C[(c0 + rr) * K + cc] : 0.f;
    }
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    for (int kk = 0; kk < K; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = As[(wr * 32 + x * 16 + li) * KP + kk + lk];
        b[x] = Bs[(wc * 32 + x * 16 + li) * KP + kk + lk];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  } else {
    unsigned short *Ah = (unsigned short *)smem;
    unsigned short *Al = Ah + 64 * KP;
    unsigned short *Bh = Al + 64 * KP;
    unsigned short *Bl = Bh + 64 * KP;
    for (int e = tid; e < 64 * K; e += 256) {
      const int rr = e / K, cc = e % K;
      const float xa = (r0 + rr < s) ? C[(r0 + rr) * K + cc] : 0.f;
      const float xb = (c0 + rr < s) ? C[(c0 + rr) * K + cc] : 0.f;
      const unsigned short ha = f32_to_bf16_rne(xa), hb = f32_to_bf16_rne(xb);
      Ah[rr * KP + cc] = ha;
      Al[rr * KP + cc] = f32_to_bf16_rne(xa - bf16_to_f32(ha));
      Bh[rr * KP + cc] = hb;
      Bl[rr * KP + cc] = f32_to_bf16_rne(xb - bf16_to_f32(hb));
    }
    __syncthreads();
    const int li = lane & 15, lk = (lane >> 4) * 4;
    for (int kk = 0; kk < K; kk += 16) {
      s16x4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int ra = (wr * 32 + x * 16 + li) * KP + kk + lk;
        const int rb = (wc * 32 + x * 16 + li) * KP + kk + lk;
        ah[x] = *(const s16x4 *)(Ah + ra);
        al[x] = *(const s16x4 *)(Al + ra);
        bh[x] = *(const s16x4 *)(Bh + rb);
        bl[x] = *(const s16x4 *)(Bl + rb);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          f32x4 c = acc[x][y];
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[x], bh[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bl[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bh[y], c, 0, 0, 0);
          acc[x][y] = c;
        }
    }
  }
  // D[i][j] for lane: i = 4*(lane/16) + q, j = lane % 16 within each 16 x 16 block
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = r0 + wr * 32 + x * 16 + 4 * (lane >> 4) + q;
        const int64_t gj = c0 + wc * 32 + y * 16 + (lane & 15);
        if (gi < s && gj < s) G[gi * ldg + gj] -= (double)acc[x][y][q];
      }
}

// ------------------------------------------------------------- small helpers
__global__ void k_copy_strided(int64_t R, int64_t Cn, const double *__restrict__ src,
                               int64_t rs, int64_t cs, double *__restrict__ dst, int64_t ldd,
                               const SvDevInfo *__restrict__ info) {
  if (info && info->status) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= R * Cn) return;
  const int64_t i = e / Cn, j = e % Cn;
  dst[i * ldd + j] = src[i * rs + j * cs];
}

__global__ void k_max_into(int64_t n, const double *__restrict__ v, SvDevInfo *info,
                           int which) {
  __shared__ double red[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  m = block_max(m, red);
  if (threadIdx.x == 0) {
    if (which == 0) info->scale = m; else info->scale2 = m;
  }
}

__global__ void k_build_K_rows(int K, int64_t s, const double *__restrict__ sig,
                               const double *__restrict__ Cp, const double *__restrict__ L,
                               int64_t ldl, double *__restrict__ Ko,
                               const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t N = K + s;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int64_t r = e / N, c = e % N;
  double v = 0.0;
  if (r < K) {
    v = (c == r) ? sig[r] : 0.0;
  } else if (c < K) {
    v = Cp[(r - K) * K + c];
  } else if (c - K <= r - K) {
    v = L[(r - K) * ldl + (c - K)];
  }
  Ko[e] = v;
}

// The leading k rows and columns of M = K K^T for K = [[Sigma, 0], [C', R^T]]:
// M = [[Sigma^2, Sigma C'^T], [C' Sigma, S]], whose block S = E E^T (the
// sparse Gram, since R^T R = S - C' C'^T) is copied in beforehand.  One thread
// per entry of the border (2 k N - k^2 entries).
__global__ void k_build_M_border(int K, int64_t s, const double *__restrict__ sig,
                                 const double *__restrict__ Cp, double *__restrict__ M,
                                 const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t N = K + s;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * N) return;
  const int64_t r = e / N, c = e % N;   // border row r < K, column c
  double v;
  if (c < K) v = (c == r) ? sig[r] * sig[r] : 0.0;
  else v = sig[r] * Cp[(c - K) * K + r];
  M[r * N + c] = v;
  if (c >= K) M[c * N + r] = v;
}

__global__ void k_build_X(int K, int64_t s, const double *__restrict__ Cp,
                          const double *__restrict__ L, int64_t ldl, double *__restrict__ X,
                          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int64_t N = K + s;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * s) return;
  const int64_t r = e / s, c = e % s;
  double v;
  if (r < K) v = Cp[c * K + r];
  else v = (c >= r - K) ? L[c * ldl + (r - K)] : 0.0;   // (L^T)[r-K][c] = L[c][r-K]
  X[e] = v;
}

__global__ void k_add_sigma_diag(int K, const double *__restrict__ sig, double *__restrict__ Ko,
                                 int64_t ld, const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int i = threadIdx.x;
  if (i < K) Ko[(int64_t)i * ld + i] += sig[i];
}

__global__ void k_theta_scale(int K, const double *__restrict__ lam, double *__restrict__ theta,
                              double *__restrict__ Gv, int64_t N, int32_t *__restrict__ complete,
                              const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int j = blockIdx.x;
  const double t0 = sqrt(fmax(lam[0], 0.0));
  const double tj = sqrt(fmax(lam[j], 0.0));
  const bool tiny = !(tj > 1e-12 * t0) || t0 <= 0.0;
  if (threadIdx.x == 0) {
    theta[j] = tj;
    complete[j] = tiny ? 1 : 0;
  }
  const double inv = tiny ? 0.0 : 1.0 / tj;
  for (int64_t c = threadIdx.x; c < N; c += blockDim.x) Gv[(int64_t)j * N + c] *= inv;
}

// Cholesky factor of the K x K Gram Gm (K <= 128) and the inverse of the
// factor, by one block of SMALL_NT threads.  The factorisation is
// right-looking on the unscaled columns (A[i][c] -= A[i][j] A[c][j] / d_j),
// one barrier per column, the trailing lower triangle spread over all
// threads; the columns are scaled at the end.  A non-positive pivot is taken
// as 1 (the rows are then far from orthonormal, which the caller's checks
// catch).  The inverse X = L^{-1} is formed column by column in parallel:
// SMALL_NT / K threads per column share each forward-substitution dot
// product; X is kept transposed in the strict upper triangle of the same
// array, its diagonal apart.
constexpr int SMALL_NT = 256;

__global__ void __launch_bounds__(SMALL_NT)
k_chol_inv_small(int K, const double *__restrict__ Gm, double *__restrict__ Linv,
                 const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double Ls[];   // K x (K+1): L below the diagonal, X^T above
  const int LD = K + 1;
  double *dg = Ls + K * LD;        // K: pivots, then the diagonal of X
  const int tid = threadIdx.x;
  for (int e = tid; e < K * K; e += SMALL_NT) {
    const int i = e / K, j = e % K;
    if (j <= i) Ls[i * LD + j] = Gm[e];
  }
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const double d = Ls[j * LD + j];
    const double invd = d > 0.0 ? 1.0 / d : 1.0;
    // rows over the waves, columns over the lanes
    for (int i = j + 1 + (tid >> 6); i < K; i += SMALL_NT / 64) {
      const double lij = Ls[i * LD + j] * invd;
      for (int c = j + 1 + (tid & 63); c <= i; c += 64) Ls[i * LD + c] -= lij * Ls[c * LD + j];
    }
    __syncthreads();
  }
  // scale: L[i][j] = A[i][j] / sqrt(d_j), L[j][j] = sqrt(d_j) (d_j <= 0: 1)
  for (int j = tid; j < K; j += SMALL_NT) {
    const double d = Ls[j * LD + j];
    dg[j] = d > 0.0 ? sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int i = tid >> 6; i < K; i += SMALL_NT / 64)
    for (int j = tid & 63; j <= i; j += 64) Ls[i * LD + j] = (j < i) ? Ls[i * LD + j] / dg[j] : dg[i];
  __syncthreads();
  // X = L^{-1}: column c = tid / TPC; its TPC threads split the terms p of
  // x_i = (delta_ic - sum_{c<=p<i} L[i][p] x_p) / L[i][i] by p mod TPC.
  // X[p][c] lives at Ls[c][p] (p > c) or dg[c] (p = c).
  const int TPC = SMALL_NT / K;
  const int c = tid / TPC, q = tid % TPC;
  for (int i = 0; i < K; ++i) {
    double acc = 0.0;
    if (c < K && i > c)
      for (int p = c + q; p < i; p += TPC)
        acc += Ls[i * LD + p] * (p == c ? dg[c] : Ls[c * LD + p]);
    for (int o = 1; o < TPC; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (c < K && q == 0 && i >= c) {
      const double x = ((i == c ? 1.0 : 0.0) - acc) / Ls[i * LD + i];
      if (i == c) dg[c] = x;
      else Ls[c * LD + i] = x;
    }
    // the TPC threads of a column are lanes of one wave: the next step reads
    // x_i through LDS after this wave's store
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += SMALL_NT) {
    const int r = e / K, cc = e % K;
    Linv[e] = cc < r ? Ls[cc * LD + r] : (cc == r ? dg[r] : 0.0);
  }
}

// L^{-1} of the Cholesky factor of the K x K Gram Gm (K <= 64) by one wave,
// right-looking: lane i holds row i of the reduced matrix and row i of the
// inverse in registers.  Per column j the pivot, the column of multipliers
// l_cj and the finished row j of the inverse reach the other lanes by
// readlane (no LDS and no barriers, so the whole factorisation is one block
// of straight-line code the compiler can schedule across columns), for the
// rank-1 updates a_ic -= l_ij l_cj and z_i -= l_ij z_j.  Rows at or above j
// take a zero multiplier.  A non-positive pivot is taken as 1 (the rows are
// then far from orthonormal, which the caller's checks catch).  Linv (K x K,
// zeros above the diagonal) is written to global memory.
template <int K>
__global__ void __launch_bounds__(64)
k_chol_inv_wave(const double *__restrict__ Gm, double *__restrict__ Linv,
                const SvDevInfo *__restrict__ info) {
  static_assert(K <= 64, "one row per lane");
  if (info->status) return;
  const int i = threadIdx.x;
  double a[K], z[K];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    a[c] = (i < K && c <= i) ? Gm[i * K + c] : 0.0;
    z[c] = c == i ? 1.0 : 0.0;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double d = readlane_dbl(a[j], j);
    const double sd = d > 0.0 ? sqrt(d) : 1.0;
    const double r = 1.0 / sd;
    const double l = a[j] * r;   // l_ij in lane i > j
    const double li = i > j ? l : 0.0;
#pragma unroll
    for (int c = 0; c <= j; ++c) {   // row j of the inverse is final once scaled
      const double zj = readlane_dbl(z[c], j) * r;
      z[c] = i == j ? zj : z[c] - li * zj;
    }
#pragma unroll
    for (int c = j + 1; c < K; ++c) a[c] -= li * readlane_dbl(l, c);
  }
  if (i < K)
#pragma unroll
    for (int c = 0; c < K; ++c) Linv[i * K + c] = c <= i ? z[c] : 0.0;
}

__global__ void k_fill_random_rows(int K, int64_t N, double *__restrict__ X,
                                   const int32_t *__restrict__ complete, uint64_t seed,
                                   const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  const int j = blockIdx.x;
  if (!complete[j]) return;
  for (int64_t c = threadIdx.x; c < N; c += blockDim.x)
    X[(int64_t)j * N + c] = hash_unit(seed * 1000003ull + (uint64_t)j * 7919ull +
                                      (uint64_t)c * 2654435761ull);
}

// Gauss-Jordan inverse with partial pivoting of the K x K matrix W (K <= 128)
// in place in LDS, with the 1-norm condition number
// kappa_1 = ||W||_1 ||W^{-1}||_1 and the reset flag (kappa_1 > cond_reset or
// W numerically singular).  One block (256 threads, 512 at K = 128).  Per
// column c: the pivot is the largest |A[r][c]| over rows r >= c (lowest row
// on ties), the pivot row and row c are exchanged, row c is scaled by
// 1/pivot and every other row subtracts its multiple of it, the inverse
// taking column c's place (A[r][c] = -f_r / pivot); four barriers.  The row interchanges are
// undone at the end as one column permutation.  (Holding the rows in
// registers, 64 doubles a lane at K = 128, the compiler put the array in
// scratch memory: 2.3 ms per inverse at K = 128, 1.3 ms here.)
// threads of the block inverse: two waves per SIMD at K = 128, so that one
// wave's LDS latency hides behind the other's
constexpr int inv_block_nt(int K) { return K == 128 ? 512 : 256; }

template <int K>
__device__ __forceinline__ void
inverse_cond_block(const double *__restrict__ W, double *__restrict__ Winv,
                   int32_t *__restrict__ flag, double cond_reset, SvDevInfo *__restrict__ info,
                   int side) {
  if (info->status) return;
  constexpr int NT = inv_block_nt(K);
  static_assert(NT % K == 0, "a thread's elements share one column");
  static_assert(K <= NT, "one pivot candidate per thread");
  constexpr int GJ_PER = (K * K + NT - 1) / NT, GJ_RS = NT / K;
  constexpr int GJ_UB = GJ_PER < 16 ? GJ_PER : 16;
  static_assert(GJ_PER % GJ_UB == 0, "whole batches");
  __shared__ double As[K][K + 1];
  __shared__ double rowc[K], colf[K];
  __shared__ double cand_v[NT / 64];
  __shared__ int cand_i[NT / 64];
  __shared__ double red[NT / 64];
  __shared__ int piv[K], perm[K];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int e = t; e < K * K; e += NT) As[e / K][e % K] = W[e];
  __syncthreads();
  // ||W||_1: the largest column sum
  double cs = 0.0;
  for (int j = t; j < K; j += NT) {
    double sacc = 0.0;
    for (int r = 0; r < K; ++r) sacc += fabs(As[r][j]);
    cs = fmax(cs, sacc);
  }
  cs = wave_max(cs);
  if (lane == 0) red[w] = cs;
  __syncthreads();
  double n1 = red[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) n1 = fmax(n1, red[q]);
  const bool finite_in = isfinite(n1);
  bool sing = !finite_in;
  for (int c = 0; c < K && !sing; ++c) {
    // pivot candidate of each wave (rows r >= c it covers), then the block's
    // (K <= NT: thread t covers row c + t only, so rows rise with the lane
    // and the lowest lane holding the wave's maximum has the lowest row)
    const int rt = c + t;
    const double v = rt < K ? fabs(As[rt][c]) : -1.0;
    const double wb = wave_max(v);
    const unsigned long long hit = __ballot(v == wb && rt < K);
    const int bi = hit ? c + (t & ~63) + __builtin_ctzll(hit) : K;
    if (lane == 0) { cand_v[w] = hit ? wb : -1.0; cand_i[w] = bi; }
    __syncthreads();
    double pb = cand_v[0];
    int p = cand_i[0];
#pragma unroll
    for (int q = 1; q < NT / 64; ++q)
      if (cand_v[q] > pb || (cand_v[q] == pb && cand_i[q] < p)) { pb = cand_v[q]; p = cand_i[q]; }
    if (!(pb > 1e-300) || !(pb > 1e-15 * n1)) { sing = true; break; }
    // exchange rows c and p; keep row c (the pivot row) and column c
    for (int j = t; j < K; j += NT) {
      const double vp = As[p][j], vc = As[c][j];
      As[p][j] = vc;
      rowc[j] = vp;
    }
    if (t == 0) piv[c] = p;
    __syncthreads();
    for (int r = t; r < K; r += NT) colf[r] = r == c ? 0.0 : As[r][c];
    __syncthreads();
    const double pinv = 1.0 / rowc[c];
    // NT is a multiple of K, so all of a thread's elements lie in column
    // j = t mod K, rows t / K + u NT / K.  Loads of UB elements are issued
    // before their stores (one wave per SIMD here: each element's LDS latency
    // hides only behind the others', and a store between two loads of As
    // would keep the compiler from hoisting the second).
    const int j = t % K;
    const double pj = j == c ? pinv : rowc[j] * pinv;
#pragma unroll
    for (int u0 = 0; u0 < GJ_PER; u0 += GJ_UB) {
      double v[GJ_UB], f[GJ_UB];
#pragma unroll
      for (int u = 0; u < GJ_UB; ++u) {
        const int r = t / K + (u0 + u) * GJ_RS;
        v[u] = r < K ? As[r][j] : 0.0;
        f[u] = r < K ? colf[r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < GJ_UB; ++u) {
        const int r = t / K + (u0 + u) * GJ_RS;
        if (r < K) As[r][j] = r == c ? pj : (j == c ? -f[u] * pinv : v[u] - f[u] * pj);
      }
    }
    __syncthreads();
  }
  // the inverse is the final matrix with its columns permuted: column j of
  // W^{-1} is column perm[j] of A (the row interchanges undone in reverse)
  if (t == 0 && !sing) {
    for (int j = 0; j < K; ++j) perm[j] = j;
    for (int c = K - 1; c >= 0; --c) {
      const int p = piv[c];
      const int tmp = perm[c];
      perm[c] = perm[p];
      perm[p] = tmp;
    }
  }
  __syncthreads();
  // ||W^{-1}||_1 (max column sum, invariant under the column permutation)
  double ci = 0.0;
  for (int j = t; j < K; j += NT) {
    double sacc = 0.0;
    for (int r = 0; r < K; ++r) sacc += fabs(As[r][j]);
    ci = fmax(ci, sacc);
  }
  ci = wave_max(ci);
  __syncthreads();
  if (lane == 0) red[w] = ci;
  __syncthreads();
  double ninv = red[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) ninv = fmax(ninv, red[q]);
  const double kappa = sing ? INFINITY : n1 * ninv;
  if (!sing)
    for (int e = t; e < K * K; e += NT) Winv[e] = As[e / K][perm[e % K]];
  if (t == 0) {
    const bool reset = !(kappa <= cond_reset);
    *flag = reset ? 1 : 0;
    if (side == 0) info->kappa_U = kappa; else info->kappa_V = kappa;
    if (!finite_in) {
      if (atomicCAS(&info->status, 0, 4) == 0) info->failed_seq = -1;
    }
  }
}

struct InvJob {
  const double *W;
  double *Winv;
  int32_t *flag;
  int side;
};

// The same inverse and condition estimate for K <= 64 by one wave: lane r
// holds row r of W in registers and the Gauss-Jordan elimination runs in
// place with implicit partial pivoting (the pivot of column c is the largest
// |a[r][c]| over the rows not pivoted yet, lowest row on ties, and no row
// moves): the pivot row goes through LDS (alternating buffers, one wave
// barrier per column), every other row subtracts its multiple of it.  A pivot
// row is scaled by 1/pivot only at the end (later columns update it linearly,
// so the scaling commutes with them), which keeps K multiplications per
// column out of the branch of the pivot lane.  With
// p_c the pivot row of column c, the final array S holds W^{-1}[i][m] =
// S[p_i][q_m] with q the inverse of p.  The loop over columns is unrolled,
// so every register index is static.  1-norms through an LDS copy, one
// column per lane.  Flags, status and kappa as inverse_cond_block.
template <int K>
__device__ __forceinline__ void
inverse_cond_wave(const double *__restrict__ W, double *__restrict__ Winv,
                  int32_t *__restrict__ flag, double cond_reset, SvDevInfo *__restrict__ info,
                  int side) {
  if (info->status) return;
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double S[K][K + 1];
  __shared__ __align__(16) double prow[2][K];
  __shared__ int pv[K], qv[K];
  const int lane = threadIdx.x;
  const bool mine = lane < K;
  double a[K];
#pragma unroll
  for (int j = 0; j < K; ++j) a[j] = mine ? W[lane * K + j] : 0.0;
  // ||W||_1 = max column sum
  if (mine)
#pragma unroll
    for (int j = 0; j < K; ++j) S[lane][j] = a[j];
  wave_sync();
  double csum = 0.0;
  if (mine)
    for (int r = 0; r < K; ++r) csum += fabs(S[r][lane]);
  const double n1 = wave_max(csum);
  const bool finite_in = isfinite(n1);
  bool sing = !finite_in;
  bool used = !mine;
  double rs = 1.0;
#pragma clang loop unroll(full)
  for (int c = 0; c < K; ++c) {
    if (!sing) {
      const double cand = used ? -1.0 : fabs(a[c]);
      const double best = wave_max(cand);
      const unsigned long long hit = __ballot(cand == best && !used);
      const int p = hit ? __builtin_ctzll(hit) : 0;
      if (!(best > 1e-300) || !(best > 1e-15 * n1)) {
        sing = true;
      } else {
        double *pr = prow[c & 1];
        if (lane == p) {   // 16-byte stores: half the instructions of the one lane
#pragma unroll
          for (int j = 0; j < K; j += 2) *(d2 *)(pr + j) = d2{a[j], a[j + 1]};
          pv[c] = p;
        }
        wave_sync();
        const double pinv = 1.0 / pr[c];
        if (lane == p) {   // the pivot row's scaling by 1/pivot waits for the end
          used = true;
          rs = pinv;
          a[c] = 1.0;
        } else {
          const double g = a[c] * pinv;   // the row's multiplier
#pragma unroll
          for (int j = 0; j < K; j += 2) {
            const d2 q = *(const d2 *)(pr + j);
            a[j] = j == c ? -g : fma(-g, q.x, a[j]);
            a[j + 1] = j + 1 == c ? -g : fma(-g, q.y, a[j + 1]);
          }
        }
      }
    }
  }
  wave_sync();
  double kappa = INFINITY;
  if (!sing) {
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] *= rs;
    if (mine) qv[pv[lane]] = lane;
    wave_sync();
    // W^{-1}[i][m] = a_{p_i}[q_m]: lane r (= p_i for i = q_r) holds row i
    if (mine) {
      const int i = qv[lane];
#pragma unroll
      for (int j = 0; j < K; ++j) S[i][pv[j]] = a[j];
    }
    wave_sync();
    double ci = 0.0;
    if (mine)
      for (int r = 0; r < K; ++r) ci += fabs(S[r][lane]);
    kappa = n1 * wave_max(ci);
    for (int e = lane; e < K * K; e += 64) Winv[e] = S[e / K][e % K];
  }
  if (lane == 0) {
    const bool reset = !(kappa <= cond_reset);
    *flag = reset ? 1 : 0;
    if (side == 0) info->kappa_U = kappa; else info->kappa_V = kappa;
    if (!finite_in) {
      if (atomicCAS(&info->status, 0, 4) == 0) info->failed_seq = -1;
    }
  }
}

template <int K>
__global__ void __launch_bounds__(64)
k_inverse_cond2_wave(InvJob a, InvJob b, double cond_reset, SvDevInfo *__restrict__ info) {
  const InvJob j = blockIdx.x ? b : a;
  inverse_cond_wave<K>(j.W, j.Winv, j.flag, cond_reset, info, j.side);
}

template <int K>
__global__ void __launch_bounds__(512)
k_inverse_cond(const double *__restrict__ W, double *__restrict__ Winv,
               int32_t *__restrict__ flag, double cond_reset, SvDevInfo *__restrict__ info,
               int side) {
  inverse_cond_block<K>(W, Winv, flag, cond_reset, info, side);
}

// The two sides' inverses of one update in one launch (block 0: side a,
// block 1: side b); they are independent, so they run side by side.

template <int K>
__global__ void __launch_bounds__(512)
k_inverse_cond2(InvJob a, InvJob b, double cond_reset, SvDevInfo *__restrict__ info) {
  const InvJob j = blockIdx.x ? b : a;
  inverse_cond_block<K>(j.W, j.Winv, j.flag, cond_reset, info, j.side);
}

__global__ void k_commit_small(int K, const double *__restrict__ Wnew,
                               const int32_t *__restrict__ flag, double *__restrict__ W,
                               const double *__restrict__ theta, double *__restrict__ sig,
                               SvDevInfo *__restrict__ info, int side) {
  if (info->status) return;
  const bool reset = *flag != 0;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x)
    W[e] = reset ? ((e / K == e % K) ? 1.0 : 0.0) : Wnew[e];
  if (sig && threadIdx.x < K) sig[threadIdx.x] = theta[threadIdx.x];
  if (threadIdx.x == 0 && reset) {
    if (side == 0) info->resets_U += 1; else info->resets_V += 1;
  }
}

__global__ void k_check_finite(int64_t n, const double *__restrict__ x, SvDevInfo *info, int seq) {
  if (info->status) return;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) bad |= !isfinite(x[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) {
    if (atomicCAS(&info->status, 0, 4) == 0) info->failed_seq = seq;
  }
}

__global__ void k_op_begin(SvDevInfo *info, int two_sided) {
  if (info->status) return;
  info->rank = 0;
  info->rank2 = two_sided ? 0 : -1;
  info->min_kept = INFINITY;
  info->max_dropped = -1.0;
  info->reset_U = 0;
  info->reset_V = 0;
}

__global__ void k_op_end(SvDevInfo *info) {
  if (info->status) return;
  info->updates += 1;
}

__global__ void k_fill_identity(int K, double *W) {
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) W[e] = (e / K == e % K) ? 1.0 : 0.0;
}

// --------------------------------------------------------- realisation GEMM
// FP64 FMA variant: one block = 64 rows; the row tile is staged in LDS.
template <typename Tin, typename Tout, int K>
__global__ void __launch_bounds__(256)
k_realise_f64(int64_t rows, const Tin *__restrict__ in, const double *__restrict__ W,
              Tout *__restrict__ out, const int32_t *__restrict__ flag,
              const SvDevInfo *__restrict__ info) {
  if (info && info->status) return;
  if (flag && *flag == 0) return;
  constexpr int RB = K >= 128 ? 32 : 64;
  __shared__ double tile[RB][K + 1];
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int nr = (int)((rows - r0) < RB ? (rows - r0) : RB);
  for (int e = threadIdx.x; e < nr * K; e += blockDim.x)
    tile[e / K][e % K] = (double)in[(r0 + e / K) * K + e % K];
  __syncthreads();
  for (int e = threadIdx.x; e < nr * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    double acc = 0.0;
#pragma unroll 8
    for (int l = 0; l < K; ++l) acc += tile[r][l] * W[l * K + c];
    out[(r0 + r) * K + c] = (Tout)acc;
  }
}

// FP32 (MODE 1) and BF16x3 (MODE 2) MFMA variants, float in / float out.
// One block = 64 rows (4 waves x 16 rows), all K output columns per wave.
template <int MODE, int K>
__global__ void __launch_bounds__(256)
k_realise_lowp(int64_t rows, const float *__restrict__ in, const double *__restrict__ W,
               float *__restrict__ out, const int32_t *__restrict__ flag,
               const SvDevInfo *__restrict__ info) {
  if (info && info->status) return;
  if (flag && *flag == 0) return;
  constexpr int KP = K + 8;
  extern __shared__ unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int nr = (int)((rows - r0) < 64 ? (rows - r0) : 64);
  const int li = lane & 15;
  if constexpr (MODE == 1) {
    float *At = (float *)smem;            // 64 x KP
    float *Wt = At + 64 * KP;             // K x KP, W^T (row j = column j of W)
    for (int e = tid; e < 64 * K; e += 256) {
      const int r = e / K, c = e % K;
      At[r * KP + c] = r < nr ? in[(r0 + r) * K + c] : 0.f;
    }
    for (int e = tid; e < K * K; e += 256) Wt[(e % K) * KP + e / K] = (float)W[e];
    __syncthreads();
    const int lk = lane >> 4;
    for (int cb = 0; cb < K / 16; ++cb) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int kk = 0; kk < K; kk += 4) {
        const float a = At[(w * 16 + li) * KP + kk + lk];
        const float b = Wt[(cb * 16 + li) * KP + kk + lk];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = w * 16 + 4 * (lane >> 4) + q;
        if (r < nr) out[(r0 + r) * K + cb * 16 + li] = acc[q];
      }
    }
  } else {
    unsigned short *Ah = (unsigned short *)smem;   // 64 x KP
    unsigned short *Al = Ah + 64 * KP;
    unsigned short *Wh = Al + 64 * KP;             // K x KP (W^T)
    unsigned short *Wl = Wh + K * KP;
    for (int e = tid; e < 64 * K; e += 256) {
      const int r = e / K, c = e % K;
      const float x = r < nr ? in[(r0 + r) * K + c] : 0.f;
      const unsigned short h = f32_to_bf16_rne(x);
      Ah[r * KP + c] = h;
      Al[r * KP + c] = f32_to_bf16_rne(x - bf16_to_f32(h));
    }
    for (int e = tid; e < K * K; e += 256) {
      const float x = (float)W[e];
      const unsigned short h = f32_to_bf16_rne(x);
      Wh[(e % K) * KP + e / K] = h;
      Wl[(e % K) * KP + e / K] = f32_to_bf16_rne(x - bf16_to_f32(h));
    }
    __syncthreads();
    const int lk = (lane >> 4) * 4;
    f32x4 accs[K / 16];
#pragma unroll
    for (int cb = 0; cb < K / 16; ++cb) accs[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < K; kk += 16) {
      const int ra = (w * 16 + li) * KP + kk + lk;
      const s16x4 ah = *(const s16x4 *)(Ah + ra);
      const s16x4 al = *(const s16x4 *)(Al + ra);
#pragma unroll
      for (int cb = 0; cb < K / 16; ++cb) {
        const int rb = (cb * 16 + li) * KP + kk + lk;
        const s16x4 bh = *(const s16x4 *)(Wh + rb);
        const s16x4 bl = *(const s16x4 *)(Wl + rb);
        f32x4 c = accs[cb];
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
        accs[cb] = c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < K / 16; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = w * 16 + 4 * (lane >> 4) + q;
        if (r < nr) out[(r0 + r) * K + cb * 16 + li] = accs[cb][q];
      }
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
namespace svl {

// Kernels whose dynamic LDS may exceed 64 KiB must opt in once per process.
template <typename F>
static void allow_big_lds(F *f) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}


void gemm_f64(hipStream_t st, bool tA, bool tB, int64_t M, int64_t N, int64_t K, double alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
              double *C, int64_t ldc, const SvDevInfo *info) {
  if (M <= 0 || N <= 0) return;
  gemm_f64_sk(st, tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, 0, info);
}

// 64-wide column tiles, or 32-wide for widths 64 q + r with 0 < r <= 32
static int gemm_tile_n(int64_t N) { return (N % 64 != 0 && N % 64 <= 32) ? 32 : 64; }

// split K when the tiles alone leave CUs idle: about two blocks per CU,
// chunks whole stages, at most 64 (and at most max_parts) partial sums
static int64_t gemm_split_count(int64_t M, int64_t N, int64_t K, int64_t max_parts) {
  const int BN = gemm_tile_n(N);
  const int64_t tiles = ((N + BN - 1) / BN) * ((M + GB_M - 1) / GB_M);
  if (tiles >= 256 || K < 4 * GB_K) return 1;
  const int64_t stages = (K + GB_K - 1) / GB_K;
  int64_t splits = std::min<int64_t>(stages, (512 + tiles - 1) / tiles);
  splits = std::max<int64_t>(1, std::min<int64_t>({splits, max_parts, 64}));
  const int64_t per = (stages + splits - 1) / splits;   // stages per split
  return (stages + per - 1) / per;
}

int64_t gemm_f64_splits(int64_t M, int64_t N, int64_t K) {
  return gemm_split_count(M, N, K, 64);
}

void gemm_f64_sk(hipStream_t st, bool tA, bool tB, int64_t M, int64_t N, int64_t K, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                 double *C, int64_t ldc, double *ws, size_t ws_len, const SvDevInfo *info) {
  if (M <= 0 || N <= 0) return;
  const int BN = gemm_tile_n(N);
  const int64_t by_ws = ws ? (int64_t)(ws_len / (size_t)(M * N)) : 1;
  const int64_t splits = gemm_split_count(M, N, K, by_ws);
  double *part = splits > 1 ? ws : nullptr;
  const int64_t kchunk =
      splits > 1 ? ((K + GB_K - 1) / GB_K + splits - 1) / splits * GB_K : K;
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + GB_M - 1) / GB_M),
            (unsigned)splits);
  static const bool once = [] {
    allow_big_lds(k_gemm_f64<false, false, 64>); allow_big_lds(k_gemm_f64<false, true, 64>);
    allow_big_lds(k_gemm_f64<true, false, 64>); allow_big_lds(k_gemm_f64<true, true, 64>);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
#define SV_GM(TA_, TB_) do { \
    if (BN == 64) hipLaunchKernelGGL((k_gemm_f64<TA_, TB_, 64>), grid, dim3(256), gemm_lds_bytes<64>(), st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, info); \
    else hipLaunchKernelGGL((k_gemm_f64<TA_, TB_, 32>), grid, dim3(256), gemm_lds_bytes<32>(), st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, info); \
  } while (0)
  if (!tA && !tB) SV_GM(false, false);
  else if (!tA && tB) SV_GM(false, true);
  else if (tA && !tB) SV_GM(true, false);
  else SV_GM(true, true);
#undef SV_GM
  if (part)
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, st, M,
                       N, (int)splits, part, beta, C, ldc, info);
}

void gram_lowp(hipStream_t st, int mode, int64_t s, int K, const float *C, double *G,
               int64_t ldg, const SvDevInfo *info) {
  if (s <= 0) return;
  const int64_t nt = (s + 63) / 64;
  const unsigned tiles = (unsigned)(nt * (nt + 1) / 2);
  constexpr int KP = 128 + 8;
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    allow_big_lds(k_gram_lowp<1>); allow_big_lds(k_gram_lowp<2>);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  if (mode == 1) {
    const size_t sh = 2 * 64 * KP * sizeof(float);
    hipLaunchKernelGGL((k_gram_lowp<1>), dim3(tiles), dim3(256), sh, st, s, K, C, G, ldg, info);
  } else {
    const size_t sh = 4 * 64 * KP * sizeof(unsigned short);
    hipLaunchKernelGGL((k_gram_lowp<2>), dim3(tiles), dim3(256), sh, st, s, K, C, G, ldg, info);
  }
}

void copy_strided(hipStream_t st, int64_t R, int64_t C, const double *src, int64_t rs,
                  int64_t cs, double *dst, int64_t ldd, const SvDevInfo *info) {
  const int64_t n = R * C;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_strided, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, R, C,
                     src, rs, cs, dst, ldd, info);
}

void max_into(hipStream_t st, int64_t n, const double *v, SvDevInfo *info, int which) {
  hipLaunchKernelGGL(k_max_into, dim3(1), dim3(1024), 0, st, n, v, info, which);
}


void build_K_rows(hipStream_t st, int K, int64_t s, const double *sig, const double *Cp,
                  const double *L, int64_t ldl, double *Ko, const SvDevInfo *info) {
  const int64_t N = K + s, n = N * N;
  hipLaunchKernelGGL(k_build_K_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, s,
                     sig, Cp, L, ldl, Ko, info);
}

void build_M_border(hipStream_t st, int K, int64_t s, const double *sig, const double *Cp,
                    double *M, const SvDevInfo *info) {
  const int64_t n = (int64_t)K * (K + s);
  hipLaunchKernelGGL(k_build_M_border, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, s,
                     sig, Cp, M, info);
}

void build_X(hipStream_t st, int K, int64_t s, const double *Cp, const double *L, int64_t ldl,
             double *X, const SvDevInfo *info) {
  const int64_t n = (K + s) * s;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_build_X, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, s, Cp,
                     L, ldl, X, info);
}

void add_sigma_diag(hipStream_t st, int K, const double *sig, double *Ko, int64_t ld,
                    const SvDevInfo *info) {
  hipLaunchKernelGGL(k_add_sigma_diag, dim3(1), dim3(128), 0, st, K, sig, Ko, ld, info);
}

void theta_scale(hipStream_t st, int K, const double *lam, double *theta, double *Gv, int64_t N,
                 int32_t *complete, const SvDevInfo *info) {
  hipLaunchKernelGGL(k_theta_scale, dim3(K), dim3(256), 0, st, K, lam, theta, Gv, N, complete,
                     info);
}

void orthonormalize_rows(hipStream_t st, int K, int64_t N, double *X, const int32_t *complete,
                         uint64_t seed, double *Gm, double *Linv, double *Xtmp, double *ws,
                         size_t ws_len, const SvDevInfo *info) {
  if (complete)
    hipLaunchKernelGGL(k_fill_random_rows, dim3(K), dim3(256), 0, st, K, N, X, complete, seed,
                       info);
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const bool once = [] {
    allow_big_lds(k_chol_inv_small);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  // One Cholesky QR pass: the rows come in orthonormal to a few ulps (or, for
  // completion rows, as random vectors far from the span of the others), and
  // the orthogonality CholQR leaves is ~ u kappa^2 with kappa ~ 1 here.
  // L^{-1} by one wave (K <= 32) or by the blocked factor-and-invert of
  // 16 x 16 diagonal blocks (K = 64, 128; its dropping threshold 0, so only a
  // pivot that is not positive is dropped, leaving a zero row: the rows were
  // then far from orthonormal), then X <- L^{-1} X as a GEMM (each output row
  // its own dot products, no chain through earlier rows).  The drop flags go
  // to ws, which the Gram's reduction has finished reading by then.
  gemm_f64_sk(st, false, true, K, K, N, 1.0, X, N, X, N, 0.0, Gm, K, ws, ws_len, info);
  if (K == 16) {
    hipLaunchKernelGGL((k_chol_inv_wave<16>), dim3(1), dim3(64), 0, st, Gm, Linv, info);
  } else if (K == 32) {
    hipLaunchKernelGGL((k_chol_inv_wave<32>), dim3(1), dim3(64), 0, st, Gm, Linv, info);
  } else if (K == 64 || K == 128) {
    chol_drop_if(st, K, Gm, Linv, reinterpret_cast<int32_t *>(ws), 0.0, info, nullptr);
  } else {
    const size_t sh = (size_t)(K * (K + 1) + K) * sizeof(double);
    hipLaunchKernelGGL(k_chol_inv_small, dim3(1), dim3(SMALL_NT), sh, st, K, Gm, Linv, info);
  }
  gemm_f64(st, false, false, K, N, K, 1.0, Linv, K, X, N, 0.0, Xtmp, N, info);
  (void)hipMemcpyAsync(X, Xtmp, (size_t)K * N * sizeof(double), hipMemcpyDeviceToDevice, st);
}

void inverse_cond(hipStream_t st, int K, const double *W, double *Winv, int32_t *flag,
                  double cond_reset, SvDevInfo *info, int side) {
#define SV_INV(KK) hipLaunchKernelGGL((k_inverse_cond<KK>), dim3(1), dim3(inv_block_nt(KK)), 0, \
                                      st, W, Winv, flag, cond_reset, info, side)
  switch (K) {
    case 16: SV_INV(16); break;
    case 32: SV_INV(32); break;
    case 64: SV_INV(64); break;
    case 128: SV_INV(128); break;
  }
#undef SV_INV
}

void inverse_cond_pair(hipStream_t st, int K, const double *Wa, double *Wia, int32_t *fa, int sa,
                       const double *Wb, double *Wib, int32_t *fb, int sb, double cond_reset,
                       SvDevInfo *info) {
  const InvJob a{Wa, Wia, fa, sa}, b{Wb, Wib, fb, sb};
#define SV_INV2(KK) hipLaunchKernelGGL((k_inverse_cond2<KK>), dim3(2), dim3(inv_block_nt(KK)), 0, \
                                       st, a, b, cond_reset, info)
#define SV_INV2W(KK) hipLaunchKernelGGL((k_inverse_cond2_wave<KK>), dim3(2), dim3(64), 0, st, a, \
                                        b, cond_reset, info)
  switch (K) {
    case 16: SV_INV2W(16); break;
    case 32: SV_INV2W(32); break;
    case 64: SV_INV2W(64); break;
    case 128: SV_INV2(128); break;
  }
#undef SV_INV2
#undef SV_INV2W
}

void inverse_cond_one(hipStream_t st, int K, const double *W, double *Winv, int32_t *flag,
                      int side, double cond_reset, SvDevInfo *info) {
  const InvJob a{W, Winv, flag, side};
#define SV_INV1W(KK) hipLaunchKernelGGL((k_inverse_cond2_wave<KK>), dim3(1), dim3(64), 0, st, a, a, \
                                        cond_reset, info)
  switch (K) {
    case 16: SV_INV1W(16); break;
    case 32: SV_INV1W(32); break;
    case 64: SV_INV1W(64); break;
    case 128:
      hipLaunchKernelGGL((k_inverse_cond2<128>), dim3(1), dim3(inv_block_nt(128)), 0, st, a, a,
                         cond_reset, info);
      break;
  }
#undef SV_INV1W
}

void commit_small(hipStream_t st, int K, const double *Wnew, const int32_t *flag, double *W,
                  const double *theta, double *sig, SvDevInfo *info, int side) {
  hipLaunchKernelGGL(k_commit_small, dim3(1), dim3(256), 0, st, K, Wnew, flag, W, theta, sig,
                     info, side);
}

void check_finite(hipStream_t st, int64_t n, const double *x, SvDevInfo *info, int seq) {
  hipLaunchKernelGGL(k_check_finite, dim3(1), dim3(256), 0, st, n, x, info, seq);
}

void op_begin(hipStream_t st, SvDevInfo *info, int two_sided) {
  hipLaunchKernelGGL(k_op_begin, dim3(1), dim3(1), 0, st, info, two_sided);
}

void op_end(hipStream_t st, SvDevInfo *info) {
  hipLaunchKernelGGL(k_op_end, dim3(1), dim3(1), 0, st, info);
}

void fill_identity(hipStream_t st, int K, double *W) {
  hipLaunchKernelGGL(k_fill_identity, dim3(1), dim3(256), 0, st, K, W);
}

template <typename Tin, typename Tout>
void realise(hipStream_t st, int mode, int K, int64_t rows, const Tin *in, const double *W,
             Tout *out, const int32_t *flag, const SvDevInfo *info) {
  if (rows <= 0) return;
  const unsigned blocks = (unsigned)((rows + 63) / 64);
  if constexpr (std::is_same<Tin, float>::value && std::is_same<Tout, float>::value) {
    if (mode == 1 || mode == 2) {
      const int KP = K + 8;
      const size_t sh1 = (size_t)(64 + K) * KP * sizeof(float);
      const size_t sh2 = (size_t)2 * (64 + K) * KP * sizeof(unsigned short);
#define SV_RL(MM, KK, SH) do { allow_big_lds(k_realise_lowp<MM, KK>); (void)hipGetLastError(); hipLaunchKernelGGL((k_realise_lowp<MM, KK>), dim3(blocks), dim3(256), SH, st, rows, in, W, out, flag, info); } while (0)
      if (mode == 1) {
        switch (K) { case 16: SV_RL(1, 16, sh1); break; case 32: SV_RL(1, 32, sh1); break;
                     case 64: SV_RL(1, 64, sh1); break; case 128: SV_RL(1, 128, sh1); break; }
      } else {
        switch (K) { case 16: SV_RL(2, 16, sh2); break; case 32: SV_RL(2, 32, sh2); break;
                     case 64: SV_RL(2, 64, sh2); break; case 128: SV_RL(2, 128, sh2); break; }
      }
#undef SV_RL
      return;
    }
  }
#define SV_RF(KK) hipLaunchKernelGGL((k_realise_f64<Tin, Tout, KK>), dim3((unsigned)((rows + (KK >= 128 ? 31 : 63)) / (KK >= 128 ? 32 : 64))), dim3(256), 0, st, rows, in, W, out, flag, info)
  switch (K) { case 16: SV_RF(16); break; case 32: SV_RF(32); break;
               case 64: SV_RF(64); break; case 128: SV_RF(128); break; }
#undef SV_RF
}
template void realise<float, float>(hipStream_t, int, int, int64_t, const float *, const double *, float *, const int32_t *, const SvDevInfo *);
template void realise<double, double>(hipStream_t, int, int, int64_t, const double *, const double *, double *, const int32_t *, const SvDevInfo *);
template void realise<float, double>(hipStream_t, int, int, int64_t, const float *, const double *, double *, const int32_t *, const SvDevInfo *);
template void realise<double, float>(hipStream_t, int, int, int64_t, const double *, const double *, float *, const int32_t *, const SvDevInfo *);

}  // namespace svl
