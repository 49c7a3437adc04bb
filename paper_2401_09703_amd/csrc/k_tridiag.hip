// Householder tridiagonalisation Q^T M Q = T of a symmetric FP64 matrix, the
// first stage of the top-k eigensolver behind the (k+s) Rayleigh-Ritz SVD
// (Section 2.1, step 2), as one cooperative kernel.  Each block owns the rows
// r = g, g + G, ... of M (cyclic, so the shrinking trailing matrix stays
// balanced).  Per column one grid-wide barrier: every block recomputes the
// next reflector redundantly from the published row, applies the pending
// rank-2 update to its own rows fused with the product p = tau M v, and
// publishes its part of p.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

using namespace svk;

namespace {

constexpr int TRI_MAX_BLOCKS = svl::TRI_MAX_BLOCKS;

// Householder tridiagonalisation, one cooperative launch (all blocks
// co-resident).  Block g owns rows r = g, g + G, ...; with LDS_ROWS they live
// in LDS for the whole reduction, otherwise in A.  Reflector i is left in row
// i of A (columns i+1 .., unit leading entry), d, e, tau in work arrays.
// NT = 64 (one wave per block: block-wide reductions and barriers are nearly
// free) for moderate N, 256 when the owned rows need more lanes.
template <bool LDS_ROWS, int NT>
__global__ void __launch_bounds__(NT)
k_tridiag(int N, double *__restrict__ A, int64_t lda, double *__restrict__ d,
          double *__restrict__ e, double *__restrict__ tau, double *__restrict__ pbuf,
          double *__restrict__ rowbuf, unsigned *__restrict__ flags, unsigned epoch0,
          const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double sm[];
  const int G = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int nw = NT / 64;
  if (N < 3) {
    if (g == 0 && tid == 0) {
      d[0] = A[0];
      if (N == 2) { e[0] = A[1]; d[1] = A[lda + 1]; }
    }
    return;
  }
  double *X = sm, *VP = sm + N, *WP = sm + 2 * N;
  double *rows = sm + 3 * N;   // LDS_ROWS: owned rows, local index (r - g) / G
  if constexpr (LDS_ROWS) {
    const int nr = (N - g + G - 1) / G;
    for (int lr = w; lr < nr; lr += nw) {
      const double *src = A + (int64_t)(g + lr * G) * lda;
      for (int j = lane; j < N; j += 64) rows[(int64_t)lr * N + j] = src[j];
    }
  }
  // Every per-entry loop below gives entry j to thread j mod NT, so a thread
  // only reads back what it wrote itself; the two block barriers per column
  // (plus the grid barrier's) cover the cross-thread reads: the scalars
  // alpha, w_{i+1}, the two reductions, and the row loop that reads whole
  // vectors.  The new column X stays unscaled until after the grid barrier:
  // the row loop applies the reflector's scale on the fly.
  __shared__ double red0[NT / 64], red1[NT / 64];
  __shared__ double p_lead;   // p_{i+1}, published by its owner thread
  auto first = [&](int lo) {
    int o = (tid - lo) % NT;
    return lo + (o < 0 ? o + NT : o);
  };
  double part = 0.0;   // sum of X[j]^2 over j >= i + 2, carried between iterations
  for (int j = tid; j < N; j += NT) {
    const double x = A[j];
    X[j] = x;
    if (j >= 2) part += x * x;
  }
  part = wave_sum(part);
  if (lane == 0) red1[w] = part;
  __syncthreads();
  for (int i = 0; i <= N - 3; ++i) {
    const double dii = X[i];
    const double alpha = X[i + 1];
    double xn2 = 0.0;
#pragma unroll
    for (int q = 0; q < nw; ++q) xn2 += red1[q];
    double beta, t, scl;
    if (xn2 == 0.0) {
      t = 0.0; beta = alpha; scl = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xn2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scl = 1.0 / (alpha - beta);
    }
    double *pb = pbuf + (int64_t)(i & 1) * N;
    double *rb = rowbuf + (int64_t)(i & 1) * N;
    // owned rows r >= i+1: pending rank-2 update, then p = tau M v
    const int lr0 = (i + 1 - g + G - 1) / G > 0 ? (i + 1 - g + G - 1) / G : 0;
    for (int lr = lr0 + w; g + lr * G < N; lr += nw) {
      const int r = g + lr * G;
      double *Ar;
      if constexpr (LDS_ROWS) Ar = rows + (int64_t)lr * N;
      else Ar = A + (int64_t)r * lda;
      const double vpr = i >= 1 ? VP[r] : 0.0, wpr = i >= 1 ? WP[r] : 0.0;
      const bool pub = (r == i + 1);
      // p_r = tau (a_{r,i+1} + scl sum_{j>i+1} a_rj X_j): v_{i+1} = 1, v_j = scl X_j
      double acc = 0.0, lead = 0.0;
#pragma unroll 4
      for (int j = i + 1 + lane; j < N; j += 64) {
        double a = Ar[j];
        if (i >= 1) {
          a -= vpr * WP[j] + wpr * VP[j];
          Ar[j] = a;
        }
        if (pub) st_coh(&rb[j], a);
        if (j == i + 1) lead = a;
        else acc += a * X[j];
      }
      acc = wave_sum(acc);
      if (lane == 0) st_coh(&pb[r], t * (lead + scl * acc));   // lane 0 holds a_{r,i+1}
    }
    flag_barrier(flags, epoch0 + (unsigned)i + 1u);
    const bool owner = (g == i % G);   // row i of M is finished: keep the reflector there
    if (owner && tid == 0) { d[i] = dii; e[i] = beta; tau[i] = t; }
    // w = p - (tau/2)(p.v) v, and the next row: published row minus update i
    double *Xn = VP;
    double part2 = 0.0;
    for (int j = first(i + 1); j < N; j += NT) {
      const double pj = ld_coh(&pb[j]);
      const double rj = ld_coh(&rb[j]);
      const double xj = (j == i + 1) ? 1.0 : X[j] * scl;   // v_j
      X[j] = xj;
      if (owner) A[(int64_t)i * lda + j] = xj;
      if (j == i + 1) p_lead = pj;
      WP[j] = pj;
      Xn[j] = rj;
      part2 += pj * xj;
    }
    part2 = wave_sum(part2);
    if (lane == 0) red0[w] = part2;
    __syncthreads();
    double pv = 0.0;
#pragma unroll
    for (int q = 0; q < nw; ++q) pv += red0[q];
    const double aw = -0.5 * t * pv;
    const double wi1 = p_lead + aw;   // w_{i+1} (v_{i+1} = 1)
    part = 0.0;
    for (int j = first(i + 1); j < N; j += NT) {
      const double xj = X[j];
      const double wj = WP[j] + aw * xj;
      WP[j] = wj;
      const double xn = Xn[j] - (wj + wi1 * xj);
      Xn[j] = xn;
      if (j >= i + 3) part += xn * xn;
    }
    part = wave_sum(part);
    if (lane == 0) red1[w] = part;
    __syncthreads();
    VP = X;
    X = Xn;
  }
  if (g == 0 && tid == 0) {
    d[N - 2] = X[N - 2];
    e[N - 2] = X[N - 1];
  }
  if (g == (N - 1) % G && tid == 0) {
    double a;
    if constexpr (LDS_ROWS) a = rows[(int64_t)((N - 1 - g) / G) * N + N - 1];
    else a = A[(int64_t)(N - 1) * lda + N - 1];
    d[N - 1] = a - 2.0 * VP[N - 1] * WP[N - 1];
  }
}

// The same reduction for small N (N <= TRI_SMALL_N) in one block with the
// whole matrix in LDS (row stride N + 1), three block barriers per column.
// Four threads own row i+1+q of the trailing matrix, one in four columns
// each: they form its entry of p = tau M v and of w, apply the rank-2 update
// to the row, and the four owning the next column's row also form that row's
// norm for the next reflector.  Every row loop issues its LDS loads in
// batches of 8 before using them (an LDS round trip is ~120 cycles, so a
// dependent load per iteration would dominate).  v is read from row i of S
// (v_j = scl x_j), which no later step of the column writes.  Conventions
// and outputs as k_tridiag: beta = -sign(alpha) ||x||, tau = (beta - alpha) /
// beta, v_{i+1} = 1, reflector i left in row i of A (columns i+1 ..).
constexpr int TRI_SMALL_N = 128;
constexpr int TRI_SMALL_NT = 512;
constexpr int TS_TPR = 4;                             // threads per row
constexpr int TS_CPT = TRI_SMALL_N / TS_TPR;          // columns per thread (max)
constexpr int TS_B = 8;                               // loads in flight

__global__ void __launch_bounds__(TRI_SMALL_NT)
k_tridiag_small(int N, double *__restrict__ A, int64_t lda, double *__restrict__ d,
                double *__restrict__ e, double *__restrict__ tau,
                const SvDevInfo *__restrict__ info) {
  if (info->status) return;
  extern __shared__ double sm[];
  constexpr int NT = TRI_SMALL_NT, nw = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = tid / TS_TPR, sub = tid % TS_TPR;
  if (N < 3) {
    if (tid == 0) {
      d[0] = A[0];
      if (N == 2) { e[0] = A[1]; d[1] = A[lda + 1]; }
    }
    return;
  }
  const int ld = N + 1;
  double *S = sm, *P = sm + (int64_t)N * ld;
  // d, e, tau and the reflectors' scales stay in LDS until the end: a global
  // store inside the loop would make every block barrier wait for it
  double *dd = P + N, *ee = dd + N, *tt = ee + N, *sc = tt + N;
  __shared__ double red[nw];
  __shared__ double xn2_s, alpha_s;
  for (int r = tid / 64; r < N; r += nw)
    for (int c = lane; c < N; c += 64) S[r * ld + c] = A[(int64_t)r * lda + c];
  double part = 0.0;
  for (int j = 2 + tid; j < N; j += NT) part += A[j] * A[j];   // row 0 = column 0
  part = wave_sum(part);
  if (lane == 0) red[w] = part;
  __syncthreads();
  if (tid == 0) {
    double x = 0.0;
    for (int u = 0; u < nw; ++u) x += red[u];
    xn2_s = x;
    alpha_s = S[1];
  }
  __syncthreads();
  for (int i = 0; i <= N - 3; ++i) {
    const double *Si = S + i * ld;
    const double xn2 = xn2_s, alpha = alpha_s;
    double beta, t, scl;
    if (xn2 == 0.0) {
      t = 0.0; beta = alpha; scl = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xn2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scl = 1.0 / (alpha - beta);
    }
    if (tid == 0) { dd[i] = Si[i]; ee[i] = beta; tt[i] = t; sc[i] = scl; }
    const int r = i + 1 + q;
    const bool act = r < N;
    const int c0 = i + 1 + sub;                   // this thread's first column
    const int nc = act && c0 < N ? (N - c0 + TS_TPR - 1) / TS_TPR : 0;
    double *Sr = S + (act ? r : i) * ld;
    // p_r = tau sum_j M_rj v_j
    double acc = 0.0;
    for (int u0 = 0; u0 < nc; u0 += TS_B) {
      double a[TS_B], x[TS_B];
#pragma unroll
      for (int u = 0; u < TS_B; ++u) {
        const int c = c0 + (u0 + u) * TS_TPR;
        const int cc = c < N ? c : c0;
        a[u] = Sr[cc];
        x[u] = Si[cc];
      }
#pragma unroll
      for (int u = 0; u < TS_B; ++u) {
        const int c = c0 + (u0 + u) * TS_TPR;
        if (c < N) acc += a[u] * (c == i + 1 ? 1.0 : x[u] * scl);
      }
    }
    acc = quad_sum(acc);   // the four threads of a row are one lane quad
    const double pr = t * acc;
    const double vr = act ? ((r == i + 1) ? 1.0 : Si[r] * scl) : 0.0;
    double pv = (act && sub == 0) ? pr * vr : 0.0;
    pv = wave_sum(pv);
    if (lane == 0) red[w] = pv;
    __syncthreads();
    double pvs = 0.0;
#pragma unroll
    for (int u = 0; u < nw; ++u) pvs += red[u];
    const double wr = pr - 0.5 * t * pvs * vr;   // w_r
    if (act && sub == 0) P[r] = wr;
    __syncthreads();
    // M22 -= v w^T + w v^T on the row; the next reflector's row norm
    double nn = 0.0;
    for (int u0 = 0; u0 < nc; u0 += TS_B) {
      double a[TS_B], x[TS_B], pw[TS_B];
#pragma unroll
      for (int u = 0; u < TS_B; ++u) {
        const int c = c0 + (u0 + u) * TS_TPR;
        const int cc = c < N ? c : c0;
        a[u] = Sr[cc];
        x[u] = Si[cc];
        pw[u] = P[cc];
      }
#pragma unroll
      for (int u = 0; u < TS_B; ++u) {
        const int c = c0 + (u0 + u) * TS_TPR;
        if (c < N) {
          const double vc = (c == i + 1) ? 1.0 : x[u] * scl;
          const double v = a[u] - (vr * pw[u] + wr * vc);
          Sr[c] = v;
          if (r == i + 1) {
            if (c >= i + 3) nn += v * v;
            if (c == i + 2) alpha_s = v;
          }
        }
      }
    }
    nn = quad_sum(nn);   // converged: every lane takes part
    if (q == 0 && sub == 0) xn2_s = nn;   // the quad of row i + 1
    __syncthreads();
  }
  if (tid == 0) {
    dd[N - 2] = S[(N - 2) * ld + N - 2];
    ee[N - 2] = S[(N - 2) * ld + N - 1];
    dd[N - 1] = S[(N - 1) * ld + N - 1];
  }
  __syncthreads();
  // row i of S (columns > i) is no longer touched after column i: it still
  // holds x, and v_j = scl_i x_j
  for (int i = w; i <= N - 3; i += nw)
    for (int j = i + 1 + lane; j < N; j += 64)
      A[(int64_t)i * lda + j] = (j == i + 1) ? 1.0 : S[i * ld + j] * sc[i];
  for (int i = tid; i < N; i += NT) {
    d[i] = dd[i];
    if (i < N - 1) e[i] = ee[i];
    if (i < N - 2) tau[i] = tt[i];
  }
}

// The same reduction with the matrix in registers, one block of
// NT = NMAX * TPR threads: thread t holds row r = t / TPR at the columns
// c = t % TPR + TPR j (j < NMAX / TPR), so the TPR threads of a row are one
// TPR-lane group of a wave (row sums by DPP steps).  N <= 128 takes eight
// threads per row (1024 threads, 16 entries each); 128 < N <= 160 four
// (640 threads, 40 entries each: the registers of 1024 threads cannot hold
// more).  Per column: the threads of row i form the reflector from their
// registers and publish v, every thread forms its row's share of p = tau M v,
// a block reduction gives p.v, and each thread applies the rank-2 update to
// its entries with w rebuilt from p and v in LDS.  Two block barriers per
// column; v, p and the partial sums alternate between two LDS buffers so
// that the next column's writes never meet this column's reads.  A wave
// whose rows are all <= i only takes part in the reduction.  The reflectors
// stay in the registers of their rows (which no later update changes) and
// d, e, tau in LDS until the end: a global store inside the loop would hold
// up every block barrier until it completed.  Conventions as k_tridiag.
constexpr int TR_N = 128, TR_NT = 1024;
constexpr int TR2_N = svl::EIG_ONE_BLOCK_N, TR2_TPR = 4, TR2_NT = TR2_N * TR2_TPR;

__device__ __forceinline__ double sum8(double v) {
  v = quad_sum(v);
  return v + dpp_d<DPP_ROW_HALF_MIRROR>(v);
}

template <int TPR>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(TPR == 2 || TPR == 4 || TPR == 8, "row group");
  if (TPR == 8) return sum8(v);
  if (TPR == 4) return quad_sum(v);
  return v + dpp_d<DPP_QUAD_XOR1>(v);
}

template <int TPR, int NMAX>
__global__ void __launch_bounds__(NMAX * TPR)
k_tridiag_reg(int N, double *__restrict__ A, int64_t lda, double *__restrict__ d,
              double *__restrict__ e, double *__restrict__ tau, const SvDevInfo *__restrict__ info) {
  constexpr int NT = NMAX * TPR, CPT = NMAX / TPR, RPW = 64 / TPR;
  if (info->status) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = tid / TPR, s = tid % TPR;
  if (N < 3) {
    if (tid == 0) {
      d[0] = A[0];
      if (N == 2) { e[0] = A[1]; d[1] = A[lda + 1]; }
    }
    return;
  }
  __shared__ double vb[2][NMAX];
  __shared__ double pb[2][NMAX];
  __shared__ double part[2][NT / 64];
  __shared__ double tb[2];
  __shared__ double dd[NMAX], ee[NMAX], tt[NMAX], sc[NMAX], xr[NMAX];
  double a[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = s + TPR * j;
    a[j] = (r < N && c < N) ? A[(int64_t)r * lda + c] : 0.0;
  }
  for (int c = tid; c < 2 * NMAX; c += NT) vb[c / NMAX][c % NMAX] = 0.0;
  __syncthreads();
  for (int i = 0; i <= N - 3; ++i) {
    const int b = i & 1;
    // row i: its group copies the row to xr, reads d_i = x_i, alpha =
    // x_{i+1} and ||x_{i+2..}||^2 back and writes the reflector v to vb (1
    // at i + 1, scl x_c beyond; vb[b] already holds 0 up to column i - 2 and
    // beyond N - 1 from its last use two columns ago, and columns i - 1, i
    // are cleared here).  The registers keep x (no later update changes row
    // i); the reflector is written out from x and scl at the end.  No
    // per-column conditions on the register array: those compile to one
    // lane mask per column.
    if (r == i) {
      double *xw = &xr[s];
#pragma unroll
      for (int j = 0; j < CPT; ++j) xw[TPR * j] = a[j];
      // the group is TPR lanes of one wave, whose LDS accesses are in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int q = 0;
      for (int c = i + 2 + s; c < N; c += TPR, ++q) {
        const double x = xr[c];
        s4[q & 3] += x * x;
      }
      const double ss = group_sum<TPR>((s4[0] + s4[1]) + (s4[2] + s4[3]));
      const double di = xr[i], al = xr[i + 1];
      double beta, t, scl;
      if (ss == 0.0) {
        t = 0.0; beta = al; scl = 0.0;
      } else {
        const double nrm = sqrt(al * al + ss);
        beta = al >= 0.0 ? -nrm : nrm;
        t = (beta - al) / beta;
        scl = 1.0 / (al - beta);
      }
      for (int c = i + 2 + s; c < N; c += TPR) vb[b][c] = xr[c] * scl;
      if (s == 0) {
        if (i >= 1) vb[b][i - 1] = 0.0;
        vb[b][i] = 0.0;
        vb[b][i + 1] = 1.0;
        tb[b] = t;
        dd[i] = di;
        ee[i] = beta;
        tt[i] = t;
        sc[i] = scl;
      }
    }
    __syncthreads();
    const double t = tb[b];
    const bool wact = RPW * w + RPW - 1 > i && RPW * w < N;
    double pr = 0.0, vr = 0.0, pv = 0.0;
    if (wact) {
      // v is zero at columns <= i and p at rows <= i, so no per-column
      // condition is needed
      // (one base address per buffer, the columns at immediate offsets)
      const double *vs = &vb[b][s];
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < CPT; ++j) a4[j & 3] += a[j] * vs[TPR * j];
      const double acc = group_sum<TPR>((a4[0] + a4[1]) + (a4[2] + a4[3]));
      const bool act = r > i && r < N;
      pr = act ? t * acc : 0.0;
      vr = act ? vb[b][r] : 0.0;
      if (s == 0) pb[b][r] = pr;
      pv = (s == 0) ? pr * vr : 0.0;
      pv = wave_sum(pv);
    } else if (s == 0) {
      pb[b][r] = 0.0;
    }
    if (lane == 0) part[b][w] = pv;
    __syncthreads();
    if (wact) {
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) p4[q & 3] += part[b][q];
      const double pvs = (p4[0] + p4[1]) + (p4[2] + p4[3]);
      const double K = 0.5 * t * pvs;
      const double wr = pr - K * vr;
      // M_rc -= v_r w_c + w_r v_c, w_c = p_c - K v_c
      const double *vs = &vb[b][s], *ps = &pb[b][s];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const double vc = vs[TPR * j];
        a[j] -= vr * (ps[TPR * j] - K * vc) + wr * vc;
      }
    }
  }
  // the last 2 x 2 block, the reflectors (rows 0 .. N-3 of A, columns > r:
  // 1 at r + 1, scl_r x_c beyond) and d, e, tau
  __syncthreads();
  const double scr = r <= N - 3 ? sc[r] : 0.0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = s + TPR * j;
    if (r == N - 2 && c == N - 2) d[N - 2] = a[j];
    if (r == N - 2 && c == N - 1) e[N - 2] = a[j];
    if (r == N - 1 && c == N - 1) d[N - 1] = a[j];
    if (r <= N - 3 && c > r && c < N) A[(int64_t)r * lda + c] = c == r + 1 ? 1.0 : a[j] * scr;
  }
  __syncthreads();
  for (int q = tid; q <= N - 3; q += NT) {
    d[q] = dd[q];
    e[q] = ee[q];
    tau[q] = tt[q];
  }
}

}  // namespace

namespace svl {

// Work layout: d, e, tau (3N), pbuf, rowbuf (4N), inverse-iteration scratch.
// flags: TRI_MAX_BLOCKS * FLAG_STRIDE unsigned, zero-initialised once; *epoch
// is advanced past the epochs this launch uses.
int eig_tridiag(hipStream_t st, int64_t N64, double *A, double *work, unsigned *flags,
                unsigned *epoch, const SvDevInfo *info) {
  const int N = (int)N64;
  if (N64 > eig_max_n() || N < 1) return -1;
  double *d = work, *e = d + N, *tau = e + N, *pbuf = tau + N, *rowbuf = pbuf + 2 * N;
  if (N <= TR_N && !getenv("SVLCOV_TRI_LDS")) {   // one block, the matrix in registers
    hipLaunchKernelGGL((k_tridiag_reg<8, TR_N>), dim3(1), dim3(TR_NT), 0, st, N, A, N64, d, e,
                       tau, info);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  if (N <= TR2_N) {   // the same with four threads per row
    hipLaunchKernelGGL((k_tridiag_reg<TR2_TPR, TR2_N>), dim3(1), dim3(TR2_NT), 0, st, N, A, N64,
                       d, e, tau, info);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  if (N <= TRI_SMALL_N) {   // one block, the matrix in LDS
    // thread-safe one-time set-up (dispatch may run on several host threads)
    static const bool small_once = [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag_small),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      return true;
    }();
    (void)small_once;
    const size_t sh = ((size_t)N * (N + 1) + 5 * N) * sizeof(double);
    hipLaunchKernelGGL(k_tridiag_small, dim3(1), dim3(TRI_SMALL_NT), sh, st, N, A, N64, d, e,
                       tau, info);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  // block widths: 256 threads, or one wave per owned row (5..8 waves) when
  // the rows live in LDS, so that no wave carries two rows
  static const void *const fns_lds[5] = {
      reinterpret_cast<const void *>(k_tridiag<true, 256>),
      reinterpret_cast<const void *>(k_tridiag<true, 320>),
      reinterpret_cast<const void *>(k_tridiag<true, 384>),
      reinterpret_cast<const void *>(k_tridiag<true, 448>),
      reinterpret_cast<const void *>(k_tridiag<true, 512>)};
  static const void *const fn_mem = reinterpret_cast<const void *>(k_tridiag<false, 256>);
  // thread-safe one-time set-up (dispatch may run on several host threads)
  static const int ncu = [] {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 0) n = 1;
    if (n > TRI_MAX_BLOCKS) n = TRI_MAX_BLOCKS;
    const int lim = 160 * 1024;
    for (const void *f : fns_lds)
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute(fn_mem, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipGetLastError();
    return n;
  }();
  // block count G: one block per 8 rows from N = 512 while those 8 rows and
  // the three work vectors fit in LDS, else one per 4 rows (measured on
  // MI355X: at N = 1064, 133 blocks of 8 rows beat 266 of 4 by 5 %, fewer
  // blocks meeting at each column's grid barrier and reading the published
  // row; small N want the rows spread, and a block whose rows leave LDS is
  // several times slower); at most one block per CU; SVLCOV_TRI_BLOCKS
  // overrides it for tuning sweeps
  // (rounded up, so that no block gets a ninth or fifth row: with a floor,
  // N not a multiple of the row count left some waves with two rows, or a
  // block's rows outside LDS)
  const bool eight = N >= 512 && (size_t)(3 + 8) * N * sizeof(double) <= (size_t)150 * 1024;
  const int rows = eight ? 8 : 4;
  int G = (N + rows - 1) / rows;
  if (const char *ev = getenv("SVLCOV_TRI_BLOCKS")) G = atoi(ev);
  if (G < 1) G = 1;
  if (G > ncu) G = ncu;
  const int rmax = (N + G - 1) / G;
  const size_t base_sh = (size_t)3 * N * sizeof(double);
  const size_t rows_sh = (size_t)rmax * N * sizeof(double);
  const bool lds_rows = base_sh + rows_sh <= (size_t)150 * 1024;
  const size_t sh = lds_rows ? base_sh + rows_sh : base_sh;
  int waves = 4;
  if (lds_rows) waves = rmax < 4 ? 4 : (rmax > 8 ? 8 : rmax);
  const int NT = 64 * waves;
  const void *fn = lds_rows ? fns_lds[waves - 4] : fn_mem;
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, sh);
  (void)hipGetLastError();
  if (nb < 1) return -2;
  if (G > nb * ncu) return -2;   // (cannot happen: G <= ncu) every block must be co-resident
  unsigned e0 = take_epochs(st, flags, epoch, (unsigned)N);
  int64_t lda = N64;
  void *args[] = {(void *)&N, (void *)&A, (void *)&lda, (void *)&d, (void *)&e, (void *)&tau,
                  (void *)&pbuf, (void *)&rowbuf, (void *)&flags, (void *)&e0, (void *)&info};
  hipError_t err = hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, sh, st);
  return err == hipSuccess ? 0 : -3;
}

}  // namespace svl
