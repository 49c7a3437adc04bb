// Launchers of the initial SVD's kernels (k_rsvd.hip) beyond those shared
// with the update path: Cholesky QR passes that run only when the previous
// pass left work for them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace svl {

// Off-diagonal bound of the column-scaled Gram below which one Cholesky QR
// pass suffices (condition number at most 1 + 1.3e-4 for 128 columns).
constexpr double ORTH_GATE_TAU = 1e-6;

// ts_gram / chol_drop that do nothing (chol_drop: Out = I and no column to
// complete) when *need == 0; need == NULL runs them always.
void ts_gram_if(hipStream_t st, int64_t R, int L, const double *Y, double *G, double *ws,
                const SvDevInfo *info, const int32_t *need);
void chol_drop_if(hipStream_t st, int L, const double *G, double *Out, int32_t *complete,
                  double rtol, const SvDevInfo *info, const int32_t *need);
// Orthonormal basis of the columns of the R x L panel X (R >= L) by one pass
// of Cholesky QR with dropping and completion, and a second pass only when
// the first completed a column or its input was not orthonormal to within
// ORTH_GATE_TAU; need is one device word of scratch.  The result is in X.
// gate_tau replaces ORTH_GATE_TAU where the caller can accept more: one pass
// of Cholesky QR leaves an orthogonality error of about u cond^2, and the
// gate bounds cond by 1 + (L - 1) gate_tau.
double *orth_cols_cond(hipStream_t st, int64_t R, int L, double *X, double *Y, double *G,
                       double *Out, int32_t *complete, int32_t *need, double *ws, size_t ws_len,
                       uint64_t seed, double rtol, const SvDevInfo *info,
                       double gate_tau = ORTH_GATE_TAU);

}  // namespace svl
