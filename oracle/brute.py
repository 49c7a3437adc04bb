"""O0 -- the definition of one update, computed directly (small inputs only).

Definition 2 and Theorem 1: an update maps (U, s, V) to SVD_k of the updated
matrix built from A~ = U diag(s) V^T with one of the three forms of Section 2.
Here the updated matrix is formed densely and decomposed with LAPACK's dense
SVD; nothing of the Zha-Simon factorisation or of SV-LCOV is used.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _dense(x):
    if sp.issparse(x):
        return x.toarray()
    if hasattr(x, "to_dense"):
        return x.to_dense()
    return np.asarray(x, dtype=np.float64)


def updated_matrix(U, s, V, update):
    """The dense updated matrix for ("rows", E) | ("cols", Ec_T) |
    ("weights", D_T, Em_T)."""
    A = (U * s) @ V.T
    kind = update[0]
    if kind == "rows":
        return np.vstack([A, _dense(update[1])])
    if kind == "cols":
        return np.hstack([A, _dense(update[1]).T])
    if kind == "weights":
        return A + _dense(update[1]).T @ _dense(update[2])
    raise ValueError(kind)


def apply(U, s, V, update):
    """Top-k singular triplets of the updated matrix and its full spectrum."""
    k = s.size
    Abar = updated_matrix(U, s, V, update)
    Ub, th, Vt = np.linalg.svd(Abar, full_matrices=False)
    return Ub[:, :k].copy(), th[:k].copy(), Vt[:k].T.copy(), dict(theta_hat=th,
                                                                   Abar=Abar)
