"""O5 -- the initial truncated SVD from a sparse matrix (test infrastructure).

The step before the update path: every experiment of Section 5 starts from a
truncated SVD of the initial half of the matrix, and the paper does not say
how it is computed; the introduction points to randomised numerical linear
algebra for it.  This oracle takes the randomised range finder with power
iterations (Halko, Martinsson and Tropp, 2011, Algorithms 4.4 and 5.1), with
the Gaussian test matrix Omega given by the caller:

    Y = A Omega,  Q = orth(Y)
    repeat q times:  Z = orth(A^T Q),  Q = orth(A Z)
    B = Q^T A  (l x n),  B = U_B S V_B^T  (small dense SVD)
    U = Q U_B[:, :k],  S = S[:k],  V = V_B[:, :k]

Plain FP64 (Householder QR, LAPACK SVD); dense where it is small.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _orth(X: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(X)
    return Q


def rsvd(A, k: int, Omega: np.ndarray, power: int = 2):
    """Rank-k randomised SVD of the sparse (or dense) m x n matrix A with the
    n x l test matrix Omega (l >= k) and ``power`` power iterations.
    Returns U (m x k), s (k), V (n x k)."""
    A = sp.csr_matrix(A) if sp.issparse(A) or hasattr(A, "toarray") else sp.csr_matrix(np.asarray(A))
    Omega = np.asarray(Omega, dtype=np.float64)
    assert Omega.shape[0] == A.shape[1] and Omega.shape[1] >= k
    Q = _orth(A @ Omega)
    for _ in range(power):
        Z = _orth(A.T @ Q)
        Q = _orth(A @ Z)
    B = np.asarray((A.T @ Q).T)                       # l x n
    Ub, s, Vbt = np.linalg.svd(B, full_matrices=False)
    return Q @ Ub[:, :k], s[:k].copy(), Vbt[:k].T.copy()
