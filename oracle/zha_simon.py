"""O1 -- the Zha-Simon update scheme in plain FP64 (NumPy / SciPy / LAPACK).

An update replaces the maintained factors ``(U, s, V)`` of ``A~ = U diag(s) V^T``
by the rank-k truncated SVD of the updated matrix (Definition 2; Theorem 1):

  add rows      [A~ ; E_r]
  add columns   [A~ , E_c]
  update weights A~ + D E_m^T

(Section 2, the three update forms.)  The Zha-Simon scheme (Section 2.1) writes
the updated matrix exactly as a product through a small matrix K, using a QR
factorisation of the *augmented matrix* (I - U U^T) B (Section 2): for new
columns

  [A~ , E_c] = [U , Q] [[diag(s), U^T E_c], [0, R]] blkdiag(V, I)^T,

where (I - U U^T) E_c = Q R.  Because this is an identity, SVD_k of K rotated by
the outer factors *is* SVD_k of the updated matrix; the result has a plain
definition and O0 (``oracle.brute``) computes that definition directly on small
inputs.  Rows are the transpose of columns (Algorithm 11's K); the weight form
uses two QRs (Section 2.1, weight-update equation).

Rank deficiency (the paper leaves it open): the QR is Householder with column
pivoting (LAPACK dgeqp3) and a direction is kept iff |R_jj| > rtol * (largest
row norm of the update); dropped directions are removed from Q and R, so K is
(k + s) x (k + r).  Everything here is dense and slow by design.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

RANK_RTOL = 1e-10


def _dense(x):
    if sp.issparse(x):
        return x.toarray()
    if hasattr(x, "to_dense"):
        return x.to_dense()
    return np.asarray(x, dtype=np.float64)


def _sparse(x):
    if sp.issparse(x):
        return sp.csr_matrix(x)
    if hasattr(x, "to_scipy"):
        return x.to_scipy()
    return sp.csr_matrix(np.asarray(x, dtype=np.float64))


def augmented_qr(B, Ubasis, rtol: float = RANK_RTOL):
    """QR of the augmented matrix Z = (I - Ubasis Ubasis^T) B (Section 2).

    B: m x s (sparse or dense), Ubasis: m x k orthonormal.
    Returns (C, Q, R, r): C = Ubasis^T B (k x s), Q (m x r) orthonormal and
    orthogonal to Ubasis, R (r x s) with Z = Q R up to the dropped directions,
    and the numerical rank r."""
    Bs = _sparse(B)
    C = np.asarray((Bs.T @ Ubasis).T)                 # k x s
    Z = Bs.toarray() - Ubasis @ C                     # m x s, dense
    s = Z.shape[1]
    if s == 0:
        return C, np.zeros((Z.shape[0], 0)), np.zeros((0, 0)), 0
    Q, R, piv = sla.qr(Z, mode="economic", pivoting=True)
    scale = float(np.sqrt(np.max(np.asarray(Bs.multiply(Bs).sum(axis=0)))))
    d = np.abs(np.diag(R))
    r = int(np.sum(d > rtol * scale)) if scale > 0 else 0
    Q = Q[:, :r]
    Rp = np.zeros((r, s))
    Rp[:, piv] = R[:r, :]                              # undo the column pivoting
    return C, Q, Rp, r


def svd_k(K: np.ndarray, k: int):
    """SVD_k (Section 2): top-k singular triplets of K and its full spectrum."""
    F, th, Gt = np.linalg.svd(K, full_matrices=False)
    return F[:, :k], th[:k].copy(), Gt[:k].T.copy(), th


def add_rows(U, s, V, E, rtol: float = RANK_RTOL):
    """[A~ ; E] with E s x n.  K = [[diag(s), 0], [E V, R^T]] (the K of
    Algorithm 11) where (I - V V^T) E^T = Q R; U_new = [[U F[:k]], [F[k:]]],
    V_new = [V, Q] G."""
    k = s.size
    C, Q, R, r = augmented_qr(_sparse(E).T, V, rtol)    # C = V^T E^T  (k x s)
    sE = C.shape[1]
    K = np.zeros((k + sE, k + r))
    K[:k, :k] = np.diag(s)
    K[k:, :k] = C.T                                    # E V
    K[k:, k:] = R.T
    F, th, G, th_all = svd_k(K, k)
    U_new = np.vstack([U @ F[:k], F[k:]])
    V_new = np.hstack([V, Q]) @ G
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, rank=r, C=C, R=R)


def add_cols(U, s, V, Ec_T, rtol: float = RANK_RTOL):
    """[A~ , E_c] with E_c = Ec_T^T (m x s).  K = [[diag(s), U^T E_c], [0, R]]
    (Section 2.1; the K of Algorithm 3) where (I - U U^T) E_c = Q R;
    U_new = [U, Q] F, V_new = [[V G[:k]], [G[k:]]]."""
    k = s.size
    C, Q, R, r = augmented_qr(_sparse(Ec_T).T, U, rtol)  # C = U^T E_c (k x s)
    sE = C.shape[1]
    K = np.zeros((k + r, k + sE))
    K[:k, :k] = np.diag(s)
    K[:k, k:] = C
    K[k:, k:] = R
    F, th, G, th_all = svd_k(K, k)
    U_new = np.hstack([U, Q]) @ F
    V_new = np.vstack([V @ G[:k], G[k:]])
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, rank=r, C=C, R=R)


def update_weights(U, s, V, D_T, Em_T, rtol: float = RANK_RTOL):
    """A~ + D E_m^T with D = D_T^T (m x s), E_m = Em_T^T (n x s).
    K = [[diag(s), 0], [0, 0]] + [U^T D ; R_D] [V^T E_m ; R_E]^T
    (Section 2.1, weight-update equation; the K of Algorithm 4);
    U_new = [U, Q_D] F, V_new = [V, Q_E] G."""
    k = s.size
    CD, QD, RD, rD = augmented_qr(_sparse(D_T).T, U, rtol)
    CE, QE, RE, rE = augmented_qr(_sparse(Em_T).T, V, rtol)
    X = np.vstack([CD, RD])                            # (k + rD) x s
    Y = np.vstack([CE, RE])                            # (k + rE) x s
    K = X @ Y.T
    K[:k, :k] += np.diag(s)
    F, th, G, th_all = svd_k(K, k)
    U_new = np.hstack([U, QD]) @ F
    V_new = np.hstack([V, QE]) @ G
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, rank=(rD, rE))


def apply(U, s, V, update, rtol: float = RANK_RTOL):
    """Apply one update tuple ("rows", E) | ("cols", Ec_T) |
    ("weights", D_T, Em_T) as produced by ``synth.workloads``."""
    kind = update[0]
    if kind == "rows":
        return add_rows(U, s, V, update[1], rtol)
    if kind == "cols":
        return add_cols(U, s, V, update[1], rtol)
    if kind == "weights":
        return update_weights(U, s, V, update[1], update[2], rtol)
    raise ValueError(kind)
