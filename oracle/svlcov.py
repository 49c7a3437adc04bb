"""O2 -- the paper's own update method, as written, on the CPU in FP64.

The factors are kept in the extended decomposition of Section 3.2,
``U' U'' diag(s) V''^T V'^T`` with U', V' tall and U'', V'' k x k (initially the
identity, U' and V' the singular vectors).  The augmented matrix is
orthogonalised in SV-LCOV form (Definition 1) by the SV-LCOV modified
Gram-Schmidt process (Algorithm 2, with the operations of Lemma 2); the drivers
follow Algorithms 3 (add columns), 4 (update weights) and 11 (add rows).

Readings taken where the text is silent or garbled:
  * the C used in the k x k factor updates of Algorithms 3, 4 and 11 is the
    normalised C returned by Algorithm 2, while K is assembled from the raw
    product U_k^T E; Equation (1) fixes this.
  * in Algorithm 4 the V' update multiplies by the inverse of V'' (the printed
    U'' is a typo: the V' update must be undone through V'').
  * Algorithm 2 divides by alpha, which is zero for a column already in the
    span of U_k and the previous columns; such a column is dropped (R_ii = 0,
    b_i = 0, c_i = 0) when alpha <= rtol * (largest column norm of B).
  * The k x k factors are inverted by an LU solve; when the new factor's
    condition number exceeds ``cond_reset`` it is folded into the tall factor
    and reset to the identity (the remedy named at the end of Section 3.2).

This module is slow on purpose (one sparse column operation at a time).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ALPHA_RTOL = 1e-7
COND_RESET = 1e8


def _csc(x):
    if sp.issparse(x):
        return sp.csc_matrix(x)
    if hasattr(x, "to_scipy"):
        return sp.csc_matrix(x.to_scipy())
    return sp.csc_matrix(np.asarray(x, dtype=np.float64))


def svlcov_qr(E, Uk, rtol: float = ALPHA_RTOL):
    """Algorithm 2 (SV-LCOV's QR process).

    E: m x s sparse, Uk: m x k orthonormal (given as a dense array).
    Returns (b, C, R, C_raw): b is the list of s sparse m-vectors of the
    normalised tuples, C (k x s) their dense parts, R (s x s) upper triangular
    and C_raw = Uk^T E before normalisation (Lemma 1: only rows of Uk at the
    nonzeros of each column are touched)."""
    Ecsc = _csc(E)
    m, s = Ecsc.shape
    b = [Ecsc[:, i] for i in range(s)]
    C = np.zeros((Uk.shape[1], s))
    for i in range(s):
        col = b[i]
        C[:, i] = Uk[col.indices].T @ col.data if col.nnz else 0.0
    C_raw = C.copy()
    scale = max((float(np.sqrt(bi.multiply(bi).sum())) for bi in b), default=0.0)
    R = np.zeros((s, s))
    for i in range(s):
        a2 = float(b[i].multiply(b[i]).sum()) - float(C[:, i] @ C[:, i])
        if a2 <= (rtol * scale) ** 2:
            # column i lies in span(Uk, previous columns): drop it
            b[i] = sp.csc_matrix((m, 1))
            C[:, i] = 0.0
            continue
        alpha = np.sqrt(a2)
        R[i, i] = alpha
        b[i] = b[i] / alpha
        C[:, i] /= alpha
        for j in range(i + 1, s):
            beta = float(b[i].multiply(b[j]).sum()) - float(C[:, i] @ C[:, j])
            R[i, j] = beta
            b[j] = b[j] - beta * b[i]
            C[:, j] -= beta * C[:, i]
    return b, C, R, C_raw


def _bmat(b, m):
    if not b:
        return sp.csc_matrix((m, 0))
    return sp.hstack(b, format="csc")


class ExtendedSVD:
    """The extended decomposition U' U'' diag(s) V''^T V'^T (Section 3.2)."""

    def __init__(self, U, s, V, rtol: float = ALPHA_RTOL,
                 cond_reset: float = COND_RESET):
        k = s.size
        self.Up = np.array(U, dtype=np.float64)
        self.Upp = np.eye(k)
        self.s = np.array(s, dtype=np.float64)
        self.Vp = np.array(V, dtype=np.float64)
        self.Vpp = np.eye(k)
        self.rtol = rtol
        self.cond_reset = cond_reset
        self.resets = 0

    @property
    def k(self):
        return self.s.size

    def factors(self):
        return self.Up @ self.Upp, self.s.copy(), self.Vp @ self.Vpp

    def query(self, i: int, side: str = "U"):
        """Query(i) of Theorem 1: one row of U (or V) in O(k^2)."""
        return (self.Up[i] @ self.Upp) if side == "U" else (self.Vp[i] @ self.Vpp)

    def _new_inner(self, old_inner, new_inner, tall):
        """Either keep the new inner factor (returning its inverse) or, if it
        is ill conditioned, fold it into the tall factor (reset)."""
        if np.linalg.cond(new_inner) > self.cond_reset:
            self.resets += 1
            return tall @ new_inner, np.eye(self.k), None
        return tall, new_inner, np.linalg.inv(new_inner)

    def add_cols(self, Ec):
        """Algorithm 3 with E_c = Ec (m x s)."""
        k = self.k
        Uk = self.Up @ self.Upp
        b, C, R, C_raw = svlcov_qr(Ec, Uk, self.rtol)
        s_ = R.shape[0]
        K = np.zeros((k + s_, k + s_))
        K[:k, :k] = np.diag(self.s)
        K[:k, k:] = C_raw
        K[k:, k:] = R
        F, th, Gt = np.linalg.svd(K)
        F, th, G = F[:, :k], th[:k], Gt[:k].T
        B = _bmat(b, Uk.shape[0])
        new_Upp = self.Upp @ (F[:k] - C @ F[k:])
        Up, Upp, inv = self._new_inner(self.Upp, new_Upp, self.Up)
        if inv is None:                                            # reset
            self.Up = Up + B @ F[k:]
        else:
            self.Up = Up + B @ F[k:] @ inv
        self.Upp = Upp
        self.s = th.copy()
        new_Vpp = self.Vpp @ G[:k]
        Vp, Vpp, inv = self._new_inner(self.Vpp, new_Vpp, self.Vp)
        app = G[k:] if inv is None else G[k:] @ inv
        self.Vp = np.vstack([Vp, app])
        self.Vpp = Vpp
        return np.linalg.svd(K, compute_uv=False)

    def add_rows(self, Er):
        """Algorithm 11 with E_r = Er (s x n)."""
        k = self.k
        Vk = self.Vp @ self.Vpp
        Er_T = _csc(Er).T
        b, C, R, C_raw = svlcov_qr(Er_T, Vk, self.rtol)
        s_ = R.shape[0]
        K = np.zeros((k + s_, k + s_))
        K[:k, :k] = np.diag(self.s)
        K[k:, :k] = C_raw.T                                        # E_r V_k
        K[k:, k:] = R.T
        F, th, Gt = np.linalg.svd(K)
        F, th, G = F[:, :k], th[:k], Gt[:k].T
        new_Upp = self.Upp @ F[:k]
        Up, Upp, inv = self._new_inner(self.Upp, new_Upp, self.Up)
        app = F[k:] if inv is None else F[k:] @ inv
        self.Up = np.vstack([Up, app])
        self.Upp = Upp
        self.s = th.copy()
        B = _bmat(b, Vk.shape[0])
        new_Vpp = self.Vpp @ (G[:k] - C @ G[k:])
        Vp, Vpp, inv = self._new_inner(self.Vpp, new_Vpp, self.Vp)
        self.Vp = Vp + (B @ G[k:] if inv is None else B @ G[k:] @ inv)
        self.Vpp = Vpp
        return np.linalg.svd(K, compute_uv=False)

    def update_weights(self, D, Em):
        """Algorithm 4 with D (m x s) and E_m (n x s)."""
        k = self.k
        Uk = self.Up @ self.Upp
        Vk = self.Vp @ self.Vpp
        bD, CD, RD, CD_raw = svlcov_qr(D, Uk, self.rtol)
        bE, CE, RE, CE_raw = svlcov_qr(Em, Vk, self.rtol)
        X = np.vstack([CD_raw, RD])
        Y = np.vstack([CE_raw, RE])
        K = X @ Y.T
        K[:k, :k] += np.diag(self.s)
        F, th, Gt = np.linalg.svd(K)
        F, th, G = F[:, :k], th[:k], Gt[:k].T
        BD = _bmat(bD, Uk.shape[0])
        BE = _bmat(bE, Vk.shape[0])
        new_Upp = self.Upp @ (F[:k] - CD @ F[k:])
        Up, Upp, inv = self._new_inner(self.Upp, new_Upp, self.Up)
        self.Up = Up + (BD @ F[k:] if inv is None else BD @ F[k:] @ inv)
        self.Upp = Upp
        self.s = th.copy()
        new_Vpp = self.Vpp @ (G[:k] - CE @ G[k:])
        Vp, Vpp, inv = self._new_inner(self.Vpp, new_Vpp, self.Vp)
        self.Vp = Vp + (BE @ G[k:] if inv is None else BE @ G[k:] @ inv)
        self.Vpp = Vpp
        return np.linalg.svd(K, compute_uv=False)

    def apply(self, update):
        """Apply ("rows", E) | ("cols", Ec_T) | ("weights", D_T, Em_T)."""
        kind = update[0]
        if kind == "rows":
            return self.add_rows(update[1].to_scipy() if hasattr(update[1], "to_scipy")
                                 else update[1])
        if kind == "cols":
            Ec_T = update[1].to_scipy() if hasattr(update[1], "to_scipy") else update[1]
            return self.add_cols(sp.csc_matrix(Ec_T).T)
        if kind == "weights":
            D_T, Em_T = (u.to_scipy() if hasattr(u, "to_scipy") else u
                         for u in update[1:3])
            return self.update_weights(sp.csc_matrix(D_T).T, sp.csc_matrix(Em_T).T)
        raise ValueError(kind)
