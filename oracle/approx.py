"""O3 -- the -GKL and -RPI variants in plain FP64 (test infrastructure only).

The variants (the paper's appendix on approximating the augmented space, and
the paragraph on the proposed variants in Section 4) replace the QR of the
augmented matrix Z = (I - U U^T) B by an l-dimensional orthonormal basis Q of
a subspace of range(Z), together with P = Z^T Q, so that Z is approximated by
Q P^T.  K then has k + l columns on the side that Q extends instead of k + s,
and the rest of the update (SVD_k of K, the rotation of the factors) is the
Zha-Simon scheme of Section 2.1 with R replaced by P^T.

  GKL   the Golub-Kahan-Lanczos process (the appendix's GKL algorithm) from a
        unit start vector p_1 in R^s, with every new p orthogonalised against
        all previous ones; Q = [q_1 .. q_l], P = P_{l+1} H^T with
        H = diag(alpha) + superdiag(beta) (l x (l+1)).
  RPI   random power iteration (the appendix's RPI algorithm) from an s x l
        start P_0 with t rounds of P <- QR(P), Q <- QR(Z P), P <- Z^T Q.

Readings where the paper is silent (listed in the design notes):
  * l is clamped to s (the augmented space has at most s dimensions).
  * GKL stops at a breakdown: when alpha_i or beta_i falls to
    rtol * (largest row norm of the update) or below, that coefficient is set
    to zero and every later q, p, alpha, beta is zero.
  * RPI's QR of Z P keeps a direction iff its pivot exceeds the same threshold
    (Householder with column pivoting); the QR of P keeps a direction iff its
    pivot exceeds rtol times the largest; dropped directions leave zero
    columns.
  * The start vectors are inputs: GKL's p_1 (normalised here; all ones when
    none is given) and RPI's P_0 are drawn by the caller.

Everything is dense and slow by design; Z is formed explicitly.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from oracle.zha_simon import RANK_RTOL, _sparse, svd_k


def augmented(B, Ubasis):
    """Z = (I - Ubasis Ubasis^T) B (dense m x s) and C = Ubasis^T B (k x s);
    also the largest column norm of B (the breakdown scale)."""
    Bs = _sparse(B)
    C = np.asarray((Bs.T @ Ubasis).T)
    Z = Bs.toarray() - Ubasis @ C
    scale = float(np.sqrt(np.max(np.asarray(Bs.multiply(Bs).sum(axis=0))))) if Bs.shape[1] else 0.0
    return Z, C, scale


def gkl(Z, l, p1=None, scale=None, rtol=RANK_RTOL):
    """Golub-Kahan-Lanczos on Z (m x s) for l steps from p_1.

    Returns Q (m x l), P = P_{l+1} H^T (s x l), the coefficients Y (s x l)
    with Q = Z Y, and alpha, beta (l each)."""
    m, s = Z.shape
    l = min(l, s)
    if scale is None:
        scale = float(np.max(np.linalg.norm(Z, axis=0))) if s else 0.0
    thr = rtol * scale
    p = np.ones(s) if p1 is None else np.asarray(p1, dtype=np.float64).copy()
    p = p / np.linalg.norm(p)
    Pv = np.zeros((s, l + 1))
    Pv[:, 0] = p
    Q = np.zeros((m, l))
    Y = np.zeros((s, l))
    alpha = np.zeros(l)
    beta = np.zeros(l)
    q_prev = np.zeros(m)
    y_prev = np.zeros(s)
    b_prev = 0.0
    for i in range(l):
        # q_i = Z p_i - beta_{i-1} q_{i-1}, kept with its coefficients in R^s
        q = Z @ Pv[:, i] - b_prev * q_prev
        y = Pv[:, i] - b_prev * y_prev
        a = float(np.linalg.norm(q))
        if a <= thr:
            break
        q, y = q / a, y / a
        alpha[i] = a
        Q[:, i], Y[:, i] = q, y
        # p_{i+1} = Z^T q_i - alpha_i p_i, orthogonalised against p_1 .. p_i
        pn = Z.T @ q - a * Pv[:, i]
        for _ in range(2):
            pn = pn - Pv[:, : i + 1] @ (Pv[:, : i + 1].T @ pn)
        b = float(np.linalg.norm(pn))
        if b <= thr:
            break
        beta[i] = b
        Pv[:, i + 1] = pn / b
        q_prev, y_prev, b_prev = q, y, b
    H = np.zeros((l, l + 1))
    H[np.arange(l), np.arange(l)] = alpha
    H[np.arange(l), np.arange(1, l + 1)] = beta
    P = Pv @ H.T
    return Q, P, Y, alpha, beta


def rpi(Z, l, t, P0, scale=None, rtol=RANK_RTOL):
    """Random power iteration on Z (m x s): t rounds of P <- QR(P),
    Q <- QR(Z P) (pivoted, dropping directions at or below the threshold),
    P <- Z^T Q.  P0 is s x l.  Returns Q (m x l), P (s x l), Y (s x l) with
    Q = Z Y, and the kept rank."""
    m, s = Z.shape
    l = min(l, s)
    if scale is None:
        scale = float(np.max(np.linalg.norm(Z, axis=0))) if s else 0.0
    thr = rtol * scale
    P = np.asarray(P0, dtype=np.float64)[:, :l].copy()
    Q = np.zeros((m, l))
    Y = np.zeros((s, l))
    r = 0
    for _ in range(t):
        # P <- QR(P); a direction whose pivot falls to rtol times the largest
        # one is dropped (zero column), so a rank-deficient Z^T Q stays so
        Qp, Rp, _pv = sla.qr(P, mode="economic", pivoting=True)
        dp = np.abs(np.diag(Rp))
        rp = int(np.sum(dp > rtol * dp.max())) if dp.size and dp.max() > 0 else 0
        P = np.zeros_like(P)
        P[:, :rp] = Qp[:, :rp]
        X = Z @ P
        Qf, R, piv = sla.qr(X, mode="economic", pivoting=True)
        d = np.abs(np.diag(R))
        r = int(np.sum(d > thr))
        # Q = X[:, piv[:r]] R[:r,:r]^{-1}: the coefficients follow from P
        Q = np.zeros((m, l))
        Y = np.zeros((s, l))
        Q[:, :r] = Qf[:, :r]
        Rinv = sla.solve_triangular(R[:r, :r], np.eye(r))
        Y[:, :r] = P[:, piv[:r]] @ Rinv
        P = Z.T @ Q
    return Q, P, Y, r


def _basis(Z, scale, method, l, t, start, rtol):
    if method == "gkl":
        Q, P, Y, _, _ = gkl(Z, l, start, scale, rtol)
    elif method == "rpi":
        Q, P, Y, _ = rpi(Z, l, t, start, scale, rtol)
    else:
        raise ValueError(method)
    return Q, P, Y


def add_rows(U, s, V, E, method="gkl", l=10, t=3, start=None, rtol=RANK_RTOL):
    """[A~ ; E] with E s x n.  Z = (I - V V^T) E^T approximated by Q P^T;
    K = [[diag(s), 0], [E V, P]] ((k+s) x (k+l)); U_new = [[U F[:k]], [F[k:]]],
    V_new = [V, Q] G."""
    k = s.size
    Z, C, scale = augmented(_sparse(E).T, V)
    Q, P, Y = _basis(Z, scale, method, l, t, start, rtol)
    sE, lq = C.shape[1], Q.shape[1]
    K = np.zeros((k + sE, k + lq))
    K[:k, :k] = np.diag(s)
    K[k:, :k] = C.T
    K[k:, k:] = P
    F, th, G, th_all = svd_k(K, k)
    U_new = np.vstack([U @ F[:k], F[k:]])
    V_new = np.hstack([V, Q]) @ G
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, Q=Q, P=P, Y=Y, C=C)


def add_cols(U, s, V, Ec_T, method="gkl", l=10, t=3, start=None, rtol=RANK_RTOL):
    """[A~ , E_c] with E_c = Ec_T^T (m x s): the appendix's column form,
    K = [[diag(s), U^T E_c], [0, P^T]] ((k+l) x (k+s)); U_new = [U, Q] F,
    V_new = [[V G[:k]], [G[k:]]]."""
    k = s.size
    Z, C, scale = augmented(_sparse(Ec_T).T, U)
    Q, P, Y = _basis(Z, scale, method, l, t, start, rtol)
    sE, lq = C.shape[1], Q.shape[1]
    K = np.zeros((k + lq, k + sE))
    K[:k, :k] = np.diag(s)
    K[:k, k:] = C
    K[k:, k:] = P.T
    F, th, G, th_all = svd_k(K, k)
    U_new = np.hstack([U, Q]) @ F
    V_new = np.vstack([V @ G[:k], G[k:]])
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, Q=Q, P=P, Y=Y, C=C)


def update_weights(U, s, V, D_T, Em_T, method="gkl", l=10, t=3, start=None, rtol=RANK_RTOL):
    """A~ + D E_m^T: the appendix's weight form, one basis per side,
    K = [[diag(s), 0], [0, 0]] + [U^T D ; P_D^T] [V^T E_m ; P_E^T]^T;
    start is a pair (start for D, start for E_m)."""
    k = s.size
    st_D, st_E = (None, None) if start is None else start
    ZD, CD, scD = augmented(_sparse(D_T).T, U)
    ZE, CE, scE = augmented(_sparse(Em_T).T, V)
    QD, PD, _ = _basis(ZD, scD, method, l, t, st_D, rtol)
    QE, PE, _ = _basis(ZE, scE, method, l, t, st_E, rtol)
    X = np.vstack([CD, PD.T])
    Yb = np.vstack([CE, PE.T])
    K = X @ Yb.T
    K[:k, :k] += np.diag(s)
    F, th, G, th_all = svd_k(K, k)
    U_new = np.hstack([U, QD]) @ F
    V_new = np.hstack([V, QE]) @ G
    return U_new, th, V_new, dict(K=K, theta_hat=th_all, QD=QD, QE=QE)
