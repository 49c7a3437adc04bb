"""Comparison metrics between two rank-k truncated SVDs (FP64).

Singular vectors are defined only up to a joint sign per triplet and up to a
rotation inside a repeated singular value, so vectors are compared through
subspaces: the sine of the largest principal angle between the leading
j-dimensional subspaces, for the largest j at which the spectrum has a gap
(the quantity bounded by Wedin's sin-theta theorem).
"""
from __future__ import annotations

import numpy as np


def orth_err(X: np.ndarray) -> float:
    """||X^T X - I||_2."""
    k = X.shape[1]
    return float(np.linalg.norm(X.T @ X - np.eye(k), 2)) if k else 0.0


def _orthonormal(X: np.ndarray) -> np.ndarray:
    u, _, vt = np.linalg.svd(X, full_matrices=False)
    return u @ vt


def sin_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Sine of the largest principal angle between range(A) and range(B)
    (same number of columns), ||(I - Qa Qa^T) Qb||_2."""
    if A.shape[1] == 0:
        return 0.0
    Qa, Qb = _orthonormal(A), _orthonormal(B)
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


def gap_prefix(theta_hat: np.ndarray, k: int, delta: float) -> int:
    """Largest j <= k with theta_hat[j-1] - theta_hat[j] >= delta*theta_hat[0]
    (theta_hat: the full descending spectrum, so theta_hat[k] is known);
    0 if no such j."""
    th = np.asarray(theta_hat, dtype=np.float64)
    if th.size == 0 or th[0] <= 0:
        return 0
    ext = np.concatenate([th, [0.0]])
    for j in range(min(k, th.size), 0, -1):
        if ext[j - 1] - ext[j] >= delta * th[0]:
            return j
    return 0


def sigma_rel_err(s_test: np.ndarray, s_ref: np.ndarray, floor: float = 1e-8):
    """max_i |s_test_i - s_ref_i| / s_ref_i over s_ref_i >= floor*s_ref_1;
    entries below the floor are measured relative to s_ref_1."""
    s_test = np.asarray(s_test, np.float64)
    s_ref = np.asarray(s_ref, np.float64)
    if s_ref.size == 0:
        return 0.0
    top = max(float(s_ref[0]), 1e-300)
    den = np.where(s_ref >= floor * top, s_ref, top)
    return float(np.max(np.abs(s_test - s_ref) / den))


def compare(test, ref, theta_hat, delta: float):
    """Compare (U, s, V) triples; returns a dict with the singular-value error,
    the principal-angle sines at the gap prefix j* and at k, and the
    orthonormality errors of the test factors."""
    Ut, st, Vt = test
    Ur, sr, Vr = ref
    k = sr.size
    j = gap_prefix(theta_hat, k, delta)
    return dict(
        sigma_rel=sigma_rel_err(st, sr),
        jstar=j,
        angle_U=sin_angle(Ut[:, :j], Ur[:, :j]) if j else 0.0,
        angle_V=sin_angle(Vt[:, :j], Vr[:, :j]) if j else 0.0,
        angle_U_k=sin_angle(Ut, Ur),
        angle_V_k=sin_angle(Vt, Vr),
        orth_U=orth_err(Ut),
        orth_V=orth_err(Vt),
    )
