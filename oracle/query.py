"""O4 -- queries and scores on maintained factors (test infrastructure only).

Theorem 1's Query(i) returns row i of U (or of V) with Sigma; the paper's
link-prediction and collaborative-filtering workloads (Section 5, the task
descriptions) score a pair (i, j) by U[i]^T Sigma V[j], and for an undirected
graph take the larger of the two directions.  Plain FP64 on dense factors.
"""
from __future__ import annotations

import numpy as np


def query_rows(X: np.ndarray, idx) -> np.ndarray:
    """Rows idx of the factor X (Query(i) for every i in idx)."""
    return np.asarray(X, dtype=np.float64)[np.asarray(idx, dtype=np.int64)]


def score_pairs(U, s, V, i, j, both: bool = False) -> np.ndarray:
    """U[i]^T diag(s) V[j] for every pair; with both, the larger of that and
    U[j]^T diag(s) V[i] (the undirected link-prediction score)."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    out = np.einsum("pk,k,pk->p", U[i], s, V[j])
    if both:
        out = np.maximum(out, np.einsum("pk,k,pk->p", U[j], s, V[i]))
    return out
