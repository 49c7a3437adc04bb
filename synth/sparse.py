"""Seeded sparse-matrix and factor generators (NumPy PCG64 only).

Every function takes a ``numpy.random.Generator`` and returns plain arrays; no
function here projects, orthogonalises or decomposes an update.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """Canonical CSR: 0-based, int64 row_ptr, int32 column ids sorted and unique
    within each row, float64 values (explicit zeros allowed)."""
    rows: int
    cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr),
                             shape=(self.rows, self.cols))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return CSR(m.shape[0], m.shape[1], m.indptr.astype(np.int64),
                   m.indices.astype(np.int32), m.data.astype(np.float64))

    @staticmethod
    def from_dense(a) -> "CSR":
        a = np.asarray(a, dtype=np.float64)
        return CSR.from_scipy(sp.csr_matrix(a))

    def row_block(self, r0: int, r1: int) -> "CSR":
        p0, p1 = int(self.row_ptr[r0]), int(self.row_ptr[r1])
        return CSR(r1 - r0, self.cols, self.row_ptr[r0:r1 + 1] - p0,
                   self.col_idx[p0:p1].copy(), self.val[p0:p1].copy())


def _coo_to_csr(r, c, v, shape) -> CSR:
    m = sp.coo_matrix((v, (r, c)), shape=shape).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR.from_scipy(m)


def bernoulli_uniform(m: int, n: int, density: float, rng) -> CSR:
    """Each entry nonzero independently with probability ``density``; values
    ``1 - U[0,1)`` in (0, 1]."""
    total = m * n
    cnt = rng.binomial(total, density)
    # sample distinct linear positions without building a dense mask
    pos = np.unique(rng.integers(0, total, size=int(cnt * 1.02) + 16))
    while pos.size < cnt:
        extra = rng.integers(0, total, size=cnt - pos.size + 16)
        pos = np.unique(np.concatenate([pos, extra]))
    pos = rng.permutation(pos)[:cnt]
    r, c = np.divmod(pos, n)
    v = 1.0 - rng.random(cnt)
    return _coo_to_csr(r, c, v, (m, n))


def chung_lu_weights(N: int, gamma: float, avg_deg: float) -> np.ndarray:
    """Expected degrees w_i = c (i + i0)^(-1/(gamma-1)); i0 is raised by
    bisection until max w <= sqrt(sum w) so that w_i w_j / sum w <= 1."""
    a = 1.0 / (gamma - 1.0)
    idx = np.arange(N, dtype=np.float64)

    def weights(i0):
        w = (idx + i0) ** (-a)
        return w * (avg_deg * N / w.sum())

    lo, hi = 0.0, float(N)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        w = weights(mid)
        if w.max() <= np.sqrt(w.sum()):
            hi = mid
        else:
            lo = mid
    return weights(hi)


def chung_lu_graph(N: int, gamma: float, avg_deg: float, rng,
                   values: str = "unit") -> CSR:
    """Undirected power-law graph, symmetric CSR without self loops.

    Edge-sampling form of the Chung-Lu model: the number of endpoint draws is
    Poisson(sum w / 2), each endpoint drawn with probability proportional to
    w; self loops are removed and repeated pairs merged.  Node ids are then
    randomly permuted so that hubs are spread over the id range.
    ``values``: "unit" (all ones) or "lognormal" (LogNormal(0, 1), one draw
    per undirected edge, mirrored)."""
    w = chung_lu_weights(N, gamma, avg_deg)
    p = w / w.sum()
    M = rng.poisson(w.sum() / 2.0)
    i = rng.choice(N, size=M, p=p)
    j = rng.choice(N, size=M, p=p)
    keep = i != j
    i, j = i[keep], j[keep]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo.astype(np.int64) * N + hi)
    lo, hi = np.divmod(key, N)
    perm = rng.permutation(N)
    lo, hi = perm[lo], perm[hi]
    if values == "unit":
        v = np.ones(lo.size)
    elif values == "lognormal":
        v = rng.lognormal(0.0, 1.0, size=lo.size)
    else:
        raise ValueError(values)
    r = np.concatenate([lo, hi])
    c = np.concatenate([hi, lo])
    return _coo_to_csr(r, c, np.concatenate([v, v]), (N, N))


def zipf_ratings(users: int, items: int, nnz: int, zipf_a: float, rng,
                 pmf=(0.1, 0.1, 0.2, 0.3, 0.3)) -> CSR:
    """User-item ratings: user uniform per rating, item by truncated Zipf over
    popularity ranks with a random rank->id permutation, repeated
    (user, item) pairs redrawn, integer values 1..5 with the given pmf."""
    ranks = np.arange(1, items + 1, dtype=np.float64)
    pz = ranks ** (-zipf_a)
    pz /= pz.sum()
    item_of_rank = rng.permutation(items)
    keys = np.empty(0, dtype=np.int64)
    need = nnz
    while need > 0:
        u = rng.integers(0, users, size=int(need * 1.1) + 64)
        it = item_of_rank[rng.choice(items, size=u.size, p=pz)]
        keys = np.unique(np.concatenate([keys, u.astype(np.int64) * items + it]))
        need = nnz - keys.size
    keys = rng.permutation(keys)[:nnz]
    r, c = np.divmod(keys, items)
    v = rng.choice(np.arange(1, 6, dtype=np.float64), size=nnz, p=np.asarray(pmf))
    return _coo_to_csr(r, c, v, (users, items))


def lognormal_values(n: int, rng) -> np.ndarray:
    return rng.lognormal(0.0, 1.0, size=n)


def _qr_signfixed(x: np.ndarray) -> np.ndarray:
    q, r = np.linalg.qr(x)
    d = np.diag(r)
    return q * np.sign(np.where(d == 0, 1.0, d))


def _orth_tall(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of a tall matrix: two Cholesky-QR
    passes (fast, accurate to rounding while cond(Y) < ~1e6), else a
    Householder QR."""
    Q = Y
    for _ in range(2):
        G = Q.T @ Q
        try:
            R = np.linalg.cholesky(G).T
        except np.linalg.LinAlgError:
            return np.linalg.qr(Y)[0]
        d = np.abs(np.diag(R))
        if d.min() <= 1e-6 * d.max():
            return np.linalg.qr(Y)[0]
        Q = Q @ np.linalg.inv(R)
    return Q


def random_orthonormal(m: int, k: int, rng) -> np.ndarray:
    """m x k with orthonormal columns: Q of a Gaussian matrix, signs fixed so
    that diag(R) > 0."""
    return _qr_signfixed(rng.standard_normal((m, k)))


def synthetic_factors(m: int, n: int, k: int, rng, scale: float = 100.0):
    """Synthetic truncated SVD: random orthonormal U, V and
    sigma_j = scale * j^(-1/2), j = 1..k."""
    U = random_orthonormal(m, k, rng)
    V = random_orthonormal(n, k, rng)
    s = scale * np.arange(1, k + 1, dtype=np.float64) ** -0.5
    return U, s, V


def randomized_init(A: CSR, k: int, rng, oversample: int = 16, power: int = 4):
    """Rank-k starting factors of a sparse matrix by a randomized range finder
    with ``power`` subspace iterations.  The result only has to be an exact
    orthonormal triple (U, s, V); how close it is to the true truncated SVD
    does not enter any comparison, which is always made against the matrix
    ``U diag(s) V^T`` that the triple represents."""
    S = A.to_scipy()
    m, n = S.shape
    l = min(k + oversample, m, n)
    Y = S @ rng.standard_normal((n, l))
    Q = _orth_tall(Y)
    for _ in range(power):
        Z = _orth_tall(S.T @ Q)
        Q = _orth_tall(S @ Z)
    Bt = S.T @ Q                         # n x l, B = Q^T S = Bt^T
    Qb = _orth_tall(Bt)                  # Bt = Qb Rb with Rb = Qb^T Bt
    Ub, s, Vst = np.linalg.svd((Qb.T @ Bt).T)   # B = Rb^T Qb^T = Ub diag(s) (Qb Vs)^T
    U = Q @ Ub[:, :k]
    V = Qb @ Vst[:k].T
    # re-orthonormalise in FP64 so that U^T U = V^T V = I to rounding (both
    # are orthonormal up to rounding already, so Cholesky-QR is exact enough)
    U = _orth_tall(U)
    V = _orth_tall(V)
    return np.ascontiguousarray(U), s[:k].copy(), np.ascontiguousarray(V)
