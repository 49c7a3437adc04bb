"""Seeded update streams with the shapes of the paper's workloads.

Each generator returns a dict with the starting factors ``U, s, V`` (FP64,
orthonormal columns) and a list of updates.  An update is one of
``("rows", E)``, ``("cols", Ec_T)`` or ``("weights", D_T, Em_T)`` where every
matrix is a ``CSR`` given row-wise in the orientation the update calls take:
``E`` is s x n (new rows), ``Ec_T`` is s x m (the transpose of the new
columns), ``D_T`` is s x m and ``Em_T`` is s x n for ``A + D Em^T``.

Master seed 240109703; one ``SeedSequence`` child per workload, spawned again
into the initial matrix, each step and (for the stream) the arrivals.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .sparse import (CSR, bernoulli_uniform, chung_lu_graph, chung_lu_weights,
                     random_orthonormal, randomized_init, synthetic_factors,
                     zipf_ratings)

MASTER_SEED = 240109703


def seed_children(config: int, count: int):
    """``count`` independent generators for workload ``config`` (1-based)."""
    root = np.random.SeedSequence(MASTER_SEED).spawn(5)[config - 1]
    return [np.random.Generator(np.random.PCG64(c)) for c in root.spawn(count)]


def _exact_topk(A: CSR, k: int):
    Ud, sd, Vt = np.linalg.svd(A.to_dense(), full_matrices=False)
    return Ud[:, :k].copy(), sd[:k].copy(), Vt[:k].T.copy()


def config1_rows(m: int = 2000, n: int = 1000, density: float = 0.005,
                 k: int = 16, steps: int = 10, s: int = 100):
    """Plain method, FP64: Bernoulli sparse A (values in (0,1]), exact top-k
    start, then ``steps`` row appends of ``s`` rows at the same density."""
    rngs = seed_children(1, steps + 1)
    A = bernoulli_uniform(m, n, density, rngs[0])
    U, sig, V = _exact_topk(A, k)
    ups = [("rows", bernoulli_uniform(s, n, density, rngs[1 + t]))
           for t in range(steps)]
    return dict(name="bernoulli-2000x1000-k16", A=A, U=U, s=sig, V=V, k=k,
                updates=ups)


def config2_graph(k: int = 64, n_init: int = 90000, step_nodes: int = 1000,
                  steps: int = 10, avg_deg: float = 20.0, gamma: float = 2.1,
                  power: int = 4):
    """Graph adjacency: Chung-Lu graph on n_init + steps*step_nodes nodes;
    start from the induced subgraph on the first n_init nodes; each step
    appends step_nodes nodes as ``add_cols(A[old, new])`` followed by
    ``add_rows(A[new, old + new])``."""
    N = n_init + steps * step_nodes
    rngs = seed_children(2, 2)
    G = chung_lu_graph(N, gamma, avg_deg, rngs[0]).to_scipy().tocsr()
    A0 = CSR.from_scipy(G[:n_init, :n_init])
    U, sig, V = randomized_init(A0, k, rngs[1], power=power)
    ups = []
    for t in range(steps):
        o = n_init + t * step_nodes
        new = slice(o, o + step_nodes)
        ups.append(("cols", CSR.from_scipy(G[new, :o])))
        ups.append(("rows", CSR.from_scipy(G[new, :o + step_nodes])))
    return dict(name=f"chung-lu-{N}-k{k}", A0=A0, U=U, s=sig, V=V, k=k,
                updates=ups, nnz_total=G.nnz)


def config2_initial_matrix(n_init: int = 90000, step_nodes: int = 1000, steps: int = 10,
                           avg_deg: float = 20.0, gamma: float = 2.1) -> CSR:
    """The starting matrix of ``config2_graph`` (same seeds and sizes): the
    adjacency of the induced subgraph on the first n_init nodes, without the
    starting factors."""
    N = n_init + steps * step_nodes
    rngs = seed_children(2, 2)
    G = chung_lu_graph(N, gamma, avg_deg, rngs[0]).to_scipy().tocsr()
    return CSR.from_scipy(G[:n_init, :n_init])


def config3_ratings(users: int = 500000, items: int = 50000,
                    nnz: int = 10_000_000, init_users: int = 400000,
                    k: int = 128, steps: int = 20, s: int = 5000,
                    zipf_a: float = 1.1, power: int = 2):
    """User-item ratings: start on the first init_users users, then
    ``steps`` appends of ``s`` user rows."""
    rngs = seed_children(3, 2)
    R = zipf_ratings(users, items, nnz, zipf_a, rngs[0]).to_scipy().tocsr()
    A0 = CSR.from_scipy(R[:init_users])
    U, sig, V = randomized_init(A0, k, rngs[1], power=power)
    ups = [("rows", CSR.from_scipy(R[init_users + t * s:init_users + (t + 1) * s]))
           for t in range(steps) if init_users + (t + 1) * s <= users]
    return dict(name=f"ratings-{users}x{items}-k{k}", A0=A0, U=U, s=sig, V=V,
                k=k, updates=ups)


def config4_weights(N: int = 1_000_000, avg_deg: float = 20.0, k: int = 64,
                    steps: int = 10, s: int = 32, perturbed: int = 50000,
                    added: int = 10000, gamma: float = 2.1, power: int = 1):
    """Weight change: LogNormal-weighted Chung-Lu graph; each step is one
    rank-s update ``A + D Em^T`` with ``D = I[:, R]`` for s rows R drawn with
    probability proportional to degree, and ``Em^T`` holding ``perturbed``
    re-weighted existing entries of those rows (new LogNormal minus old) and
    ``added`` new entries (columns by Chung-Lu weight, LogNormal values).
    When the drawn rows hold fewer than ``perturbed`` entries, all of them
    are re-weighted."""
    rngs = seed_children(4, steps + 2)
    G = chung_lu_graph(N, gamma, avg_deg, rngs[0], values="lognormal")
    U, sig, V = randomized_init(G, k, rngs[1], power=power)
    Gs = G.to_scipy().tocsr()
    deg = np.diff(Gs.indptr).astype(np.float64)
    w = chung_lu_weights(N, gamma, avg_deg)
    ups = []
    for t in range(steps):
        rng = rngs[2 + t]
        # s rows drawn with probability proportional to degree; up to 64 draws
        # are tried for a set holding ``perturbed`` existing entries and the
        # draw with the most entries is kept (a degree-biased draw of 32 rows
        # of a 1M-node graph rarely holds 50k entries)
        best = None
        for _ in range(64):
            R = rng.choice(N, size=s, replace=False, p=deg / deg.sum())
            if best is None or deg[R].sum() > deg[best].sum():
                best = R
            if deg[R].sum() >= perturbed:
                break
        R = best
        rows, cols, vals = [], [], []
        sub = Gs[R]
        nnz_sub = sub.nnz
        pick = rng.choice(nnz_sub, size=min(perturbed, nnz_sub), replace=False)
        coo = sub.tocoo()
        newv = rng.lognormal(0.0, 1.0, size=pick.size)
        rows.append(coo.row[pick]); cols.append(coo.col[pick])
        vals.append(newv - coo.data[pick])
        r_add = rng.integers(0, s, size=added)
        c_add = rng.choice(N, size=added, p=w / w.sum())
        rows.append(r_add); cols.append(c_add)
        vals.append(rng.lognormal(0.0, 1.0, size=added))
        Em_T = sp.coo_matrix((np.concatenate(vals),
                              (np.concatenate(rows), np.concatenate(cols))),
                             shape=(s, N)).tocsr()
        Em_T.sum_duplicates()
        D_T = sp.csr_matrix((np.ones(s), (np.arange(s), R)), shape=(s, N))
        ups.append(("weights", CSR.from_scipy(D_T), CSR.from_scipy(Em_T)))
    return dict(name=f"weights-{N}-k{k}", A=G, U=U, s=sig, V=V, k=k,
                updates=ups)


def config4_weights_r2(N: int = 1_000_000, avg_deg: float = 20.0, k: int = 64,
                       steps: int = 10, s: int = 32, perturbed: int = 50000,
                       added: int = 10000, gamma: float = 2.1, power: int = 1):
    """The weight change spread over the whole graph (the secondary reading
    of the weight workload): ``perturbed`` existing entries drawn uniformly
    (new LogNormal minus old) and ``added`` new entries (both endpoints by
    Chung-Lu weight, LogNormal values), applied as consecutive rank-s updates
    ``A + D Em^T`` with ``D = I[:, R_c]`` over the touched rows in ascending
    chunks of s.  The same graph and starting factors as ``config4_weights``;
    only the first ``steps`` chunks are returned, with the total count."""
    rngs = seed_children(4, 2)
    G = chung_lu_graph(N, gamma, avg_deg, rngs[0], values="lognormal")
    U, sig, V = randomized_init(G, k, rngs[1], power=power)
    Gs = G.to_scipy().tocsr()
    coo = Gs.tocoo()
    w = chung_lu_weights(N, gamma, avg_deg)
    rng = seed_children(4, 64)[63]
    pick = rng.choice(coo.nnz, size=min(perturbed, coo.nnz), replace=False)
    r_add = rng.choice(N, size=added, p=w / w.sum())
    c_add = rng.choice(N, size=added, p=w / w.sum())
    rows = np.concatenate([coo.row[pick], r_add])
    cols = np.concatenate([coo.col[pick], c_add])
    vals = np.concatenate([rng.lognormal(0.0, 1.0, size=pick.size) - coo.data[pick],
                           rng.lognormal(0.0, 1.0, size=added)])
    Delta = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    Delta.sum_duplicates()
    touched = np.flatnonzero(np.diff(Delta.indptr) > 0)
    total = (touched.size + s - 1) // s
    ups = []
    for c in range(min(steps, total)):
        R = touched[c * s:(c + 1) * s]
        D_T = sp.csr_matrix((np.ones(R.size), (np.arange(R.size), R)), shape=(R.size, N))
        ups.append(("weights", CSR.from_scipy(D_T), CSR.from_scipy(Delta[R])))
    return dict(name=f"weights-r2-{N}-k{k}", A=G, U=U, s=sig, V=V, k=k, updates=ups,
                total_updates=total, touched_rows=int(touched.size))


def config5_stream(n_mat: int = 512, requests: int = 4096, seed_offset: int = 0,
                   m_range=(5000, 200000), n_range=(1000, 50000),
                   dens_range=(5e-4, 1e-2), ks=(16, 32, 64),
                   s_range=(10, 2000), rate: float = 1000.0):
    """Streaming batch: descriptors of independent matrices with synthetic
    factors (drawn lazily by ``materialise``) and Poisson-arriving row-append
    requests.  Returns (mats, reqs); mats[i] = dict(m, n, k, density, seed),
    reqs[j] = dict(t, mat, s, seed)."""
    rngs = seed_children(5, 3)
    r = rngs[0]
    mats = [dict(m=int(r.integers(m_range[0], m_range[1] + 1)),
                 n=int(r.integers(n_range[0], n_range[1] + 1)),
                 k=int(r.choice(ks)),
                 density=float(r.uniform(*dens_range)),
                 seed=int(r.integers(0, 2**62)))
            for _ in range(n_mat)]
    ra = rngs[1]
    t = np.cumsum(ra.exponential(1.0 / rate, size=requests))
    reqs = [dict(t=float(t[j]), mat=int(ra.integers(0, n_mat)),
                 s=int(ra.integers(s_range[0], s_range[1] + 1)),
                 seed=int(ra.integers(0, 2**62)))
            for j in range(requests)]
    return mats, reqs


def materialise_matrix(desc):
    rng = np.random.Generator(np.random.PCG64(desc["seed"]))
    return synthetic_factors(desc["m"], desc["n"], desc["k"], rng)


def materialise_request(desc, mat):
    rng = np.random.Generator(np.random.PCG64(desc["seed"]))
    return bernoulli_uniform(desc["s"], mat["n"], mat["density"], rng)


def small_case(rng, m: int, n: int, k: int, s: int, kind: str = "rows",
               density: float = 0.1, dup_rows: int = 0, empty_rows: int = 0,
               in_span_rows: int = 0, scale: float = 10.0):
    """Small random case for parity tests: synthetic factors plus one update
    of the given kind with optional duplicate, empty and in-span rows (the
    last ones are rows of ``a V^T`` restricted to a random sparse
    combination, so they lie in the span of V; only meaningful for tiny n).
    """
    U, sig, V = synthetic_factors(m, n, k, rng, scale=scale)
    width = {"rows": n, "cols": m}.get(kind)

    def upd(width):
        E = bernoulli_uniform(s, width, density, rng).to_dense()
        for i in range(min(dup_rows, s - 1)):
            E[s - 1 - i] = E[i]
        for i in range(min(empty_rows, s)):
            E[(s // 2 + i) % s] = 0.0
        return E

    if kind in ("rows", "cols"):
        E = upd(width)
        if in_span_rows:
            basis = V if kind == "rows" else U
            for i in range(min(in_span_rows, s)):
                E[i] = basis @ rng.standard_normal(k)
        return dict(U=U, s=sig, V=V, k=k, kind=kind, E=CSR.from_dense(E))
    if kind == "weights":
        D = upd(m)
        Em = upd(n)
        return dict(U=U, s=sig, V=V, k=k, kind=kind, D_T=CSR.from_dense(D),
                    Em_T=CSR.from_dense(Em))
    raise ValueError(kind)
