"""Pins of O3, the -GKL and -RPI variants (the appendix on approximating the
augmented space), against facts fixed by the mathematics (CPU only).

  Krylov space   span(Q) of GKL equals the Krylov space
                 span{Z p1, (Z Z^T) Z p1, ...} built independently
  power space    span(Q) of RPI equals range(Z (Z^T Z)^(t-1) P0)
  P = Z^T Q      the returned P (P_{l+1} H^T for GKL) equals Z^T Q formed
                 directly; Q is orthonormal and orthogonal to the old basis
  full space     with l = s the variants reproduce the exact update (the dense
                 SVD of the updated matrix, Definition 2)
  projection     with l < s the result is the dense SVD_k of the updated
                 matrix with the new block projected onto span[old basis, Q]
  breakdown      a rank-deficient Z stops GKL early and still gives the
                 exact update once the Krylov space holds range(Z)
"""
import numpy as np
import pytest

from oracle import approx, brute, metrics
from synth import small_case


def _upd(c):
    if c["kind"] == "weights":
        return ("weights", c["D_T"], c["Em_T"])
    return (c["kind"], c["E"])


def _case(seed, m=40, n=30, k=4, s=12, kind="rows", dens=0.2):
    rng = np.random.default_rng(seed)
    return small_case(rng, m, n, k, s, kind=kind, density=dens), rng


def _span_angle(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    return metrics.sin_angle(qa, qb)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gkl_spans_krylov_space(seed):
    c, rng = _case(seed)
    Z, C, scale = approx.augmented(c["E"].to_dense().T, c["V"])
    p1 = rng.standard_normal(Z.shape[1])
    l = 4
    Q, P, Y, alpha, beta = approx.gkl(Z, l, p1, scale)
    # Krylov basis by repeated products, orthonormalised after every step
    v = Z @ (p1 / np.linalg.norm(p1))
    cols = []
    for _ in range(l):
        for w in cols:
            v = v - w * (w @ v)
        v = v / np.linalg.norm(v)
        cols.append(v)
        v = Z @ (Z.T @ v)
    Kr = np.stack(cols, axis=1)
    assert _span_angle(Q, Kr) <= 1e-8
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-12
    assert np.abs(c["V"].T @ Q).max() <= 1e-12
    assert np.abs(P - Z.T @ Q).max() <= 1e-12 * np.abs(Z).max()
    assert np.abs(Z @ Y - Q).max() <= 1e-12
    assert np.all(alpha > 0) and np.all(beta > 0)


@pytest.mark.parametrize("t", [1, 2, 3])
def test_rpi_spans_power_space(t):
    c, rng = _case(10 + t)
    Z, C, scale = approx.augmented(c["E"].to_dense().T, c["V"])
    l = 5
    P0 = rng.standard_normal((Z.shape[1], l))
    Q, P, Y, r = approx.rpi(Z, l, t, P0, scale)
    X = Z @ P0
    for _ in range(t - 1):
        X = Z @ (Z.T @ X)
    assert r == l
    assert _span_angle(Q, X) <= 1e-8
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-12
    assert np.abs(c["V"].T @ Q).max() <= 1e-12
    assert np.abs(P - Z.T @ Q).max() <= 1e-12 * np.abs(Z).max()
    assert np.abs(Z @ Y - Q).max() <= 1e-12


def _check(test, ref, theta_hat, sig_tol=1e-10, ang_tol=1e-8):
    r = metrics.compare(test, ref, theta_hat, 1e-8)
    assert r["sigma_rel"] <= sig_tol, r
    assert r["angle_U"] <= ang_tol and r["angle_V"] <= ang_tol, r
    assert r["orth_U"] <= 1e-11 and r["orth_V"] <= 1e-11, r


def _starts(rng, kind, c, method, l):
    def one(s):
        return rng.standard_normal(s) if method == "gkl" else rng.standard_normal((s, l))
    if kind == "weights":
        return (one(c["D_T"].rows), one(c["Em_T"].rows))
    return one(c["E"].rows)


def _apply(c, method, l, t, start):
    f = {"rows": approx.add_rows, "cols": approx.add_cols}
    if c["kind"] == "weights":
        return approx.update_weights(c["U"], c["s"], c["V"], c["D_T"], c["Em_T"],
                                     method=method, l=l, t=t, start=start)
    return f[c["kind"]](c["U"], c["s"], c["V"], c["E"], method=method, l=l, t=t, start=start)


@pytest.mark.parametrize("kind", ["rows", "cols", "weights"])
@pytest.mark.parametrize("method", ["gkl", "rpi"])
def test_full_space_is_exact(kind, method):
    c, rng = _case(20 + len(kind), s=6, kind=kind)
    s_upd = (c["D_T"] if kind == "weights" else c["E"]).rows
    start = _starts(rng, kind, c, method, s_upd)
    Ut, st, Vt, info = _apply(c, method, s_upd, 1, start)
    U0, s0, V0, i0 = brute.apply(c["U"], c["s"], c["V"], _upd(c))
    _check((Ut, st, Vt), (U0, s0, V0), i0["theta_hat"])


def _projected(c, info):
    """The updated matrix with the new block projected onto span[basis, Q]."""
    U, s, V = c["U"], c["s"], c["V"]
    A = (U * s) @ V.T
    if c["kind"] == "rows":
        Pi = V @ V.T + info["Q"] @ info["Q"].T
        return np.vstack([A, c["E"].to_dense() @ Pi])
    if c["kind"] == "cols":
        Pi = U @ U.T + info["Q"] @ info["Q"].T
        return np.hstack([A, Pi @ c["E"].to_dense().T])
    PU = U @ U.T + info["QD"] @ info["QD"].T
    PV = V @ V.T + info["QE"] @ info["QE"].T
    return A + PU @ c["D_T"].to_dense().T @ c["Em_T"].to_dense() @ PV


@pytest.mark.parametrize("kind", ["rows", "cols", "weights"])
@pytest.mark.parametrize("method,l,t", [("gkl", 3, 1), ("gkl", 5, 1), ("rpi", 3, 2), ("rpi", 4, 3)])
def test_projection_definition(kind, method, l, t):
    c, rng = _case(40 + l + t + len(kind), s=10, kind=kind)
    s_upd = (c["D_T"] if kind == "weights" else c["E"]).rows
    start = _starts(rng, kind, c, method, l)
    Ut, st, Vt, info = _apply(c, method, l, t, start)
    M = _projected(c, info)
    Ub, th, Vbt = np.linalg.svd(M, full_matrices=False)
    k = c["k"]
    _check((Ut, st, Vt), (Ub[:, :k], th[:k], Vbt[:k].T), th)


def test_gkl_breakdown_on_rank_deficient_update():
    c, rng = _case(77, s=6)
    E = c["E"].to_dense()
    E[3:] = E[:3]                        # rank(Z) <= 3
    from synth import CSR
    c["E"] = CSR.from_dense(E)
    Z, _, scale = approx.augmented(E.T, c["V"])
    Q, P, Y, alpha, beta = approx.gkl(Z, 10, rng.standard_normal(6), scale)
    assert np.count_nonzero(alpha) <= 3
    assert np.abs(Q.T @ Q - np.diag((alpha > 0).astype(float))).max() <= 1e-10
    Ut, st, Vt, info = approx.add_rows(c["U"], c["s"], c["V"], c["E"], "gkl", 10, 1,
                                       rng.standard_normal(6))
    U0, s0, V0, i0 = brute.apply(c["U"], c["s"], c["V"], ("rows", c["E"]))
    _check((Ut, st, Vt), (U0, s0, V0), i0["theta_hat"])


# ------------------------------------------------------------ planted mistakes
def _gkl_mutant(mutation):
    """The GKL process with one slip, planted in a copy (CPU only)."""
    def gkl(Z, l, p1=None, scale=None, rtol=1e-10):
        m, s = Z.shape
        l = min(l, s)
        p = np.asarray(p1, dtype=np.float64) / np.linalg.norm(p1)
        Pv = np.zeros((s, l + 1)); Pv[:, 0] = p
        Q = np.zeros((m, l)); Y = np.zeros((s, l))
        alpha = np.zeros(l); beta = np.zeros(l)
        q_prev = np.zeros(m); y_prev = np.zeros(s); b_prev = 0.0
        for i in range(l):
            bq = 0.0 if mutation == "drop_beta_in_q" else b_prev
            q = Z @ Pv[:, i] - bq * q_prev
            y = Pv[:, i] + bq * y_prev if mutation == "y_sign" else Pv[:, i] - bq * y_prev
            a = float(np.linalg.norm(q))
            q, y = q / a, y / a
            alpha[i] = a; Q[:, i], Y[:, i] = q, y
            pn = Z.T @ q - a * Pv[:, i]
            for _ in range(2):
                pn = pn - Pv[:, : i + 1] @ (Pv[:, : i + 1].T @ pn)
            b = float(np.linalg.norm(pn))
            beta[i] = b; Pv[:, i + 1] = pn / b
            q_prev, y_prev, b_prev = q, y, b
        H = np.zeros((l, l + 1))
        H[np.arange(l), np.arange(l)] = alpha
        if mutation != "drop_superdiag":
            H[np.arange(l), np.arange(1, l + 1)] = beta
        return Q, Pv @ H.T, Y, alpha, beta
    return gkl


def _rpi_mutant(mutation):
    def rpi(Z, l, t, P0, scale=None, rtol=1e-10):
        P = np.asarray(P0, dtype=np.float64)[:, :l].copy()
        for _ in range(t):
            P, _r = np.linalg.qr(P)
            X = Z @ P if mutation != "transpose_product" else Z @ (Z.T @ (Z @ P))
            Q, _r = np.linalg.qr(X)
            Pn = Z.T @ Q
            P = P if mutation == "stale_P" else Pn
        return Q, P, None, l
    return rpi


@pytest.mark.parametrize("method,mutation", [("gkl", "drop_beta_in_q"), ("gkl", "y_sign"),
                                             ("gkl", "drop_superdiag"), ("rpi", "stale_P"),
                                             ("rpi", "transpose_product")])
def test_planted_mistakes_are_caught(monkeypatch, method, mutation):
    c, rng = _case(91, s=10)
    l, t = 4, 2
    start = _starts(rng, "rows", c, method, l)
    ref = approx.add_rows(c["U"], c["s"], c["V"], c["E"], method, l, t, start)
    if method == "gkl":
        monkeypatch.setattr(approx, "gkl", _gkl_mutant(mutation))
    else:
        monkeypatch.setattr(approx, "rpi", _rpi_mutant(mutation))
    Ut, st, Vt, info = approx.add_rows(c["U"], c["s"], c["V"], c["E"], method, l, t, start)
    caught = False
    # the pins: projection definition and the Krylov / power space
    M = _projected(c, info)
    Ub, th, Vbt = np.linalg.svd(M, full_matrices=False)
    r = metrics.compare((Ut, st, Vt), (Ub[:, :4], th[:4], Vbt[:4].T), th, 1e-8)
    caught |= r["sigma_rel"] > 1e-9 or r["angle_U"] > 1e-7 or r["angle_V"] > 1e-7
    caught |= r["orth_U"] > 1e-10 or r["orth_V"] > 1e-10
    Z, _, _ = approx.augmented(c["E"].to_dense().T, c["V"])
    caught |= np.abs(info["P"] - Z.T @ info["Q"]).max() > 1e-10 * np.abs(Z).max()
    if info["Y"] is not None:
        caught |= np.abs(Z @ info["Y"] - info["Q"]).max() > 1e-10
    if method == "rpi":
        X = Z @ start
        for _ in range(t - 1):
            X = Z @ (Z.T @ X)
        caught |= _span_angle(info["Q"], X) > 1e-8
    assert caught, mutation
    assert ref is not None
