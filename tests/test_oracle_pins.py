"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own formulas (CPU only).

  closed forms   hand-derived SVD_k of tiny updated matrices (tests/golden)
  brute force    O1 (Zha-Simon) and O2 (the paper's SV-LCOV method) against a
                 dense SVD of the updated matrix (Definition 2, Theorem 1)
  exactness      rank(updated) <= k reproduces the updated matrix exactly
  energy         sum of the squared spectrum of K equals ||updated||_F^2
  interlacing    sigma_old_i <= theta_i <= sqrt(sigma_old_i^2 + ||E||_2^2)
  secular eq.    s = 1: roots of the arrowhead secular equation by bisection
  disjoint       an update on columns where V vanishes: theta = top-k of the
                 union of the old values and sigma(E)
  metamorphic    cols == rows on the transpose; rows == zero-row append + a
                 weight update (links Algorithm 4 and Algorithm 11); scaling;
                 permutation of the new rows
"""
import json
import os

import numpy as np
import pytest

from oracle import brute, metrics, svlcov, zha_simon
from synth import CSR, random_orthonormal, small_case, synthetic_factors
from synth.sparse import bernoulli_uniform

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _upd(c):
    if c["kind"] == "weights":
        return ("weights", c["D_T"], c["Em_T"])
    return (c["kind"], c["E"])


def _check(test, ref, theta_hat, sig_tol=1e-11, ang_tol=1e-9, delta=1e-8):
    r = metrics.compare(test, ref, theta_hat, delta)
    assert r["sigma_rel"] <= sig_tol, r
    assert r["angle_U"] <= ang_tol and r["angle_V"] <= ang_tol, r
    assert r["orth_U"] <= 1e-12 and r["orth_V"] <= 1e-12, r
    return r


# ----------------------------------------------------------------- closed forms
@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"],
                         ids=lambda c: c["name"])
def test_closed_forms(case):
    U = np.array(case["U"]); s = np.array(case["s"]); V = np.array(case["V"])
    kind = case["kind"]
    if kind == "rows":
        up = ("rows", CSR.from_dense(case["E"]))
    elif kind == "cols":
        up = ("cols", CSR.from_dense(case["Ec_T"]))
    else:
        up = ("weights", CSR.from_dense(case["D_T"]), CSR.from_dense(case["Em_T"]))
    for res in (zha_simon.apply(U, s, V, up)[:3], _o2(U, s, V, up)):
        Un, th, Vn = res
        np.testing.assert_allclose(th, case["sigma"], rtol=1e-13)
        if "U_expected" in case:
            for X, Xe in ((Un, case["U_expected"]), (Vn, case["V_expected"])):
                Xe = np.array(Xe)
                sgn = np.sign(np.sum(X * Xe, axis=0))
                np.testing.assert_allclose(X * sgn, Xe, atol=1e-13)


def _o2(U, s, V, up):
    ex = svlcov.ExtendedSVD(U, s, V)
    ex.apply(up)
    return ex.factors()


# ----------------------------------------------------------------- brute force
CASES = [
    # (m, n, k, s, kind, density, dup, empty, inspan)
    (40, 30, 4, 6, "rows", 0.2, 0, 0, 0),
    (40, 30, 4, 6, "cols", 0.2, 0, 0, 0),
    (40, 30, 4, 6, "weights", 0.2, 0, 0, 0),
    (50, 35, 6, 9, "rows", 0.15, 2, 1, 0),
    (50, 35, 6, 9, "cols", 0.15, 2, 1, 0),
    (50, 35, 6, 9, "weights", 0.15, 2, 1, 0),
    (30, 25, 5, 4, "rows", 0.3, 0, 0, 2),
    (30, 25, 5, 4, "cols", 0.3, 0, 0, 2),
    (60, 45, 8, 12, "rows", 0.05, 1, 3, 0),
    (20, 60, 3, 1, "rows", 0.2, 0, 0, 0),
    (60, 20, 3, 1, "cols", 0.2, 0, 0, 0),
    (25, 25, 7, 10, "weights", 0.3, 0, 2, 0),
]


@pytest.mark.parametrize("m,n,k,s,kind,dens,dup,empty,inspan", CASES)
def test_o1_o2_vs_bruteforce(m, n, k, s, kind, dens, dup, empty, inspan):
    rng = np.random.default_rng(1000 + m * 7 + n * 3 + k + s)
    c = small_case(rng, m, n, k, s, kind=kind, density=dens, dup_rows=dup,
                   empty_rows=empty, in_span_rows=inspan)
    up = _upd(c)
    U0, s0, V0, i0 = brute.apply(c["U"], c["s"], c["V"], up)
    U1, s1, V1, _ = zha_simon.apply(c["U"], c["s"], c["V"], up)
    _check((U1, s1, V1), (U0, s0, V0), i0["theta_hat"])
    U2, s2, V2 = _o2(c["U"], c["s"], c["V"], up)
    # O2 orthogonalises through inner products (Algorithm 2), whose floor is
    # sqrt(u) on directions it keeps; the generic cases here keep none near it
    _check((U2, s2, V2), (U0, s0, V0), i0["theta_hat"], sig_tol=1e-10,
           ang_tol=1e-8)


def test_zero_update_is_identity():
    rng = np.random.default_rng(7)
    U, s, V = synthetic_factors(30, 20, 4, rng)
    for up in (("rows", CSR.from_dense(np.zeros((3, 20)))),
               ("cols", CSR.from_dense(np.zeros((3, 30)))),
               ("weights", CSR.from_dense(np.zeros((2, 30))),
                CSR.from_dense(np.zeros((2, 20))))):
        Un, th, Vn, info = zha_simon.apply(U, s, V, up)
        np.testing.assert_allclose(th, s, rtol=1e-14)
        assert metrics.sin_angle(Un[:30], U) < 1e-13
        assert metrics.sin_angle(Vn[:20], V) < 1e-13


def test_sequence_o2_tracks_o1():
    """Ten row appends (the shape of the small FP64 workload, scaled down):
    the paper's extended-decomposition method stays on the Zha-Simon result."""
    rng = np.random.default_rng(11)
    A = bernoulli_uniform(120, 60, 0.05, rng).to_dense()
    Ud, sd, Vt = np.linalg.svd(A, full_matrices=False)
    k = 6
    U1, s1, V1 = Ud[:, :k], sd[:k], Vt[:k].T
    ex = svlcov.ExtendedSVD(U1, s1, V1)
    for t in range(10):
        E = bernoulli_uniform(8, 60, 0.05, rng)
        U1, s1, V1, info = zha_simon.add_rows(U1, s1, V1, E)
        ex.add_rows(E.to_scipy())
        U2, s2, V2 = ex.factors()
        r = metrics.compare((U2, s2, V2), (U1, s1, V1), info["theta_hat"], 1e-6)
        assert r["sigma_rel"] < 1e-9 and r["angle_U"] < 1e-7 and r["angle_V"] < 1e-7, (t, r)


# ----------------------------------------------------------------- exactness
@pytest.mark.parametrize("kind", ["rows", "cols", "weights"])
def test_exact_when_rank_le_k(kind):
    rng = np.random.default_rng(21)
    m, n, k, r = 40, 30, 6, 3
    U = random_orthonormal(m, k, rng)
    V = random_orthonormal(n, k, rng)
    s = np.concatenate([[5.0, 3.0, 2.0], np.zeros(k - r)])
    if kind == "rows":
        # two new directions plus rows inside the current row space
        E = rng.standard_normal((4, 2)) @ rng.standard_normal((2, n))
        E[2:] = rng.standard_normal((2, r)) @ V[:, :r].T
        up = ("rows", CSR.from_dense(E))
    elif kind == "cols":
        Ec = rng.standard_normal((m, 2)) @ rng.standard_normal((2, 4))
        up = ("cols", CSR.from_dense(Ec.T))
    else:
        D = rng.standard_normal((m, 2)); Em = rng.standard_normal((n, 2))
        up = ("weights", CSR.from_dense(D.T), CSR.from_dense(Em.T))
    Abar = brute.updated_matrix(U, s, V, up)
    for Un, th, Vn in (zha_simon.apply(U, s, V, up)[:3], _o2(U, s, V, up)):
        err = np.linalg.norm((Un * th) @ Vn.T - Abar) / np.linalg.norm(Abar)
        assert err < 1e-12, err


# ----------------------------------------------------------------- energy
@pytest.mark.parametrize("kind", ["rows", "cols", "weights"])
def test_frobenius_energy(kind):
    rng = np.random.default_rng(31)
    c = small_case(rng, 50, 40, 5, 8, kind=kind, density=0.2, dup_rows=1)
    U, s, V = c["U"], c["s"], c["V"]
    _, _, _, info = zha_simon.apply(U, s, V, _upd(c))
    lhs = float(np.sum(info["theta_hat"] ** 2))
    if kind in ("rows", "cols"):
        rhs = float(np.sum(s ** 2) + np.sum(c["E"].val ** 2))
    else:
        D = c["D_T"].to_dense().T; Em = c["Em_T"].to_dense().T
        rhs = float(np.sum(s ** 2) + 2 * np.trace(np.diag(s) @ (U.T @ D) @ (Em.T @ V))
                    + np.trace((D.T @ D) @ (Em.T @ Em)))
    assert abs(lhs - rhs) <= 1e-12 * rhs


# ----------------------------------------------------------------- interlacing
@pytest.mark.parametrize("kind", ["rows", "cols"])
def test_interlacing_weyl(kind):
    rng = np.random.default_rng(41)
    c = small_case(rng, 60, 50, 7, 10, kind=kind, density=0.15)
    _, th, _, _ = zha_simon.apply(c["U"], c["s"], c["V"], _upd(c))
    e2 = np.linalg.norm(c["E"].to_dense(), 2)
    assert np.all(th >= c["s"] * (1 - 1e-14))
    assert np.all(th <= np.sqrt(c["s"] ** 2 + e2 ** 2) * (1 + 1e-14))


# ----------------------------------------------------------------- secular eq.
def _secular_roots(sig, c, e2, k):
    """Top-k roots of f(l) = e2 - l - sum_i sig_i^2 c_i^2 / (sig_i^2 - l) by
    bisection on the intervals between consecutive poles."""
    p = sig ** 2
    w = p * c ** 2

    def f(l):
        return e2 - l - np.sum(w / (p - l))
    roots = []
    hi_top = p[0] + e2 + 1.0
    bounds = [(p[0], hi_top)] + [(p[i], p[i - 1]) for i in range(1, k)]
    for lo, hi in bounds:
        a, b = lo, hi
        for _ in range(200):
            mid = 0.5 * (a + b)
            if mid == a or mid == b:
                break
            if f(mid) > 0:
                a = mid
            else:
                b = mid
        roots.append(0.5 * (a + b))
    return np.sqrt(np.array(roots))


def test_single_row_secular_equation():
    rng = np.random.default_rng(51)
    m, n, k = 40, 30, 6
    U = random_orthonormal(m, k, rng)
    V = random_orthonormal(n, k, rng)
    s = np.array([9.0, 7.0, 5.5, 4.0, 2.5, 1.0])
    e = rng.standard_normal(n)
    _, th, _, _ = zha_simon.add_rows(U, s, V, CSR.from_dense(e[None, :]))
    ref = _secular_roots(s, V.T @ e, float(e @ e), k)
    np.testing.assert_allclose(th, ref, rtol=1e-12)


# ----------------------------------------------------------------- disjoint
def test_disjoint_support():
    rng = np.random.default_rng(61)
    m, n, k, s_ = 40, 30, 5, 4
    J = np.arange(20, 30)                       # columns where V vanishes
    U = random_orthonormal(m, k, rng)
    V = np.zeros((n, k)); V[:20] = random_orthonormal(20, k, rng)
    s = np.array([6.0, 4.0, 3.0, 2.0, 1.0])
    E = np.zeros((s_, n)); E[:, J] = rng.standard_normal((s_, J.size)) * 2.5
    _, th, _, _ = zha_simon.add_rows(U, s, V, CSR.from_dense(E))
    expect = np.sort(np.concatenate([s, np.linalg.svd(E, compute_uv=False)]))[::-1][:k]
    np.testing.assert_allclose(th, expect, rtol=1e-13)


# ----------------------------------------------------------------- metamorphic
def test_cols_equals_rows_on_transpose():
    rng = np.random.default_rng(71)
    c = small_case(rng, 45, 35, 5, 7, kind="cols", density=0.2, dup_rows=1)
    Uc, sc, Vc, _ = zha_simon.add_cols(c["U"], c["s"], c["V"], c["E"])
    Vr, sr, Ur, info = zha_simon.add_rows(c["V"], c["s"], c["U"], c["E"])
    _check((Uc, sc, Vc), (Ur, sr, Vr), info["theta_hat"], 1e-13, 1e-12)


def test_rows_equal_zero_append_plus_weights():
    """[A; E] == [A; 0] + [0; I] E  (Algorithm 11 vs Algorithm 4)."""
    rng = np.random.default_rng(81)
    m, n, k, s_ = 30, 25, 5, 6
    c = small_case(rng, m, n, k, s_, kind="rows", density=0.25)
    U, s, V, E = c["U"], c["s"], c["V"], c["E"]
    Ur, sr, Vr, info = zha_simon.add_rows(U, s, V, E)
    Uz = np.vstack([U, np.zeros((s_, k))])
    D = np.zeros((m + s_, s_)); D[m:] = np.eye(s_)
    Uw, sw, Vw, _ = zha_simon.update_weights(Uz, s, V, CSR.from_dense(D.T), E)
    _check((Uw, sw, Vw), (Ur, sr, Vr), info["theta_hat"], 1e-12, 1e-11)


def test_scaling_and_row_permutation():
    rng = np.random.default_rng(91)
    c = small_case(rng, 40, 30, 5, 6, kind="rows", density=0.3)
    U, s, V, E = c["U"], c["s"], c["V"], c["E"]
    U1, s1, V1, info = zha_simon.add_rows(U, s, V, E)
    a = 3.7
    _, s2, _, _ = zha_simon.add_rows(U, a * s, V, CSR.from_dense(a * E.to_dense()))
    np.testing.assert_allclose(s2, a * s1, rtol=1e-13)
    p = rng.permutation(6)
    Up, sp_, Vp, _ = zha_simon.add_rows(U, s, V, CSR.from_dense(E.to_dense()[p]))
    j = metrics.gap_prefix(info["theta_hat"], 5, 1e-8)
    U1p = U1.copy(); U1p[40:] = U1[40:][p]
    assert metrics.sin_angle(Up[:, :j], U1p[:, :j]) < 1e-12
    np.testing.assert_allclose(sp_, s1, rtol=1e-13)
