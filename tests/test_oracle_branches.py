"""Pins of oracle branches that ordinary inputs do not reach (CPU only).

  RPI drop branch   a rank-deficient augmented matrix Z (rank r < l) and a
                    start block with repeated columns: the power iteration
                    must keep exactly r directions, span range(Z), and make
                    the update exact (Z = Q P^T), which brute force checks
  metrics           gap_prefix, sin_angle, sigma_rel_err and orth_err on
                    hand-built spectra and subspaces at known angles
  O2 reset branch   the extended decomposition with the inner factor folded
                    into the tall one at every update (the remedy at the end
                    of Section 3.2) against O1, and the disjoint-support case
                    in which the new inner factor is exactly singular

Each group also plants a mistake in a copy of the branch and shows that its
pin fails.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import approx, brute, metrics, svlcov, zha_simon
from synth import CSR, random_orthonormal, small_case, synthetic_factors


# ------------------------------------------------------------ RPI drop branch
def _low_rank_update(rng, m, n, k, s, r):
    """Factors of a rank-k matrix and an s x n update whose residual against
    V has rank r: E = (B1 C1) + (coefficients) V^T with B1 s x r, C1 r x n."""
    U, sig, V = synthetic_factors(m, n, k, rng)
    W = rng.standard_normal((r, n))
    W -= (W @ V) @ V.T                          # r directions outside span(V)
    E = rng.standard_normal((s, r)) @ W + rng.standard_normal((s, k)) @ V.T
    return U, sig, V, E


@pytest.mark.parametrize("t", [2, 3])
def test_rpi_keeps_exactly_the_rank_of_z(t):
    rng = np.random.default_rng(101 + t)
    m, n, k, s, r, l = 60, 50, 4, 12, 3, 8
    U, sig, V, E = _low_rank_update(rng, m, n, k, s, r)
    Z, C, scale = approx.augmented(CSR.from_dense(E).to_scipy().T, V)
    assert np.linalg.matrix_rank(Z, tol=1e-10 * np.linalg.norm(Z, 2)) == r
    P0 = rng.standard_normal((s, l))
    Q, P, Y, kept = approx.rpi(Z, l, t, P0, scale)
    assert kept == r
    # the dropped directions are zero columns; the kept ones are orthonormal
    assert np.all(Q[:, r:] == 0.0) and np.all(Y[:, r:] == 0.0)
    np.testing.assert_allclose(Q[:, :r].T @ Q[:, :r], np.eye(r), atol=1e-12)
    # Q = Z Y, and span(Q) = range(Z), so Z = Q P^T exactly
    np.testing.assert_allclose(Z @ Y, Q, atol=1e-11)
    Uz = np.linalg.svd(Z, full_matrices=False)[0][:, :r]
    assert metrics.sin_angle(Q[:, :r], Uz) < 1e-10
    np.testing.assert_allclose(Q @ P.T, Z, atol=1e-11 * np.linalg.norm(Z))


def test_rpi_drops_repeated_start_columns():
    """A start block with two equal columns: the QR of P drops one direction
    (relative pivot), the iteration still finds all of range(Z)."""
    rng = np.random.default_rng(111)
    m, n, k, s, r, l = 50, 40, 4, 10, 4, 6
    U, sig, V, E = _low_rank_update(rng, m, n, k, s, r)
    Z, C, scale = approx.augmented(CSR.from_dense(E).to_scipy().T, V)
    P0 = rng.standard_normal((s, l))
    P0[:, 3] = P0[:, 1]
    P0 *= 1e-14                                  # only the relative pivot is meaningful
    Q, P, Y, kept = approx.rpi(Z, l, 3, P0, scale)
    assert kept == r
    Uz = np.linalg.svd(Z, full_matrices=False)[0][:, :r]
    assert metrics.sin_angle(Q[:, :r], Uz) < 1e-10


@pytest.mark.parametrize("kind", ["rows", "cols"])
def test_rpi_update_exact_on_rank_deficient_z(kind):
    """rank(Z) = r < l: the RPI update equals the exact update (brute force,
    Definition 2) because Z = Q P^T holds exactly."""
    rng = np.random.default_rng(121)
    m, n, k, s, r, l = 70, 55, 5, 14, 3, 9
    if kind == "rows":
        U, sig, V, E = _low_rank_update(rng, m, n, k, s, r)
        up = ("rows", CSR.from_dense(E))
        test = approx.add_rows(U, sig, V, up[1], method="rpi", l=l, t=2,
                               start=rng.standard_normal((s, l)))
    else:
        V, sig, U, E = _low_rank_update(rng, n, m, k, s, r)   # E is s x m
        up = ("cols", CSR.from_dense(E))
        test = approx.add_cols(U, sig, V, up[1], method="rpi", l=l, t=2,
                               start=rng.standard_normal((s, l)))
    Ub, sb, Vb, info = brute.apply(U, sig, V, up)
    r_ = metrics.compare(test[:3], (Ub, sb, Vb), info["theta_hat"], 1e-8)
    assert r_["sigma_rel"] < 1e-11 and r_["angle_U"] < 1e-9 and r_["angle_V"] < 1e-9, r_


def _rpi_abs_drop(Z, l, t, P0, scale=None, rtol=1e-10):
    """Planted mistake: the QR of P drops pivots below rtol in absolute
    terms instead of relative to the largest pivot."""
    m, s = Z.shape
    l = min(l, s)
    thr = rtol * scale
    P = np.asarray(P0, dtype=np.float64)[:, :l].copy()
    Q = np.zeros((m, l)); Y = np.zeros((s, l)); r = 0
    for _ in range(t):
        Qp, Rp, _pv = sla.qr(P, mode="economic", pivoting=True)
        dp = np.abs(np.diag(Rp))
        rp = int(np.sum(dp > rtol))
        P = np.zeros_like(P); P[:, :rp] = Qp[:, :rp]
        X = Z @ P
        Qf, R, piv = sla.qr(X, mode="economic", pivoting=True)
        r = int(np.sum(np.abs(np.diag(R)) > thr))
        Q = np.zeros((m, l)); Y = np.zeros((s, l))
        Q[:, :r] = Qf[:, :r]
        Y[:, :r] = P[:, piv[:r]] @ sla.solve_triangular(R[:r, :r], np.eye(r))
        P = Z.T @ Q
    return Q, P, Y, r


def _rpi_no_drop(Z, l, t, P0, scale=None, rtol=1e-10):
    """Planted mistake: every direction of Z P is kept, however small its
    pivot (the solve then turns rounding into basis vectors)."""
    m, s = Z.shape
    l = min(l, s)
    P = np.asarray(P0, dtype=np.float64)[:, :l].copy()
    Q = np.zeros((m, l)); Y = np.zeros((s, l)); r = 0
    for _ in range(t):
        P = sla.qr(P, mode="economic")[0]
        Qf, R, piv = sla.qr(Z @ P, mode="economic", pivoting=True)
        r = l
        Q = Qf.copy()
        Y = P[:, piv] @ sla.solve_triangular(R, np.eye(l))
        P = Z.T @ Q
    return Q, P, Y, r


@pytest.mark.parametrize("mutant", [_rpi_abs_drop, _rpi_no_drop], ids=["abs_drop", "no_drop"])
def test_rpi_drop_mutants_are_caught(monkeypatch, mutant):
    rng = np.random.default_rng(111)
    m, n, k, s, r, l = 50, 40, 4, 10, 4, 6
    U, sig, V, E = _low_rank_update(rng, m, n, k, s, r)
    Z, C, scale = approx.augmented(CSR.from_dense(E).to_scipy().T, V)
    P0 = rng.standard_normal((s, l))
    P0[:, 3] = P0[:, 1]
    P0 *= 1e-14
    Q, P, Y, kept = mutant(Z, l, 3, P0, scale)
    Uz = np.linalg.svd(Z, full_matrices=False)[0][:, :r]
    ok = (kept == r and np.allclose(Z @ Y, Q, atol=1e-11)
          and metrics.sin_angle(Q[:, :r], Uz) < 1e-10
          and np.allclose(Q[:, :r].T @ Q[:, :r], np.eye(r), atol=1e-12))
    assert not ok


# ------------------------------------------------------------------- metrics
def test_gap_prefix_hand_built():
    th = np.array([10.0, 9.0, 9.0, 5.0, 5.0, 5.0, 1.0])
    # j = 4 sits inside the repeated 5s, so the prefix falls back to j = 3
    assert metrics.gap_prefix(th, 4, 0.05) == 3
    assert metrics.gap_prefix(th, 3, 0.05) == 3
    assert metrics.gap_prefix(th, 6, 0.05) == 6
    # k beyond the spectrum: the value after the last one counts as 0
    assert metrics.gap_prefix(th, 7, 0.05) == 7
    # a gap of 1.0 = 0.1 theta_1 passes at delta 0.1 but not just above it
    assert metrics.gap_prefix(th, 2, 0.1) == 1
    assert metrics.gap_prefix(th, 2, 0.1000001) == 0
    assert metrics.gap_prefix(np.zeros(5), 3, 1e-3) == 0
    assert metrics.gap_prefix(np.array([]), 3, 1e-3) == 0


@pytest.mark.parametrize("theta", [1e-9, 1e-4, 0.3, 1.2])
def test_sin_angle_known_angles(theta):
    rng = np.random.default_rng(5)
    Q = random_orthonormal(6, 6, rng)
    # two 2-d subspaces with principal angles theta/3 and theta
    A = Q[:, :2]
    B = np.column_stack([np.cos(theta / 3) * Q[:, 0] + np.sin(theta / 3) * Q[:, 2],
                         np.cos(theta) * Q[:, 1] + np.sin(theta) * Q[:, 3]])
    expect = np.sin(theta)
    assert abs(metrics.sin_angle(A, B) - expect) <= 1e-14 + 1e-12 * expect
    # independent of the bases chosen for the subspaces
    M = rng.standard_normal((2, 2)) + 3 * np.eye(2)
    assert abs(metrics.sin_angle(A @ M, 5.0 * B) - expect) <= 1e-13 + 1e-10 * expect
    assert metrics.sin_angle(A, A @ M) < 1e-14
    assert metrics.sin_angle(A[:, :0], B[:, :0]) == 0.0


def test_sigma_rel_err_and_floor():
    ref = np.array([10.0, 1.0, 1e-10])
    test = np.array([10.001, 1.001, 2e-10])
    # the third value lies below 1e-8 * 10, so it is measured against 10
    assert metrics.sigma_rel_err(test, ref) == pytest.approx(1e-3, rel=1e-9)
    assert metrics.sigma_rel_err(np.array([10.0, 1.0, 0.0]), ref) == pytest.approx(1e-11, rel=1e-9)
    # with the floor at 1e-12 the same entry is relative to itself
    assert metrics.sigma_rel_err(test, ref, floor=1e-12) == pytest.approx(1.0, rel=1e-9)
    assert metrics.sigma_rel_err(np.array([]), np.array([])) == 0.0


def test_orth_err_known():
    rng = np.random.default_rng(7)
    Q = random_orthonormal(9, 4, rng)
    assert metrics.orth_err(Q) < 1e-14
    X = Q.copy()
    X[:, 2] *= 1.5                                  # X^T X - I = diag(0, 0, 1.25, 0)
    assert metrics.orth_err(X) == pytest.approx(1.25, rel=1e-12)


# ------------------------------------------------------------ O2 reset branch
@pytest.mark.parametrize("kind", ["rows", "cols", "weights"])
def test_o2_forced_reset_matches_o1(kind):
    """cond_reset below 1 folds every new inner factor into the tall one; the
    result is the same update (only rounding changes) and every side resets."""
    rng = np.random.default_rng(131)
    c = small_case(rng, 60, 45, 5, 7, kind=kind, density=0.15, dup_rows=1)
    up = ("weights", c["D_T"], c["Em_T"]) if kind == "weights" else (kind, c["E"])
    o2 = svlcov.ExtendedSVD(c["U"], c["s"], c["V"], cond_reset=0.5)
    o2.apply(up)
    assert o2.resets == 2
    assert np.array_equal(o2.Upp, np.eye(5)) and np.array_equal(o2.Vpp, np.eye(5))
    Ur, sr, Vr, info = zha_simon.apply(c["U"], c["s"], c["V"], up)
    r = metrics.compare(o2.factors(), (Ur, sr, Vr), info["theta_hat"], 1e-8)
    assert r["sigma_rel"] < 1e-11 and r["angle_U"] < 1e-9 and r["angle_V"] < 1e-9, r
    assert r["orth_U"] < 1e-12 and r["orth_V"] < 1e-12, r
    # a second update from the reset state still matches
    U1, s1, V1 = o2.factors()
    E2 = CSR.from_dense(rng.random((6, V1.shape[0])) * (rng.random((6, V1.shape[0])) < 0.15))
    o2.apply(("rows", E2))
    assert o2.resets == 4
    Ur, sr, Vr, info = zha_simon.add_rows(U1, s1, V1, E2)
    r = metrics.compare(o2.factors(), (Ur, sr, Vr), info["theta_hat"], 1e-8)
    assert r["sigma_rel"] < 1e-11 and r["angle_U"] < 1e-9 and r["angle_V"] < 1e-9, r


def _disjoint_case(rng):
    m, n, k, s_ = 40, 30, 5, 4
    J = np.arange(20, 30)
    U = random_orthonormal(m, k, rng)
    V = np.zeros((n, k)); V[:20] = random_orthonormal(20, k, rng)
    s = np.array([6.0, 4.0, 3.0, 2.0, 1.0])
    E = np.zeros((s_, n)); E[:, J] = rng.standard_normal((s_, J.size)) * 2.5
    return U, s, V, E


def test_o2_disjoint_support_resets_and_is_exact():
    """The update lives where V vanishes: new top directions are orthogonal to
    the old subspace, so the new inner factor of U is singular and the
    extended decomposition must fold it in; the result is top-k of the union
    of the spectra."""
    rng = np.random.default_rng(61)
    U, s, V, E = _disjoint_case(rng)
    expect = np.sort(np.concatenate([s, np.linalg.svd(E, compute_uv=False)]))[::-1][:5]
    assert expect[4] > s[-1]                    # some new direction enters the top k
    o2 = svlcov.ExtendedSVD(U, s, V)
    o2.apply(("rows", CSR.from_dense(E)))
    assert o2.resets >= 1
    np.testing.assert_allclose(o2.s, expect, rtol=1e-12)
    Ur, sr, Vr, info = zha_simon.add_rows(U, s, V, CSR.from_dense(E))
    r = metrics.compare(o2.factors(), (Ur, sr, Vr), info["theta_hat"], 1e-8)
    assert r["angle_U"] < 1e-9 and r["angle_V"] < 1e-9 and r["orth_U"] < 1e-12, r


def test_o2_reset_mutant_is_caught(monkeypatch):
    """Planted mistake in the reset branch: the tall factor is not multiplied
    by the new inner factor before the inner factor becomes the identity."""
    def bad_new_inner(self, old_inner, new_inner, tall):
        if np.linalg.cond(new_inner) > self.cond_reset:
            self.resets += 1
            return tall, np.eye(self.k), None
        return tall, new_inner, np.linalg.inv(new_inner)

    monkeypatch.setattr(svlcov.ExtendedSVD, "_new_inner", bad_new_inner)
    rng = np.random.default_rng(131)
    c = small_case(rng, 60, 45, 5, 7, kind="rows", density=0.15, dup_rows=1)
    o2 = svlcov.ExtendedSVD(c["U"], c["s"], c["V"], cond_reset=0.5)
    o2.apply(("rows", c["E"]))
    Ur, sr, Vr, info = zha_simon.apply(c["U"], c["s"], c["V"], ("rows", c["E"]))
    r = metrics.compare(o2.factors(), (Ur, sr, Vr), info["theta_hat"], 1e-8)
    assert r["angle_U"] > 1e-6 or r["angle_V"] > 1e-6 or r["orth_U"] > 1e-6
