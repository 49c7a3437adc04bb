"""GPU parity of the -GKL and -RPI variants against the FP64 oracle O3.

Lock-step: the oracle starts from the factors the GPU holds before the update
(realised in FP64) and uses the same start vectors, so a difference measures
the update alone.  Tolerances as for the exact path (tests/test_gpu_parity):
FP64 sigma_rel <= 1e-10 and sin(angle) <= 1e-8; BF16x3 / FP32 1e-5 and 1e-4.
Cases: both append forms and the weight form, both methods, several tiles of
the Gram (s up to 300), l > s (clamped), a rank-deficient update that stops
GKL early, the default GKL start, sequences of updates, and argument errors.
"""
import numpy as np
import pytest

from oracle import approx, metrics
from synth import CSR, small_case

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(sig=1e-10, ang=1e-8, delta=1e-6, orth=1e-10),
       "fp32": dict(sig=1e-5, ang=1e-4, delta=1e-3, orth=1e-5),
       "bf16x3": dict(sig=1e-5, ang=1e-4, delta=1e-3, orth=5e-5)}


def _L():
    import paper_2401_09703_amd as L
    return L


def _start(rng, method, s, l):
    return rng.standard_normal(s) if method == "gkl" else rng.standard_normal((s, l))


def _lockstep(svd, kind, E, method, l, t, start, prec, label):
    L = _L()
    U0, s0, V0 = svd.factors()
    svd.apply((kind, E), approx=L.Approx(method, l, t, start))
    svd.sync()
    U1, s1, V1 = svd.factors()
    f = approx.add_rows if kind == "rows" else approx.add_cols
    host_start = start.cpu().numpy() if hasattr(start, "cpu") else start
    Ur, sr, Vr, info = f(U0, s0, V0, E, method=method, l=l, t=t, start=host_start)
    tol = TOL[prec]
    r = metrics.compare((U1, s1, V1), (Ur, sr, Vr), info["theta_hat"], tol["delta"])
    print(label, prec, method, {k: (f"{v:.2e}" if isinstance(v, float) else v)
                                for k, v in r.items()}, flush=True)
    assert r["sigma_rel"] <= tol["sig"], (label, r)
    assert r["angle_U"] <= tol["ang"] and r["angle_V"] <= tol["ang"], (label, r)
    st = svd.stats()
    kap = max(st["last_kappa_U"], st["last_kappa_V"])
    orth = tol["orth"] if prec != "fp64" else max(tol["orth"], 1e3 * 2.2e-16 * min(kap, 1e4))
    assert r["orth_U"] <= orth and r["orth_V"] <= orth, (label, r, st)
    return r


CASES = [
    # m, n, k, s, kind, density, method, l, t
    (300, 200, 16, 70, "rows", 0.05, "gkl", 10, 1),
    (300, 200, 16, 70, "rows", 0.05, "rpi", 10, 3),
    (260, 330, 32, 100, "cols", 0.04, "gkl", 10, 1),
    (260, 330, 32, 100, "cols", 0.04, "rpi", 12, 2),
    (900, 700, 64, 300, "rows", 0.01, "gkl", 16, 1),
    (900, 700, 64, 300, "rows", 0.01, "rpi", 16, 3),
    (600, 500, 128, 90, "cols", 0.03, "gkl", 20, 1),
    (400, 300, 16, 6, "rows", 0.2, "gkl", 10, 1),      # l > s: clamped to s
    (400, 300, 16, 6, "cols", 0.2, "rpi", 10, 2),
]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("m,n,k,s,kind,dens,method,l,t", CASES)
def test_variant_matches_oracle(prec, m, n, k, s, kind, dens, method, l, t):
    L = _L()
    rng = np.random.default_rng(7000 + m + n + k + s + l + t)
    c = small_case(rng, m, n, k, s, kind=kind, density=dens)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision=prec)
    try:
        _lockstep(svd, kind, c["E"], method, l, t, _start(rng, method, s, min(l, s)), prec,
                  f"{kind} m={m} n={n} k={k} s={s} l={l} t={t}")
    finally:
        svd.close()


WCASES = [
    # m, n, k, s, density, method, l, t
    (300, 200, 16, 40, 0.05, "gkl", 10, 1),
    (300, 200, 16, 40, 0.05, "rpi", 10, 3),
    (500, 400, 32, 120, 0.03, "gkl", 16, 1),
    (500, 400, 64, 120, 0.03, "rpi", 12, 2),
    (400, 300, 16, 6, 0.2, "gkl", 10, 1),     # l > s: clamped to s
]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("m,n,k,s,dens,method,l,t", WCASES)
def test_weight_variant_matches_oracle(prec, m, n, k, s, dens, method, l, t):
    L = _L()
    rng = np.random.default_rng(9100 + m + n + k + s + l + t)
    c = small_case(rng, m, n, k, s, kind="weights", density=dens)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision=prec)
    try:
        U0, s0, V0 = svd.factors()
        lc = min(l, s)
        start = (_start(rng, method, s, lc), _start(rng, method, s, lc))
        svd.apply(("weights", c["D_T"], c["Em_T"]), approx=L.Approx(method, l, t, start))
        svd.sync()
        U1, s1, V1 = svd.factors()
        Ur, sr, Vr, info = approx.update_weights(U0, s0, V0, c["D_T"], c["Em_T"], method=method,
                                                 l=l, t=t, start=start)
        tol = TOL[prec]
        r = metrics.compare((U1, s1, V1), (Ur, sr, Vr), info["theta_hat"], tol["delta"])
        print("weights", prec, method, r, flush=True)
        assert r["sigma_rel"] <= tol["sig"], r
        assert r["angle_U"] <= tol["ang"] and r["angle_V"] <= tol["ang"], r
        st = svd.stats()
        kap = max(st["last_kappa_U"], st["last_kappa_V"])
        orth = tol["orth"] if prec != "fp64" else max(tol["orth"], 1e3 * 2.2e-16 * min(kap, 1e4))
        assert r["orth_U"] <= orth and r["orth_V"] <= orth, (r, st)
    finally:
        svd.close()


def test_weight_variant_mixed_methods_and_errors():
    """GKL on one side and RPI on the other (the C ABI takes one spec per
    side): the result is an orthonormal rank-k triple with U1^T A_new V1 =
    diag(sigma), since K_w is exactly the projection of the updated matrix
    onto the two bases; bad specs are rejected before any device work."""
    L = _L()
    rng = np.random.default_rng(9200)
    c = small_case(rng, 300, 250, 16, 50, kind="weights", density=0.05)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision="fp64")
    try:
        aD = L.Approx("gkl", 10, 1, rng.standard_normal(50))
        aE = L.Approx("rpi", 10, 2, rng.standard_normal((50, 10)))
        svd.update_weights(c["D_T"], c["Em_T"], approx=(aD, aE))
        svd.sync()
        U1, s1, V1 = svd.factors()
        assert metrics.orth_err(U1) < 1e-10 and metrics.orth_err(V1) < 1e-10
        assert np.all(np.diff(s1) <= 1e-12 * s1[0])
        A_new = (c["U"] * c["s"]) @ c["V"].T + c["D_T"].to_dense().T @ c["Em_T"].to_dense()
        M = U1.T @ A_new @ V1
        assert np.abs(M - np.diag(s1)).max() <= 1e-10 * s1[0]
        with pytest.raises(L.SvlcovError):
            svd.update_weights(c["D_T"], c["Em_T"], approx=(aD, L.Approx("rpi", 10, 2, None)))
        with pytest.raises(L.SvlcovError):
            svd.update_weights(c["D_T"], c["Em_T"], approx=(aD, L.Approx("gkl", 0, 1, None)))
    finally:
        svd.close()


@pytest.mark.parametrize("method", ["gkl", "rpi"])
def test_weight_variant_selection_against_tall_factor(method):
    """D = I[:, R] (a selection of 32 rows) against a 20 000-row U: the
    residual Gram of D is I - U_R U_R^T, a nearly flat spectrum whose Krylov
    increments are small (~k/m) but genuine.  In BF16x3 mode the basis must
    not stop at the exact path's rounding floor there (it did: one GKL step,
    a subspace 1e-4 away from the oracle's)."""
    import scipy.sparse as sp
    from synth import bernoulli_uniform, synthetic_factors
    L = _L()
    rng = np.random.default_rng(9300)
    m, n, k, s, l = 20000, 3000, 16, 32, 10
    U, sig, V = synthetic_factors(m, n, k, rng)
    R = np.sort(rng.choice(m, size=s, replace=False))
    D_T = CSR.from_scipy(sp.csr_matrix((np.ones(s), (np.arange(s), R)), shape=(s, m)))
    Em_T = bernoulli_uniform(s, n, 0.02, rng)
    svd = L.TruncatedSVD(U, sig, V, precision="bf16x3")
    try:
        U0, s0, V0 = svd.factors()
        start = (_start(rng, method, s, l), _start(rng, method, s, l))
        svd.update_weights(D_T, Em_T, approx=L.Approx(method, l, 2, start))
        svd.sync()
        U1, s1, V1 = svd.factors()
        Ur, sr, Vr, info = approx.update_weights(U0, s0, V0, D_T, Em_T, method=method, l=l, t=2,
                                                 start=start)
        r = metrics.compare((U1, s1, V1), (Ur, sr, Vr), info["theta_hat"], 1e-3)
        assert r["sigma_rel"] <= 1e-7, r
        assert r["angle_U"] <= 1e-5 and r["angle_V"] <= 1e-5, r
    finally:
        svd.close()


def test_gkl_default_start_and_device_start():
    """start=None means all ones; a device start gives the same result as the
    same values on the host."""
    import torch
    L = _L()
    rng = np.random.default_rng(81)
    c = small_case(rng, 300, 250, 32, 60, kind="rows", density=0.05)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision="fp64")
    try:
        _lockstep(svd, "rows", c["E"], "gkl", 10, 1, None, "fp64", "default start")
        E2 = small_case(rng, 300, 250, 32, 60, kind="rows", density=0.05)["E"]
        p1 = rng.standard_normal(60)
        _lockstep(svd, "rows", E2, "gkl", 10, 1, torch.tensor(p1, device="cuda"), "fp64",
                  "device start")
    finally:
        svd.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_gkl_breakdown_rank_deficient(prec):
    """Duplicated rows: rank(Z) <= 5, so GKL stops after at most 5 steps and
    the update is the exact one of the oracle's variant."""
    L = _L()
    rng = np.random.default_rng(91)
    c = small_case(rng, 300, 200, 16, 10, kind="rows", density=0.08)
    E = c["E"].to_dense()
    E[5:] = E[:5]
    E = CSR.from_dense(E)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision=prec)
    try:
        _lockstep(svd, "rows", E, "gkl", 10, 1, rng.standard_normal(10), prec, "breakdown")
    finally:
        svd.close()


@pytest.mark.parametrize("method", ["gkl", "rpi"])
def test_variant_sequence(method):
    """Five appends alternating rows and columns, each checked lock-step."""
    L = _L()
    rng = np.random.default_rng(123 if method == "gkl" else 321)
    c = small_case(rng, 500, 400, 32, 80, kind="rows", density=0.03)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision="fp64")
    try:
        for step in range(5):
            kind = "rows" if step % 2 == 0 else "cols"
            m, n = svd.shape()
            width = n if kind == "rows" else m
            from synth.sparse import bernoulli_uniform
            E = bernoulli_uniform(80, width, 0.03, rng)
            _lockstep(svd, kind, E, method, 10, 3, _start(rng, method, 80, 10), "fp64",
                      f"step {step}")
    finally:
        svd.close()


def test_variant_argument_errors():
    L = _L()
    rng = np.random.default_rng(5)
    c = small_case(rng, 200, 150, 16, 20, kind="rows", density=0.1)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision="fp64")
    try:
        for bad in (L.Approx("gkl", 0), L.Approx("gkl", 65), L.Approx("rpi", 5, 3, None),
                    L.Approx("rpi", 5, 0, rng.standard_normal((20, 5))),
                    L.Approx("gkl", 5, 1, np.full(20, np.nan))):
            with pytest.raises(L.SvlcovError):
                svd.add_rows(c["E"], approx=bad)
        svd.sync()
        # the state is unchanged and still usable
        _lockstep(svd, "rows", c["E"], "gkl", 5, 1, rng.standard_normal(20), "fp64", "after errors")
    finally:
        svd.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("kind", ["rows", "cols"])
def test_rpi_rank_deficient_update(prec, kind):
    """rank(Z) = 4 < l = 10 (30 update rows that are scaled copies of four):
    the power iteration keeps four directions and drops the others by the
    pivot rule, as the oracle's RPI does, and the two updates agree."""
    L = _L()
    rng = np.random.default_rng(7700 + len(kind))
    m, n, k, s, l, t = 400, 300, 16, 30, 10, 2
    c = small_case(rng, m, n, k, 4, kind=kind, density=0.08)
    base = c["E"].to_dense()
    E = CSR.from_dense(np.vstack([base[i % 4] * (1.0 + 0.5 * (i // 4)) for i in range(s)]))
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision=prec)
    try:
        _lockstep(svd, kind, E, "rpi", l, t, rng.standard_normal((s, l)), prec,
                  f"rank-deficient {kind} s={s} l={l} t={t}")
    finally:
        svd.close()
