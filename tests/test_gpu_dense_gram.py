"""Dense updates (s >= 512, density >= 2 %, >= 1024 nonzeros per row) take the Gram
E E^T through dense column blocks; the results must still match the oracle
like the sparse path's (both append forms, the weight form, the -GKL
variant, a width that is not a multiple of the block)."""
import numpy as np
import pytest

from oracle import approx, metrics, zha_simon
from synth import synthetic_factors
from synth.sparse import bernoulli_uniform

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-8, 1e-6), "bf16x3": (1e-5, 1e-4, 1e-3)}


def _check(svd, U0, s0, V0, ref, prec):
    svd.sync()
    U1, s1, V1 = svd.factors()
    Ur, sr, Vr, info = ref
    sig, ang, delta = TOL[prec]
    r = metrics.compare((U1, s1, V1), (Ur, sr, Vr), info["theta_hat"], delta)
    print(prec, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    assert r["sigma_rel"] <= sig and r["angle_U"] <= ang and r["angle_V"] <= ang, r


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("kind", ["rows", "cols", "weights", "rows-gkl"])
def test_dense_update_gram(prec, kind):
    import paper_2401_09703_amd as L
    rng = np.random.default_rng(2024 + len(kind))
    m, n, k, s = 2100, 2000, 16, 600
    U, sg, V = synthetic_factors(m, n, k, rng)
    svd = L.TruncatedSVD(U, sg, V, precision=prec)
    try:
        U0, s0, V0 = svd.factors()
        if kind == "rows":
            E = bernoulli_uniform(s, n, 0.6, rng)
            svd.apply(("rows", E))
            ref = zha_simon.add_rows(U0, s0, V0, E)
        elif kind == "cols":
            E = bernoulli_uniform(s, m, 0.6, rng)
            svd.apply(("cols", E))
            ref = zha_simon.add_cols(U0, s0, V0, E)
        elif kind == "weights":
            D = bernoulli_uniform(s, m, 0.6, rng)
            Em = bernoulli_uniform(s, n, 0.6, rng)
            svd.apply(("weights", D, Em))
            ref = zha_simon.update_weights(U0, s0, V0, D, Em)
        else:
            E = bernoulli_uniform(s, n, 0.6, rng)
            p1 = rng.standard_normal(s)
            svd.add_rows(E, approx=L.Approx("gkl", 10, 1, p1))
            ref = approx.add_rows(U0, s0, V0, E, method="gkl", l=10, start=p1)
        _check(svd, U0, s0, V0, ref, prec)
    finally:
        svd.close()
