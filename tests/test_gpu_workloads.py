"""GPU parity on the workload generators at reduced sizes (the same code
paths and update shapes as the benchmark workloads, small enough for the
oracle): lock-step against the FP64 oracle (Zha-Simon) after every update.

- graph: Chung-Lu adjacency (gamma 2.1), k = 64, nodes appended as
  add_cols(A[old, new]) then add_rows(A[new, old + new]);
- ratings: Zipf(1.1) user-item ratings 1..5, k = 128, user-row appends
  (hot columns make E E^T dense, light users give duplicate rows);
- weights: LogNormal-weighted Chung-Lu graph, k = 64, rank-32 weight updates
  A + D E_m^T with D = I[:, R] for degree-biased rows R.

Tolerances as in test_gpu_parity (sigma 1e-5 / angles 1e-4 in the FP32 and
BF16x3 modes).
"""
import numpy as np
import pytest

from oracle import metrics, zha_simon

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(sig=1e-10, ang=1e-8, delta=1e-6, orth=1e-11),
       "fp32": dict(sig=1e-5, ang=1e-4, delta=1e-3, orth=1e-5),
       "bf16x3": dict(sig=1e-5, ang=1e-4, delta=1e-3, orth=5e-5)}


def _run(cfg, prec, nup, capU, capV):
    import paper_2401_09703_amd as L
    svd = L.TruncatedSVD(cfg["U"], cfg["s"], cfg["V"], precision=prec,
                         row_capacity=capU, col_capacity=capV)
    t = TOL[prec]
    try:
        for j, up in enumerate(cfg["updates"][:nup]):
            U0, s0, V0 = svd.factors()
            svd.apply(up)
            svd.sync()
            U1, s1, V1 = svd.factors()
            Ur, sr, Vr, info = zha_simon.apply(U0, s0, V0, up)
            r = metrics.compare((U1, s1, V1), (Ur, sr, Vr), info["theta_hat"], t["delta"])
            print(cfg["name"], prec, j, {k: (f"{v:.2e}" if isinstance(v, float) else v)
                                         for k, v in r.items()}, flush=True)
            assert r["sigma_rel"] <= t["sig"], r
            assert r["angle_U"] <= t["ang"] and r["angle_V"] <= t["ang"], r
            assert r["orth_U"] <= t["orth"] and r["orth_V"] <= t["orth"], r
    finally:
        svd.close()


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp64"])
def test_graph_workload(prec):
    from synth import config2_graph
    cfg = config2_graph(k=64, n_init=6000, step_nodes=300, steps=2, power=2)
    _run(cfg, prec, 4, 6600 + 16, 6600 + 16)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_ratings_workload(prec):
    from synth import config3_ratings
    cfg = config3_ratings(users=12000, items=3000, nnz=240_000, init_users=10000, k=128,
                          steps=2, s=600)
    _run(cfg, prec, 2, 12000 + 16, 3000 + 16)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_weights_workload(prec):
    from synth import config4_weights
    cfg = config4_weights(N=20000, k=64, steps=2, s=32, perturbed=2000, added=400)
    _run(cfg, prec, 2, 20000 + 16, 20000 + 16)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_ratings_workload_large_n(prec):
    """k + s = 1928: past the size at which the residual Gram's Cholesky and
    the tridiagonalisation keep their rows on chip, so the large-N branches
    of both run, lock-step against the oracle."""
    from synth import config3_ratings
    cfg = config3_ratings(users=12000, items=4000, nnz=240_000, init_users=10000, k=128,
                          steps=1, s=1800)
    assert cfg["k"] + cfg["updates"][0][1].rows > 1745
    _run(cfg, prec, 1, 12000 + 16, 4000 + 16)
