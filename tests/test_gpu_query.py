"""GPU parity of batched Query(i) and the pair scores against O4 on the
factors the GPU holds (realised in FP64): FP64 storage to 1e-12, FP32
storage to 1e-6 relative to the largest score; out-of-range indices give
NaN; the realised factors follow an update."""
import numpy as np
import pytest

from oracle import query
from synth import small_case

pytestmark = pytest.mark.gpu


def _L():
    import paper_2401_09703_amd as L
    return L


@pytest.mark.parametrize("prec,k", [("fp64", 16), ("fp32", 32), ("bf16x3", 64), ("fp64", 128),
                                    ("bf16x3", 128), ("fp32", 16)])
def test_scores_and_queries(prec, k):
    L = _L()
    rng = np.random.default_rng(k + len(prec))
    c = small_case(rng, 700, 520, k, 40, kind="rows", density=0.05)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision=prec)
    tol = 1e-12 if prec == "fp64" else 1e-6
    try:
        svd.apply(("rows", c["E"]))      # a non-identity W on both sides
        svd.sync()
        U, s, V = svd.factors()
        m, n = U.shape[0], V.shape[0]
        for both in (False, True):
            top = min(m, n) if both else None
            i = rng.integers(0, top or m, 5003)
            j = rng.integers(0, top or n, 5003)
            got = svd.score_pairs(i, j, both=both).cpu().numpy()
            ref = query.score_pairs(U, s, V, i, j, both=both)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err <= tol, (prec, k, both, err)
        for side, X in ((0, U), (1, V)):
            idx = rng.integers(0, X.shape[0], 777)
            got = svd.query_rows(side, idx).cpu().numpy()
            ref = query.query_rows(X, idx)
            assert np.abs(got - ref).max() <= tol * max(np.abs(ref).max(), 1.0), (prec, side)
    finally:
        svd.close()


def test_out_of_range_and_refresh_after_update():
    L = _L()
    rng = np.random.default_rng(9)
    c = small_case(rng, 300, 200, 16, 20, kind="rows", density=0.1)
    svd = L.TruncatedSVD(c["U"], c["s"], c["V"], precision="fp64")
    try:
        got = svd.score_pairs([0, 299, 300, -1, 5], [0, 199, 3, 2, 200]).cpu().numpy()
        assert np.isfinite(got[:2]).all() and np.isnan(got[2:]).all()
        q = svd.query_rows(1, [0, 200, 5]).cpu().numpy()
        assert np.isfinite(q[0]).all() and np.isnan(q[1]).all() and np.isfinite(q[2]).all()
        before = svd.score_pairs([1, 2, 3], [4, 5, 6]).cpu().numpy()
        svd.apply(("rows", c["E"]))
        after = svd.score_pairs([1, 2, 3, 310], [4, 5, 6, 7]).cpu().numpy()
        U, s, V = svd.factors()
        ref = query.score_pairs(U, s, V, [1, 2, 3, 310], [4, 5, 6, 7])
        np.testing.assert_allclose(after, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert not np.allclose(before, after[:3])
        assert len(svd.score_pairs([], [])) == 0
    finally:
        svd.close()
