"""Seeded generators: determinism and the distributional shape of each
workload (CPU only, small sizes)."""
import numpy as np

from synth import (CSR, bernoulli_uniform, chung_lu_graph, chung_lu_weights,
                   config1_rows, random_orthonormal, zipf_ratings)


def _same(a: CSR, b: CSR):
    return (np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
            and np.array_equal(a.val, b.val))


def test_bernoulli_density_and_determinism():
    a = bernoulli_uniform(400, 300, 0.02, np.random.default_rng(3))
    b = bernoulli_uniform(400, 300, 0.02, np.random.default_rng(3))
    assert _same(a, b)
    assert abs(a.nnz / (400 * 300) - 0.02) < 0.003
    assert a.val.min() > 0 and a.val.max() <= 1.0
    # canonical: sorted unique columns per row
    for i in range(a.rows):
        c = a.col_idx[a.row_ptr[i]:a.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_chung_lu_shape():
    w = chung_lu_weights(100000, 2.1, 20.0)
    assert w.max() <= np.sqrt(w.sum()) * (1 + 1e-9)
    g = chung_lu_graph(20000, 2.1, 20.0, np.random.default_rng(4))
    S = g.to_scipy()
    assert (S != S.T).nnz == 0 and S.diagonal().sum() == 0
    deg = np.diff(g.row_ptr)
    assert 15 < deg.mean() < 21
    # heavy tail: the largest degree is far above the mean
    assert deg.max() > 20 * deg.mean()


def test_zipf_ratings_shape():
    r = zipf_ratings(20000, 5000, 200000, 1.1, np.random.default_rng(5))
    assert r.nnz == 200000
    vals, cnt = np.unique(r.val, return_counts=True)
    assert set(vals.tolist()) == {1.0, 2.0, 3.0, 4.0, 5.0}
    np.testing.assert_allclose(cnt / cnt.sum(), [0.1, 0.1, 0.2, 0.3, 0.3], atol=0.01)
    colcnt = np.bincount(r.col_idx, minlength=5000)
    assert colcnt.max() > 0.05 * r.nnz         # a hot item holds >5% of draws


def test_orthonormal_and_config1():
    Q = random_orthonormal(50, 7, np.random.default_rng(6))
    np.testing.assert_allclose(Q.T @ Q, np.eye(7), atol=1e-14)
    c1 = config1_rows(steps=2)
    c2 = config1_rows(steps=2)
    assert _same(c1["updates"][1][1], c2["updates"][1][1])
    assert c1["U"].shape == (2000, 16) and c1["V"].shape == (1000, 16)
