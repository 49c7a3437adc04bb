"""Bitwise reproducibility of the update path: the same updates applied to
two states built from the same factors give bitwise equal factors.  The
sparse Gram sums each entry in a fixed order and the sparse row update sorts
the nonzeros by column and sums each base row's terms in row order (no
floating-point atomics), the Cholesky and the triangular solve give each
tile one writer, and the subspace iteration draws its start from the update's
sequence number.  The inputs have real-valued entries and update rows that
share most of their columns, so that an accumulation whose order depended on
scheduling would round differently between runs."""
import numpy as np
import pytest

from synth import synthetic_factors
from synth.sparse import CSR

pytestmark = pytest.mark.gpu


def _L():
    import paper_2401_09703_amd as L
    return L


def _hub_update(rng, s, width, hubs=12, density=0.05):
    """s rows over `width` columns: every row touches most of `hubs` shared
    columns plus a sparse random rest; values are real (not integers)."""
    E = np.zeros((s, width))
    hub_cols = rng.choice(width, size=hubs, replace=False)
    for i in range(s):
        on = hub_cols[rng.random(hubs) < 0.8]
        E[i, on] = rng.uniform(0.1, 2.0, size=on.size)
        rest = rng.random(width) < density
        E[i, rest] = rng.uniform(-1.0, 1.0, size=int(rest.sum()))
    return CSR.from_dense(E)


def _run(L, U, s, V, ups, prec, deterministic=True, side_stream=True):
    svd = L.TruncatedSVD(U, s, V, precision=prec, deterministic=deterministic,
                         side_stream=side_stream)
    try:
        for up in ups:
            svd.apply(up)
        svd.sync()
        return svd.factors()
    finally:
        svd.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_update_sequence_is_bitwise_reproducible(prec):
    L = _L()
    rng = np.random.default_rng(404)
    m, n, k = 700, 500, 32
    U, s, V = synthetic_factors(m, n, k, rng)
    ups = [("rows", _hub_update(rng, 150, n)),
           ("cols", _hub_update(rng, 90, m + 150)),
           ("weights", _hub_update(rng, 24, m + 150), _hub_update(rng, 24, n + 90)),
           ("rows", _hub_update(rng, 300, n + 90))]
    a = _run(L, U, s, V, ups, prec)
    b = _run(L, U, s, V, ups, prec)
    for x, y, name in zip(a, b, "UsV"):
        assert x.shape == y.shape
        assert np.array_equal(x, y), (prec, name, float(np.max(np.abs(x - y))))


def test_atomic_row_update_matches_the_ordered_one():
    """deterministic=False (atomic accumulation) agrees with the ordered sum
    to rounding."""
    L = _L()
    rng = np.random.default_rng(405)
    m, n, k = 600, 400, 16
    U, s, V = synthetic_factors(m, n, k, rng)
    ups = [("rows", _hub_update(rng, 200, n)), ("cols", _hub_update(rng, 60, m + 200))]
    Ua, sa, Va = _run(L, U, s, V, ups, "fp64", deterministic=True)
    Ub, sb, Vb = _run(L, U, s, V, ups, "fp64", deterministic=False)
    assert np.max(np.abs(sa - sb)) <= 1e-10 * sa[0]
    # factors agree up to sign per column
    for A, B in ((Ua, Ub), (Va, Vb)):
        sg = np.sign(np.sum(A * B, axis=0))
        assert np.max(np.abs(A - B * sg)) <= 1e-8


def test_large_update_takes_the_sorted_row_update_bitwise():
    """An update with more than 32k nonzeros: the row update goes through the
    stable radix sort by column; still bitwise reproducible."""
    L = _L()
    rng = np.random.default_rng(406)
    m, n, k = 900, 800, 32
    U, s, V = synthetic_factors(m, n, k, rng)
    E = _hub_update(rng, 1200, n, hubs=16, density=0.04)
    assert E.nnz > 32768
    ups = [("rows", E)]
    a = _run(L, U, s, V, ups, "fp32")
    b = _run(L, U, s, V, ups, "fp32")
    for x, y, name in zip(a, b, "UsV"):
        assert np.array_equal(x, y), (name, float(np.max(np.abs(x - y))))


@pytest.mark.parametrize("prec,k", [("fp32", 32), ("bf16x3", 64), ("bf16x3", 128)])
def test_second_stream_gives_the_one_stream_factors(prec, k):
    """An append update with the residual Gram's Cholesky on the state's
    second stream (side_stream=True) gives bitwise the factors of the same
    updates on one stream: the two streams split independent work and every
    product keeps its order."""
    L = _L()
    rng = np.random.default_rng(407 + k)
    m, n = 900, 700
    U, s, V = synthetic_factors(m, n, k, rng)
    ups = [("rows", _hub_update(rng, 220, n)),
           ("cols", _hub_update(rng, 180, m + 220)),
           ("weights", _hub_update(rng, 200, m + 220), _hub_update(rng, 200, n + 180))]
    a = _run(L, U, s, V, ups, prec, side_stream=True)
    b = _run(L, U, s, V, ups, prec, side_stream=False)
    for x, y, name in zip(a, b, "UsV"):
        assert x.shape == y.shape
        assert np.array_equal(x, y), (prec, k, name, float(np.max(np.abs(x - y))))


@pytest.mark.parametrize("k", [32, 128])
def test_hot_column_runs_split_over_a_block(k):
    """Columns with more than 256 nonzeros in one update (a power-law hot
    column) are summed by a whole block in fixed pieces: bitwise
    reproducible, and equal to the atomic accumulation to rounding."""
    L = _L()
    rng = np.random.default_rng(408 + k)
    m, n = 900, 800
    U, s, V = synthetic_factors(m, n, k, rng)
    E = _hub_update(rng, 3000, n, hubs=4, density=0.02)
    col_counts = np.bincount(E.col_idx, minlength=n)
    assert E.nnz > 32768 and col_counts.max() > 2048
    ups = [("rows", E)]
    a = _run(L, U, s, V, ups, "fp32")
    b = _run(L, U, s, V, ups, "fp32")
    for x, y, name in zip(a, b, "UsV"):
        assert np.array_equal(x, y), (name, float(np.max(np.abs(x - y))))
    Ua, sa, Va = _run(L, U, s, V, ups, "fp64", deterministic=True)
    Ub, sb, Vb = _run(L, U, s, V, ups, "fp64", deterministic=False)
    assert np.max(np.abs(sa - sb)) <= 1e-10 * sa[0]
    for A, B in ((Ua, Ub), (Va, Vb)):
        sg = np.sign(np.sum(A * B, axis=0))
        assert np.max(np.abs(A - B * sg)) <= 1e-8
