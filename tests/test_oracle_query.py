"""Pins of O4 (queries and scores): for a matrix of rank <= k the scores are
the matrix entries themselves, whatever factorisation represents it; the
undirected score is symmetric and never below either direction; Query
returns the factor's rows."""
import numpy as np

from oracle import query


def _rank_k(rng, m, n, k):
    A = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    return A, U[:, :k], s[:k], Vt[:k].T


def test_scores_are_matrix_entries_for_rank_k():
    rng = np.random.default_rng(4)
    A, U, s, V = _rank_k(rng, 40, 30, 5)
    i = rng.integers(0, 40, 500)
    j = rng.integers(0, 30, 500)
    np.testing.assert_allclose(query.score_pairs(U, s, V, i, j), A[i, j], rtol=0, atol=1e-11)


def test_undirected_score_is_the_max_of_both_directions():
    rng = np.random.default_rng(5)
    A, U, s, V = _rank_k(rng, 25, 25, 4)
    i = rng.integers(0, 25, 300)
    j = rng.integers(0, 25, 300)
    b = query.score_pairs(U, s, V, i, j, both=True)
    np.testing.assert_allclose(b, np.maximum(A[i, j], A[j, i]), atol=1e-11)
    np.testing.assert_array_equal(b, query.score_pairs(U, s, V, j, i, both=True))


def test_query_rows():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((12, 3))
    np.testing.assert_array_equal(query.query_rows(X, [4, 0, 11]), X[[4, 0, 11]])
