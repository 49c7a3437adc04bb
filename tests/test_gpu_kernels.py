"""Kernel-level GPU parity: the FP64 top-k symmetric eigensolver behind the
(k+s) Rayleigh-Ritz SVD, against LAPACK on the CPU (numpy.linalg.eigh).

Eigenvalues are compared elementwise (relative to the largest); eigenvectors
through the principal angle of the leading block up to a spectral gap.  Cases
cover tiny N (1, 2, 3), ragged sizes around the 64-lane tiles, repeated and
clustered eigenvalues, a rank-deficient PSD matrix, the zero matrix, and the
sizes of the graph (N = 1064) and ratings (N = 5128) workloads.
"""
import numpy as np
import pytest

from oracle import metrics

pytestmark = pytest.mark.gpu


def _run(M, k):
    import torch
    import paper_2401_09703_amd as L
    Mt = torch.from_numpy(np.ascontiguousarray(M)).cuda()
    lam, vecs = L.sym_eig_topk(Mt, k)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), vecs.cpu().numpy()


def _check(M, k, tol_val=1e-12, tol_ang=1e-9, delta=1e-6):
    lam, V = _run(M, k)
    w, Q = np.linalg.eigh(M)
    w, Q = w[::-1], Q[:, ::-1]
    scale = max(abs(w[0]), abs(w[-1]), 1e-300)
    err = np.max(np.abs(lam - w[:k])) / scale
    assert err <= tol_val, err
    # orthonormal rows
    assert np.linalg.norm(V @ V.T - np.eye(k), 2) <= 1e-11
    # residual ||M v - lam v|| relative to ||M||
    res = np.max(np.linalg.norm(M @ V.T - V.T * lam, axis=0)) / scale
    assert res <= 1e-11, res
    j = metrics.gap_prefix(np.abs(w), k, delta) if np.all(w >= -1e-12 * scale) else 0
    if j:
        assert metrics.sin_angle(V[:j].T, Q[:, :j]) <= tol_ang
    return err


@pytest.mark.parametrize("N,k", [(1, 1), (2, 1), (2, 2), (3, 2), (4, 4), (16, 16), (63, 16),
                                 (65, 32), (100, 100), (127, 64), (128, 128), (130, 64),
                                 (257, 64), (1064, 64)])
def test_random_psd(N, k):
    rng = np.random.default_rng(N * 31 + k)
    X = rng.standard_normal((N, N + 3))
    _check(X @ X.T / N, k)


def test_graph_like_spectrum_with_clusters():
    rng = np.random.default_rng(3)
    N, k = 600, 64
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    w = np.concatenate([[5e4], 1000 + np.sort(rng.uniform(0, 400, 80))[::-1],
                        rng.uniform(0, 900, N - 81)])
    w[10] = w[11] = w[12]          # an exactly repeated eigenvalue in the top k
    M = (Q * w) @ Q.T
    _check((M + M.T) / 2, k, tol_val=1e-12, tol_ang=1e-8)


def test_rank_deficient_and_zero():
    rng = np.random.default_rng(4)
    N, k = 200, 32
    X = rng.standard_normal((N, 10))
    lam, V = _run(X @ X.T, k)
    w = np.linalg.eigvalsh(X @ X.T)[::-1]
    assert np.max(np.abs(lam - w[:k])) <= 1e-11 * w[0]
    assert np.linalg.norm(V @ V.T - np.eye(k), 2) <= 1e-10
    lam0, V0 = _run(np.zeros((50, 50)), 8)
    assert np.all(np.abs(lam0) <= 1e-300) and np.linalg.norm(V0 @ V0.T - np.eye(8)) <= 1e-12


def test_ratings_size():
    rng = np.random.default_rng(5)
    N, k = 5128, 128
    X = rng.standard_normal((N, 300))
    M = X @ X.T
    M += np.diag(rng.uniform(0, 1, N))
    _check(M, k, tol_val=1e-11, tol_ang=1e-8)


@pytest.mark.parametrize("N,r", [(16, 6), (32, 3), (64, 10), (128, 6)])
def test_rank_deficient_grams_of_tall_panels(N, r):
    """Grams W^T W of tall rank-r panels (as in the initial SVD's l x l
    problem): the top-k vectors include a cluster of rounding-level
    eigenvalues, whose vectors must still come out orthonormal."""
    for seed in range(4):
        rng = np.random.default_rng(1000 * N + 10 * r + seed)
        W = rng.standard_normal((3000, r)) @ rng.standard_normal((r, N))
        M = W.T @ W
        k = 3 * N // 4
        lam, V = _run(M, k)
        w = np.linalg.eigvalsh(M)[::-1]
        assert np.max(np.abs(lam - w[:k])) <= 1e-11 * w[0]
        assert np.linalg.norm(V @ V.T - np.eye(k), 2) <= 1e-10
        res = np.max(np.linalg.norm(M @ V.T - V.T * lam, axis=0)) / w[0]
        assert res <= 1e-11
