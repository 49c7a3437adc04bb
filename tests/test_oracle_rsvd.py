"""Pins of O5 (randomised initial SVD): exact on a matrix of rank <= k, and
within the randomised method's error of the LAPACK SVD on a matrix with a
fast-decaying spectrum; orthonormal factors; a planted mistake (no power
iteration on a slowly decaying spectrum, or V taken from the wrong side)
is caught by the comparison with LAPACK."""
import numpy as np
import scipy.sparse as sp

from oracle import metrics, rsvd


def _lowrank_sparse(rng, m, n, r, dens):
    # a sparse matrix of rank r: r sparse rank-one terms
    A = sp.csr_matrix((m, n))
    for _ in range(r):
        u = sp.random(m, 1, density=0.3, random_state=rng)
        v = sp.random(1, n, density=dens, random_state=rng)
        A = A + u @ v * rng.uniform(1, 10)
    return sp.csr_matrix(A)


def test_exact_on_rank_k():
    rng = np.random.default_rng(1)
    A = _lowrank_sparse(rng, 300, 200, 6, 0.2)
    U, s, V = rsvd.rsvd(A, 8, rng.standard_normal((200, 16)), power=1)
    np.testing.assert_allclose((U * s) @ V.T, A.toarray(), atol=1e-10 * abs(A).max())
    assert np.abs(U.T @ U - np.eye(8)).max() < 1e-12 and np.abs(V.T @ V - np.eye(8)).max() < 1e-12


def test_close_to_lapack_on_fast_decay():
    rng = np.random.default_rng(2)
    m, n, k = 400, 300, 10
    X = np.linalg.qr(rng.standard_normal((m, n)))[0]
    Y = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sv = 2.0 ** -np.arange(n)
    A = sp.csr_matrix((X * sv) @ Y.T)
    U, s, V = rsvd.rsvd(A, k, rng.standard_normal((n, 2 * k)), power=2)
    Ul, sl, Vlt = np.linalg.svd(A.toarray(), full_matrices=False)
    assert metrics.sigma_rel_err(s, sl[:k]) < 1e-10
    assert metrics.sin_angle(U, Ul[:, :k]) < 1e-8 and metrics.sin_angle(V, Vlt[:k].T) < 1e-8


def test_planted_mistakes_are_caught():
    rng = np.random.default_rng(3)
    m, n, k = 300, 250, 8
    X = np.linalg.qr(rng.standard_normal((m, n)))[0]
    Y = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sv = 1.0 / (1.0 + np.arange(n)) ** 0.5            # slow decay
    A = sp.csr_matrix((X * sv) @ Y.T)
    Om = rng.standard_normal((n, 2 * k))
    Ul, sl, Vlt = np.linalg.svd(A.toarray(), full_matrices=False)
    U, s, V = rsvd.rsvd(A, k, Om, power=8)
    good = metrics.sigma_rel_err(s, sl[:k])
    U0, s0, V0 = rsvd.rsvd(A, k, Om, power=0)           # mistake: no power iteration
    assert metrics.sigma_rel_err(s0, sl[:k]) > 10 * good
    # mistake: right factor from the wrong side
    assert metrics.sin_angle(U[:V.shape[0]], Vlt[:k].T) > 1e-3


def test_planted_transposed_operand_is_caught():
    """A copy of the oracle whose power step multiplies by A where A^T is
    due (a transposed operand) drifts away from LAPACK's subspaces on a
    non-symmetric matrix with a decaying spectrum."""
    rng = np.random.default_rng(4)
    m, n, k = 260, 260, 6
    X = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Y = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sv = 0.8 ** np.arange(n)
    A = (X * sv) @ Y.T                      # non-symmetric, left and right bases differ
    Om = rng.standard_normal((n, 2 * k))
    Ul, sl, Vlt = np.linalg.svd(A, full_matrices=False)

    def mutated(A, k, Om, power):
        Q = np.linalg.qr(A @ Om)[0]
        for _ in range(power):
            Z = np.linalg.qr(A @ Q)[0]      # mistake: A instead of A^T
            Q = np.linalg.qr(A @ Z)[0]
        B = (A.T @ Q).T
        Ub, s, Vbt = np.linalg.svd(B, full_matrices=False)
        return Q @ Ub[:, :k], s[:k], Vbt[:k].T

    U, s, V = rsvd.rsvd(A, k, Om, power=4)
    Um, sm, Vm = mutated(A, k, Om, 4)
    good = metrics.sin_angle(U, Ul[:, :k])
    bad = metrics.sin_angle(Um, Ul[:, :k])
    assert good < 1e-3 and bad > 10 * good


def _spectrum_matrix(rng, m, n, sv):
    X = np.linalg.qr(rng.standard_normal((m, n)))[0]
    Y = np.linalg.qr(rng.standard_normal((n, n)))[0]
    return sp.csr_matrix((X * sv) @ Y.T)


def test_within_the_power_scheme_error_bound():
    """Halko, Martinsson and Tropp (2011), the power-scheme bound: with l =
    k + p test vectors and q power iterations, except with probability at
    most 6 p^-p, ||(I - Q Q^T) A|| <= (1 + 11 sqrt(k + p) sqrt(min(m, n)))^(1/(2q+1))
    sigma_{k+1}; truncating Q^T A to rank k adds at most sigma_{k+1}.  Checked
    against sigma_{k+1} of the LAPACK SVD over several test matrices, with a
    spectrum where the bound is far below sigma_1 (so a range finder that
    ignores A fails it)."""
    rng = np.random.default_rng(6)
    m, n, k, p = 500, 400, 10, 10
    sv = 0.7 ** np.arange(n)
    A = _spectrum_matrix(rng, m, n, sv)
    Ad = A.toarray()
    s_exact = np.linalg.svd(Ad, compute_uv=False)
    for q in (0, 1, 2):
        bound = ((1 + 11 * np.sqrt(k + p) * np.sqrt(min(m, n))) ** (1 / (2 * q + 1)) + 1) * s_exact[k]
        assert bound < 0.5 * s_exact[0] or q == 0
        for trial in range(3):
            U, s, V = rsvd.rsvd(A, k, rng.standard_normal((n, k + p)), power=q)
            err = np.linalg.norm(Ad - (U * s) @ V.T, 2)
            assert s_exact[k] * (1 - 1e-12) <= err <= bound
    # a basis that ignores A: same shapes, error of order sigma_1
    Qr = np.linalg.qr(rng.standard_normal((m, k)))[0]
    err_r = np.linalg.norm(Ad - Qr @ (Qr.T @ Ad), 2)
    q1 = ((1 + 11 * np.sqrt(k + p) * np.sqrt(min(m, n))) ** (1 / 3) + 1) * s_exact[k]
    assert err_r > q1
