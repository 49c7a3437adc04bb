"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each mutant below is the oracle's add-rows / add-columns / weight update with
one plausible slip (a dropped term, a wrong sign, a transposed operand, a
wrong factor).  The brute-force pin (a dense SVD of the updated matrix) or the
energy pin must reject every one; the unmutated oracle passes both (see
test_oracle_pins).  Mistakes are planted on the CPU only.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import brute, metrics, zha_simon
from synth import small_case


def _rows(U, s, V, E, mutation):
    k = s.size
    Es = E.to_scipy()
    C = np.asarray((Es @ V)).T
    if mutation == "wrong_sign_Z":
        Z = Es.T.toarray() + V @ C
    else:
        Z = Es.T.toarray() - V @ C
    Q, R = np.linalg.qr(Z)
    if mutation == "drop_EV_block":
        C = np.zeros_like(C)
    K = np.zeros((k + C.shape[1], k + R.shape[0]))
    K[:k, :k] = np.diag(s)
    K[k:, :k] = C.T
    K[k:, k:] = R if mutation == "R_not_transposed" else R.T
    F, th, Gt = np.linalg.svd(K)
    F, th, G = F[:, :k], th[:k], Gt[:k].T
    top = U @ F[:k]
    if mutation == "U_new_uses_G":
        top = U @ G[:k]
    Un = np.vstack([top, F[k:]])
    Vn = np.hstack([V, Q]) @ (F if mutation == "V_new_uses_F" else G)
    return Un, th, Vn, np.linalg.svd(K, compute_uv=False)


def _weights(U, s, V, D_T, Em_T, mutation):
    k = s.size
    CD, QD, RD, _ = zha_simon.augmented_qr(D_T.to_scipy().T, U)
    CE, QE, RE, _ = zha_simon.augmented_qr(Em_T.to_scipy().T, V)
    X = np.vstack([CD, RD]); Y = np.vstack([CE, RE])
    K = X @ Y.T
    if mutation != "drop_sigma":
        K[:k, :k] += np.diag(s)
    if mutation == "swap_XY":
        K = Y[:X.shape[0]] @ X[:Y.shape[0]].T + np.pad(np.diag(s), ((0, X.shape[0] - k), (0, Y.shape[0] - k)))
    F, th, Gt = np.linalg.svd(K, full_matrices=False)
    Un = np.hstack([U, QD]) @ F[:, :k]
    Vn = np.hstack([V, QE]) @ Gt[:k].T
    return Un, th[:k], Vn, th


def _caught(test, ref, theta_hat, energy_ok):
    r = metrics.compare(test, ref, theta_hat, 1e-8)
    bad = (r["sigma_rel"] > 1e-9 or r["angle_U"] > 1e-7 or r["angle_V"] > 1e-7
           or r["orth_U"] > 1e-9 or r["orth_V"] > 1e-9 or not energy_ok)
    return bad, r


@pytest.mark.parametrize("mutation", ["drop_EV_block", "wrong_sign_Z",
                                      "R_not_transposed", "U_new_uses_G",
                                      "V_new_uses_F"])
def test_rows_mutants_are_caught(mutation):
    rng = np.random.default_rng(5)
    c = small_case(rng, 40, 30, 5, 6, kind="rows", density=0.3)
    U, s, V, E = c["U"], c["s"], c["V"], c["E"]
    U0, s0, V0, i0 = brute.apply(U, s, V, ("rows", E))
    Um, sm, Vm, spec = _rows(U, s, V, E, mutation)
    energy_ok = abs(np.sum(spec ** 2) - (np.sum(s ** 2) + np.sum(E.val ** 2))) < 1e-10 * np.sum(s ** 2)
    bad, r = _caught((Um, sm, Vm), (U0, s0, V0), i0["theta_hat"], energy_ok)
    assert bad, (mutation, r)
    # and the unmutated copy passes the same gate
    Uo, so, Vo, speco = _rows(U, s, V, E, None)
    ok_energy = abs(np.sum(speco ** 2) - (np.sum(s ** 2) + np.sum(E.val ** 2))) < 1e-10 * np.sum(s ** 2)
    assert not _caught((Uo, so, Vo), (U0, s0, V0), i0["theta_hat"], ok_energy)[0]


@pytest.mark.parametrize("mutation", ["drop_sigma", "swap_XY"])
def test_weights_mutants_are_caught(mutation):
    rng = np.random.default_rng(6)
    c = small_case(rng, 30, 30, 4, 5, kind="weights", density=0.3)
    U, s, V = c["U"], c["s"], c["V"]
    up = ("weights", c["D_T"], c["Em_T"])
    U0, s0, V0, i0 = brute.apply(U, s, V, up)
    Um, sm, Vm, _ = _weights(U, s, V, c["D_T"], c["Em_T"], mutation)
    bad, r = _caught((Um, sm, Vm), (U0, s0, V0), i0["theta_hat"], True)
    assert bad, (mutation, r)
