"""The allocation-free eigensolver entry point (svlcov_sym_eig_topk_noalloc)
against the allocating one (svlcov_sym_eig_topk), through the C ABI.

Both run the same kernels on the same input, so the results must agree to
rounding (compared elementwise: eigenvalues relative to the largest,
eigenvectors entry by entry; the sign convention is the same on both
sides).  Two calls in a row, the second with a smaller matrix, check that
the shared per-GPU workspace carries nothing from one call to the next; a
size beyond the workspace is refused before any device work.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _psd(N, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, N + 5))
    M = X @ X.T / N
    return M


def _both(M, k):
    import torch
    import paper_2401_09703_amd as L
    Mt = torch.from_numpy(np.ascontiguousarray(M)).cuda()
    lam_a, vec_a = L.sym_eig_topk(Mt, k)
    lam_b = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    vec_b = torch.full((k, M.shape[0]), float("nan"), dtype=torch.float64, device="cuda")
    L.sym_eig_topk_noalloc(Mt, k, lam_b, vec_b)
    torch.cuda.synchronize()
    return (lam_a.cpu().numpy(), vec_a.cpu().numpy(), lam_b.cpu().numpy(),
            vec_b.cpu().numpy())


def _agree(M, k):
    la, va, lb, vb = _both(M, k)
    scale = max(abs(la[0]), 1e-300)
    assert np.all(np.isfinite(lb)) and np.all(np.isfinite(vb))
    assert np.max(np.abs(la - lb)) / scale <= 1e-13
    assert np.max(np.abs(va - vb)) <= 1e-11
    # and both are eigenpairs of M
    w = np.linalg.eigvalsh(M)[::-1][:k]
    assert np.max(np.abs(lb - w)) / max(abs(w[0]), 1e-300) <= 1e-12


def test_noalloc_matches_allocating_entry_two_calls():
    _agree(_psd(1064, 1), 64)     # the graph workload's size, several tiles
    _agree(_psd(301, 2), 32)      # smaller second call: ragged, one-block path above 128
    _agree(_psd(97, 3), 16)       # the one-block small path


def test_noalloc_rejects_sizes_beyond_the_workspace():
    import torch
    import paper_2401_09703_amd as L
    lib = L._lib
    big = 2048                    # 32 MiB for the copy of M alone
    lam = torch.empty(64, dtype=torch.float64, device="cuda")
    vec = torch.empty((64, 4), dtype=torch.float64, device="cuda")
    M = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    rc = lib.svlcov_sym_eig_topk_noalloc(big, M.data_ptr(), 64, lam.data_ptr(),
                                         vec.data_ptr(), None)
    assert rc == 7  # SVLCOV_E_UNSUPPORTED, nothing launched
    assert lib.svlcov_sym_eig_topk_noalloc(4, M.data_ptr(), 5, lam.data_ptr(),
                                           vec.data_ptr(), None) == 1
