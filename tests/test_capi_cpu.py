"""The C-ABI library loads on a machine without a GPU, exports every entry
point declared in include/svlcov.h, and rejects bad arguments before touching
the device (CPU only; no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svlcov.h")


def _declared():
    txt = open(HEADER).read()
    decl = r"^\s*(?:svlcov_status|void\s*\*|void|int32_t|const\s+char\s*\*)\s*(svlcov_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("svlcov_init", "svlcov_add_rows", "svlcov_add_cols", "svlcov_update_weights",
              "svlcov_get_factors", "svlcov_sync", "svlcov_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2401_09703_amd as L
    lib = C.CDLL(L.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) <= set(_declared())


def test_status_strings_and_defaults():
    import paper_2401_09703_amd as L
    lib = L._lib
    assert lib.svlcov_status_str(0) == b"ok"
    assert lib.svlcov_status_str(2) == b"shape mismatch"
    opt = L._Options()
    lib.svlcov_default_options(C.byref(opt))
    assert opt.precision == 0 and opt.validate_device_inputs == 1 and opt.stream is None
    assert opt.deterministic == 1 and opt.side_stream == 1


def test_init_rejects_bad_arguments_before_device_use():
    import paper_2401_09703_amd as L
    lib = L._lib
    h = C.c_void_p()
    U = np.zeros((4, 16)); V = np.zeros((3, 16)); s = np.ones(16)
    # unsupported k
    assert lib.svlcov_init(C.byref(h), 4, 3, 7, U.ctypes.data, s[:7].ctypes.data,
                           V.ctypes.data, 0, None) == 7
    # increasing sigma
    bad = np.arange(16, dtype=np.float64)
    assert lib.svlcov_init(C.byref(h), 4, 3, 16, U.ctypes.data, bad.ctypes.data,
                           V.ctypes.data, 0, None) == 1
    # non-finite factor
    U2 = U.copy(); U2[0, 0] = np.nan
    assert lib.svlcov_init(C.byref(h), 4, 3, 16, U2.ctypes.data, s.ctypes.data,
                           V.ctypes.data, 0, None) == 4
    assert not h.value
    # NULL state handles
    assert lib.svlcov_sync(None) == 1
    assert lib.svlcov_add_rows(None, None) == 1


def test_rsvd_rejects_bad_arguments_before_device_use():
    import paper_2401_09703_amd as L
    lib = L._lib
    rp = np.zeros(41, np.int64)
    keep = []
    A = L._csr_struct(type("M", (), dict(rows=40, cols=30, row_ptr=rp,
                                         col_idx=np.zeros(0, np.int32),
                                         val=np.zeros(0)))(), keep)
    buf = np.zeros(64)
    p = buf.ctypes.data
    call = lambda k, l, power, csr=A: lib.svlcov_rsvd(C.byref(csr), k, l, power, p, p, p, p,
                                                      None, None)
    assert call(8, 48, 1) == 7          # l outside {16, 32, 64, 128}
    assert call(20, 16, 1) == 1         # k > l
    assert call(8, 16, -1) == 1         # negative power
    assert call(8, 32, 1) == 2          # l > min(m, n)
    assert lib.svlcov_rsvd(None, 8, 16, 1, p, p, p, p, None, None) == 1
    A.val_dtype = 5
    assert call(8, 16, 1) == 1


def test_server_rejects_bad_arguments_before_device_use():
    import paper_2401_09703_amd as L
    lib = L._lib
    opt = L._ServerOptions()
    lib.svlcov_server_default_options(C.byref(opt))
    assert opt.max_inflight == 8 and opt.workspace_budget == 8 << 30
    h = C.c_void_p()
    opt.max_inflight = 0
    assert lib.svlcov_server_create(C.byref(h), C.byref(opt)) == 1
    opt.max_inflight = 65
    assert lib.svlcov_server_create(C.byref(h), C.byref(opt)) == 1
    assert not h.value
    t = C.c_int64()
    assert lib.svlcov_server_submit(None, 0, 0, None, None, C.byref(t)) == 1
    assert lib.svlcov_server_drain(None) == 1
    assert lib.svlcov_server_attach(None, None, None) == 1


def test_server_binding_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the server starts normally there")
    import paper_2401_09703_amd as L
    with pytest.raises(L.SvlcovError) as e:
        L.Server(max_inflight=2)
    assert e.value.code == 5


def test_spmm_tuning_table_without_gpu(tmp_path):
    """The fused projection's tile-shape table: variants, set/get round trip,
    key and variant validation, and the JSON cache loader (no device use)."""
    import json
    import paper_2401_09703_amd as L
    shapes = L.spmm_variants()
    assert shapes[0] == (8, 8) and len(shapes) == len(set(shapes)) >= 4
    saved = {(f, k, b): L.spmm_tune_get(f, k, b) for f in (0, 1) for k in (16, 32, 64, 128)
             for b in range(4)}
    try:
        L.spmm_tune_set(1, 32, 3, len(shapes) - 1)
        assert L.spmm_tune_get(1, 32, 3) == len(shapes) - 1
        for bad in ((2, 64, 0, 0), (0, 48, 0, 0), (0, 64, 4, 0), (0, 64, 0, len(shapes)),
                    (0, 64, -1, 0)):
            with pytest.raises(L.SvlcovError):
                L.spmm_tune_set(*bad)
        with pytest.raises(L.SvlcovError):
            L.spmm_tune_get(0, 64, 9)
        assert [L.spmm_row_bin(x) for x in (0, 15.9, 16, 63, 64, 255, 256, 1e6)] == \
            [0, 0, 1, 1, 2, 2, 3, 3]
        p = tmp_path / "tune.json"
        p.write_text(json.dumps({"entries": [{"fp64": 0, "k": 16, "row_bin": 1, "variant": 2},
                                             {"fp64": 1, "k": 128, "row_bin": 0, "variant": 1}]}))
        assert L.load_spmm_tuning(str(p)) == 2
        assert L.spmm_tune_get(0, 16, 1) == 2 and L.spmm_tune_get(1, 128, 0) == 1
        assert L.load_spmm_tuning(str(tmp_path / "missing.json")) == 0
    finally:
        for (f, k, b), v in saved.items():
            L.spmm_tune_set(f, k, b, v)


def test_noalloc_eig_rejects_bad_sizes_before_device_use():
    import paper_2401_09703_amd as L
    lib = L._lib
    buf = np.zeros(64)
    p = buf.ctypes.data
    assert lib.svlcov_sym_eig_topk_noalloc(2048, p, 64, p, p, None) == 7   # beyond the workspace
    assert lib.svlcov_sym_eig_topk_noalloc(7000, p, 64, p, p, None) == 7   # N > 6144
    assert lib.svlcov_sym_eig_topk_noalloc(8, p, 9, p, p, None) == 1       # k > N
    assert lib.svlcov_sym_eig_topk_noalloc(8, None, 4, p, p, None) == 1
