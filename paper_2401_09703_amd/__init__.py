"""Python binding of libsvlcov.so (ctypes; argument marshalling only).

Every step of an update runs in the library's HIP kernels; this module only
turns NumPy arrays or torch tensors into the C structs and pointers the C ABI
takes, and raises on non-OK status codes.  It never falls back to another
implementation: if the shared library is missing or fails to load, importing
the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:
    # torch and this library must share one HIP runtime: both link
    # libamdhip64.so.7, and the first copy loaded into the process is the one
    # every later user binds to.  Loading torch first keeps its device memory
    # and streams valid for the library.
    import torch  # noqa: F401
except ImportError:  # CPU-only environments without torch
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvlcov.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
_STATUS = {0: "ok", 1: "invalid argument", 2: "shape mismatch", 3: "out of device memory",
           4: "non-finite value", 5: "HIP runtime error", 6: "state busy",
           7: "unsupported size or option"}


class SvlcovError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {_STATUS.get(code, code)} (status {code})")
        self.code = code


class _Csr(C.Structure):
    _fields_ = [("rows", C.c_int64), ("cols", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("val_dtype", C.c_int32), ("on_device", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
                ("row_capacity", C.c_int64), ("col_capacity", C.c_int64),
                ("rank_tol", C.c_double), ("cond_reset", C.c_double),
                ("validate_device_inputs", C.c_int32),
                ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN), ("alloc_ctx", C.c_void_p),
                ("deterministic", C.c_int32), ("side_stream", C.c_int32)]


def _torch_alloc(nbytes, stream, ctx):
    """dev_alloc hook backed by torch's caching allocator (ctx = device ordinal):
    the block is tied to the state's stream, so torch reuses it only for work
    ordered after the state's earlier work."""
    try:
        import torch
        dev = int(ctx or 0)
        s = torch.cuda.ExternalStream(stream, device=dev) if stream else None
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=s))
    except Exception:
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# one pair of C callbacks for the whole process (they must outlive every state)
_TORCH_HOOKS = (_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))


class _Stats(C.Structure):
    _fields_ = [("updates", C.c_int64), ("resets_U", C.c_int64), ("resets_V", C.c_int64),
                ("last_rank", C.c_int32), ("last_rank2", C.c_int32),
                ("last_kappa_U", C.c_double), ("last_kappa_V", C.c_double),
                ("last_min_kept_pivot", C.c_double), ("last_max_dropped_pivot", C.c_double),
                ("iter_runs", C.c_int64), ("iter_steps", C.c_int64), ("iter_fallbacks", C.c_int64),
                ("iter_flops", C.c_double)]


class _Approx(C.Structure):
    _fields_ = [("method", C.c_int32), ("l", C.c_int32), ("t", C.c_int32),
                ("start_on_device", C.c_int32), ("start", C.c_void_p)]


class Approx:
    """The -GKL / -RPI variant of an append (svlcov_add_rows_approx /
    svlcov_add_cols_approx): method "gkl" or "rpi", dimension l, RPI rounds t,
    and the start (GKL: p_1 of s values or None for all ones; RPI: an s x l
    array whose columns are P_0), a host array or a device tensor."""

    METHODS = {"gkl": 1, "rpi": 2}

    def __init__(self, method: str = "gkl", l: int = 10, t: int = 3, start=None):
        if method not in self.METHODS:
            raise ValueError(method)
        self.method, self.l, self.t, self.start = method, int(l), int(t), start

    def _struct(self, keep: list) -> "_Approx":
        st = _Approx(self.METHODS[self.method], self.l, self.t, 0, None)
        x = self.start
        if x is None:
            return st
        if _is_torch(x):
            import torch
            v = x.detach().to(torch.float64)
            v = (v.t() if v.dim() == 2 else v).contiguous()   # RPI: vector j at j*s
            keep.append(v)
            st.start_on_device = 1 if v.is_cuda else 0
            st.start = v.data_ptr()
        else:
            v = np.asarray(x, dtype=np.float64)
            v = np.ascontiguousarray(v.T if v.ndim == 2 else v)
            keep.append(v)
            st.start = v.ctypes.data
        return st


class _ServerOptions(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_inflight", C.c_int32),
                ("workspace_budget", C.c_int64)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("peak_inflight", C.c_int64), ("peak_workspace_bytes", C.c_int64),
                ("fused_launches", C.c_int64), ("fused_requests", C.c_int64),
                ("fused_ms", C.c_double)]


EXPORTS = ["svlcov_default_options", "svlcov_init", "svlcov_add_rows", "svlcov_add_cols",
           "svlcov_update_weights", "svlcov_get_factors", "svlcov_query_row", "svlcov_sync",
           "svlcov_get_stats", "svlcov_stream", "svlcov_destroy", "svlcov_status_str",
           "svlcov_profile", "svlcov_profile_phases", "svlcov_phase_times", "svlcov_phase_name",
           "svlcov_sym_eig_topk", "svlcov_server_default_options", "svlcov_server_create",
           "svlcov_server_attach", "svlcov_server_submit", "svlcov_server_wait",
           "svlcov_server_poll", "svlcov_server_drain", "svlcov_server_get_stats",
           "svlcov_server_destroy", "svlcov_project_batch", "svlcov_add_rows_approx",
           "svlcov_add_cols_approx", "svlcov_spmm_variant_count", "svlcov_spmm_variant_shape",
           "svlcov_spmm_tune_set", "svlcov_spmm_tune_get", "svlcov_query_rows",
           "svlcov_score_pairs", "svlcov_rsvd", "svlcov_update_weights_approx",
           "svlcov_sym_eig_topk_noalloc"]
NUM_PHASES = 17
RSVD_PHASES = ("transpose", "products", "orthonormalise", "small_eig", "final")


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libsvlcov.so not built at {path}; run python paper_2401_09703_amd/build.py")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.svlcov_default_options.argtypes = [C.POINTER(_Options)]
    lib.svlcov_default_options.restype = None
    lib.svlcov_init.argtypes = [C.POINTER(P), I64, I64, I32, P, P, P, I32, C.POINTER(_Options)]
    lib.svlcov_add_rows.argtypes = [P, C.POINTER(_Csr)]
    lib.svlcov_add_cols.argtypes = [P, C.POINTER(_Csr)]
    lib.svlcov_update_weights.argtypes = [P, C.POINTER(_Csr), C.POINTER(_Csr)]
    lib.svlcov_query_rows.argtypes = [P, I32, I64, P, P]
    lib.svlcov_score_pairs.argtypes = [P, I64, P, P, I32, P, C.POINTER(C.c_float)]
    lib.svlcov_spmm_variant_count.argtypes = []
    lib.svlcov_spmm_variant_count.restype = I32
    lib.svlcov_spmm_variant_shape.argtypes = [I32, C.POINTER(I32), C.POINTER(I32)]
    lib.svlcov_spmm_tune_set.argtypes = [I32, I32, I32, I32]
    lib.svlcov_spmm_tune_get.argtypes = [I32, I32, I32, C.POINTER(I32)]
    lib.svlcov_add_rows_approx.argtypes = [P, C.POINTER(_Csr), C.POINTER(_Approx)]
    lib.svlcov_add_cols_approx.argtypes = [P, C.POINTER(_Csr), C.POINTER(_Approx)]
    lib.svlcov_update_weights_approx.argtypes = [P, C.POINTER(_Csr), C.POINTER(_Csr),
                                                 C.POINTER(_Approx), C.POINTER(_Approx)]
    lib.svlcov_update_weights_approx.restype = I32
    lib.svlcov_get_factors.argtypes = [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32), I32,
                                       I32, P, P, P]
    lib.svlcov_query_row.argtypes = [P, I32, I64, P]
    lib.svlcov_sync.argtypes = [P]
    lib.svlcov_get_stats.argtypes = [P, C.POINTER(_Stats)]
    lib.svlcov_stream.argtypes = [P]
    lib.svlcov_stream.restype = P
    lib.svlcov_destroy.argtypes = [P]
    lib.svlcov_destroy.restype = None
    lib.svlcov_profile.argtypes = [P, I32]
    lib.svlcov_profile.restype = I32
    lib.svlcov_profile_phases.argtypes = [P, C.c_uint32]
    lib.svlcov_profile_phases.restype = I32
    lib.svlcov_phase_times.argtypes = [P, P, P, I32]
    lib.svlcov_phase_times.restype = I32
    lib.svlcov_phase_name.argtypes = [I32]
    lib.svlcov_phase_name.restype = C.c_char_p
    lib.svlcov_sym_eig_topk.argtypes = [I64, P, I32, P, P, P]
    lib.svlcov_sym_eig_topk.restype = I32
    lib.svlcov_sym_eig_topk_noalloc.argtypes = [I64, P, I32, P, P, P]
    lib.svlcov_sym_eig_topk_noalloc.restype = I32
    lib.svlcov_rsvd.argtypes = [C.POINTER(_Csr), I32, I32, I32, P, P, P, P, P, P]
    lib.svlcov_rsvd.restype = I32
    lib.svlcov_status_str.argtypes = [I32]
    lib.svlcov_status_str.restype = C.c_char_p
    lib.svlcov_project_batch.argtypes = [I32, P, P, P, P, P, P, C.POINTER(C.c_float)]
    lib.svlcov_project_batch.restype = I32
    lib.svlcov_server_default_options.argtypes = [C.POINTER(_ServerOptions)]
    lib.svlcov_server_default_options.restype = None
    lib.svlcov_server_create.argtypes = [C.POINTER(P), C.POINTER(_ServerOptions)]
    lib.svlcov_server_attach.argtypes = [P, P, C.POINTER(I32)]
    lib.svlcov_server_submit.argtypes = [P, I32, I32, C.POINTER(_Csr), C.POINTER(_Csr),
                                         C.POINTER(I64)]
    lib.svlcov_server_wait.argtypes = [P, I64, C.POINTER(I32), C.POINTER(C.c_double)]
    lib.svlcov_server_poll.argtypes = [P, I64, C.POINTER(I32), C.POINTER(I32),
                                       C.POINTER(C.c_double)]
    lib.svlcov_server_drain.argtypes = [P]
    lib.svlcov_server_get_stats.argtypes = [P, C.POINTER(_ServerStats)]
    lib.svlcov_server_destroy.argtypes = [P]
    lib.svlcov_server_destroy.restype = None
    for name in ("svlcov_server_create", "svlcov_server_attach", "svlcov_server_submit",
                 "svlcov_server_wait", "svlcov_server_poll", "svlcov_server_drain",
                 "svlcov_server_get_stats"):
        getattr(lib, name).restype = I32
    for name in ("svlcov_init", "svlcov_add_rows", "svlcov_add_cols", "svlcov_update_weights",
                 "svlcov_get_factors", "svlcov_query_row", "svlcov_sync", "svlcov_get_stats"):
        getattr(lib, name).restype = I32
    return lib


_lib = load_library()

# Every live state and server, closed explicitly at interpreter exit (servers
# first): their HIP frees and stream/event destroys then run while the HIP
# runtime and any profiler attached to it are still up, not from __del__ during
# module teardown.
import atexit as _atexit
import weakref as _weakref

_LIVE_STATES = _weakref.WeakSet()
_LIVE_SERVERS = _weakref.WeakSet()


@_atexit.register
def close_all():
    """Close every live Server, then every live TruncatedSVD."""
    for srv in list(_LIVE_SERVERS):
        srv.close()
    for svd in list(_LIVE_STATES):
        svd.close()


def _check(code: int, where: str):
    if code != 0:
        raise SvlcovError(code, where)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class DeviceCSR:
    """CSR whose arrays are torch tensors on the GPU (int64 row_ptr, int32
    col_idx, float64/float32 val).  Keeps the tensors alive."""

    def __init__(self, rows, cols, row_ptr, col_idx, val):
        self.rows, self.cols = int(rows), int(cols)
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val

    @staticmethod
    def from_host(m, device="cuda"):
        import torch
        return DeviceCSR(m.rows, m.cols,
                         torch.as_tensor(np.ascontiguousarray(m.row_ptr, dtype=np.int64), device=device),
                         torch.as_tensor(np.ascontiguousarray(m.col_idx, dtype=np.int32), device=device),
                         torch.as_tensor(np.ascontiguousarray(m.val, dtype=np.float64), device=device))


def _csr_struct(m, keep: list) -> _Csr:
    """Marshal a CSR given with .rows .cols .row_ptr .col_idx .val (NumPy
    arrays = host, CUDA torch tensors = device)."""
    rp, ci, v = m.row_ptr, m.col_idx, m.val
    if _is_torch(rp):
        import torch
        assert rp.dtype == torch.int64 and ci.dtype == torch.int32
        assert v.dtype in (torch.float64, torch.float32)
        for t in (rp, ci, v):
            assert t.is_cuda and t.is_contiguous()
        keep.extend([rp, ci, v])
        return _Csr(m.rows, m.cols, int(ci.numel()),
                    rp.data_ptr(), ci.data_ptr(), v.data_ptr(),
                    1 if v.dtype == torch.float64 else 0, 1)
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    v = np.ascontiguousarray(v)
    if v.dtype not in (np.float64, np.float32):
        v = v.astype(np.float64)
    keep.extend([rp, ci, v])
    return _Csr(int(m.rows), int(m.cols), int(ci.size), rp.ctypes.data, ci.ctypes.data,
                v.ctypes.data, 1 if v.dtype == np.float64 else 0, 0)


def sym_eig_topk(M, k: int, stream=None):
    """Top-k eigenpairs of a symmetric FP64 CUDA tensor M (N x N) on the GPU:
    returns (lam, vecs) as CUDA tensors, lam descending, vecs k x N."""
    import torch as _t
    assert M.is_cuda and M.dtype == _t.float64 and M.is_contiguous()
    N = M.shape[0]
    lam = _t.empty(k, dtype=_t.float64, device=M.device)
    vecs = _t.empty((k, N), dtype=_t.float64, device=M.device)
    st = stream if stream is not None else _t.cuda.current_stream().cuda_stream
    _check(_lib.svlcov_sym_eig_topk(N, M.data_ptr(), k, lam.data_ptr(), vecs.data_ptr(), st),
           "svlcov_sym_eig_topk")
    return lam, vecs


def sym_eig_topk_noalloc(M, k: int, lam=None, vecs=None, stream=None):
    """sym_eig_topk through svlcov_sym_eig_topk_noalloc: the library allocates
    nothing (its workspace is a fixed per-GPU array).  lam (k) and vecs (k x N)
    may be passed in as preallocated FP64 CUDA tensors."""
    import torch as _t
    assert M.is_cuda and M.dtype == _t.float64 and M.is_contiguous()
    N = M.shape[0]
    if lam is None:
        lam = _t.empty(k, dtype=_t.float64, device=M.device)
    if vecs is None:
        vecs = _t.empty((k, N), dtype=_t.float64, device=M.device)
    assert lam.is_cuda and lam.dtype == _t.float64 and lam.numel() >= k
    assert vecs.is_cuda and vecs.dtype == _t.float64 and vecs.is_contiguous()
    assert vecs.numel() >= k * N
    st = stream if stream is not None else _t.cuda.current_stream().cuda_stream
    _check(_lib.svlcov_sym_eig_topk_noalloc(N, M.data_ptr(), k, lam.data_ptr(),
                                            vecs.data_ptr(), st),
           "svlcov_sym_eig_topk_noalloc")
    return lam, vecs


def rsvd(A, k: int, l: int = None, power: int = 2, Omega=None, seed: int = 0, stream=None,
         timing: dict = None):
    """Initial rank-k truncated SVD of the sparse matrix A (DeviceCSR or a
    host CSR with .rows .cols .row_ptr .col_idx .val) on the GPU by the
    randomised range finder with ``power`` subspace iterations
    (svlcov_rsvd).  Omega is the n x l FP64 CUDA test matrix; when None it is
    drawn (standard normal) from a torch generator seeded with ``seed``.  l
    defaults to the smallest of 16, 32, 64, 128 that is >= 2k (or 128).
    Returns (U, s, V) as FP64 CUDA tensors; ``timing`` (a dict) receives the
    per-phase milliseconds."""
    import torch as _t
    m, n = int(A.rows), int(A.cols)
    if l is None:
        l = next((c for c in (16, 32, 64, 128) if c >= 2 * k), 128)
    if Omega is None:
        g = _t.Generator(device="cuda")
        g.manual_seed(int(seed))
        Omega = _t.randn((n, l), generator=g, device="cuda", dtype=_t.float64)
    assert Omega.is_cuda and Omega.dtype == _t.float64 and Omega.is_contiguous()
    assert tuple(Omega.shape) == (n, l)
    U = _t.empty((m, k), dtype=_t.float64, device=Omega.device)
    V = _t.empty((n, k), dtype=_t.float64, device=Omega.device)
    s = _t.empty(k, dtype=_t.float64, device=Omega.device)
    keep = []
    cs = _csr_struct(A, keep)
    st = stream if stream is not None else _t.cuda.current_stream().cuda_stream
    ms = (C.c_double * len(RSVD_PHASES))()
    _check(_lib.svlcov_rsvd(C.byref(cs), k, l, power, Omega.data_ptr(), U.data_ptr(),
                            s.data_ptr(), V.data_ptr(), ms if timing is not None else None, st),
           "svlcov_rsvd")
    if timing is not None:
        timing.update({name: ms[i] for i, name in enumerate(RSVD_PHASES)})
    return U, s, V


class TruncatedSVD:
    """A rank-k truncated SVD kept on the GPU in the extended form
    U = U_base W_U, V = V_base W_V (Section 3.2), updated by the library.
    allocator="torch" makes torch's caching allocator own the state's device
    memory (the svlcov_options allocator hooks); the default is the library's
    own stream-ordered HIP allocations.  deterministic=False accumulates the
    sparse row update with atomics (faster, rounding order free) instead of
    summing each base row's terms in a fixed order.  side_stream=False keeps
    an append update on the state's stream alone (the factors are the same
    bit for bit; the second stream only lets the Cholesky run beside the
    eigensolver)."""

    def __init__(self, U, s, V, precision: str = "fp64", device: int = 0, stream=None,
                 row_capacity: int = 0, col_capacity: int = 0, rank_tol: float = 0.0,
                 cond_reset: float = 0.0, validate_device_inputs: bool = True,
                 allocator: str = None, deterministic: bool = True,
                 side_stream: bool = True):
        on_dev = 0
        if _is_torch(U):
            # device factors (FP64 CUDA tensors), read on the state's stream
            import torch
            for t in (U, s, V):
                assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            torch.cuda.synchronize()
            on_dev = 1
            m_, n_, k_ = U.shape[0], V.shape[0], s.numel()
            pU, ps, pV = U.data_ptr(), s.data_ptr(), V.data_ptr()
        else:
            U = np.ascontiguousarray(U, dtype=np.float64)
            V = np.ascontiguousarray(V, dtype=np.float64)
            s = np.ascontiguousarray(s, dtype=np.float64)
            m_, n_, k_ = U.shape[0], V.shape[0], s.size
            pU, ps, pV = U.ctypes.data, s.ctypes.data, V.ctypes.data
        opt = _Options()
        _lib.svlcov_default_options(C.byref(opt))
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.device = device
        opt.stream = stream
        opt.row_capacity = row_capacity
        opt.col_capacity = col_capacity
        opt.rank_tol = rank_tol
        opt.cond_reset = cond_reset
        opt.validate_device_inputs = 1 if validate_device_inputs else 0
        opt.deterministic = 1 if deterministic else 0
        opt.side_stream = 1 if side_stream else 0
        if allocator == "torch":
            # the state's factors and workspaces come from torch's caching allocator
            opt.dev_alloc, opt.dev_free = _TORCH_HOOKS
            opt.alloc_ctx = device
        elif allocator is not None:
            raise ValueError(f"allocator must be None or 'torch', not {allocator!r}")
        h = C.c_void_p()
        _check(_lib.svlcov_init(C.byref(h), m_, n_, k_, pU, ps, pV, on_dev, C.byref(opt)),
               "svlcov_init")
        self._h = h
        self.k = int(k_)
        self.precision = precision
        self._keep = []
        self._server = None   # the Server this state is attached to, if any
        _LIVE_STATES.add(self)

    # -- updates (asynchronous; inputs must stay alive until sync).  Device
    # inputs are read on the state's stream, which first waits for torch's
    # current stream, so whatever torch enqueued to produce them comes first.
    def _order_inputs(self, *objs):
        if any(_is_torch(getattr(o, "row_ptr", o)) for o in objs if o is not None):
            self._follow_torch()

    def add_rows(self, E, approx: "Approx" = None):
        st = _csr_struct(E, self._keep)
        self._order_inputs(E, approx.start if approx is not None else None)
        if approx is None:
            _check(_lib.svlcov_add_rows(self._h, C.byref(st)), "svlcov_add_rows")
        else:
            a = approx._struct(self._keep)
            _check(_lib.svlcov_add_rows_approx(self._h, C.byref(st), C.byref(a)),
                   "svlcov_add_rows_approx")

    def add_cols(self, Ec_T, approx: "Approx" = None):
        st = _csr_struct(Ec_T, self._keep)
        self._order_inputs(Ec_T, approx.start if approx is not None else None)
        if approx is None:
            _check(_lib.svlcov_add_cols(self._h, C.byref(st)), "svlcov_add_cols")
        else:
            a = approx._struct(self._keep)
            _check(_lib.svlcov_add_cols_approx(self._h, C.byref(st), C.byref(a)),
                   "svlcov_add_cols_approx")

    def update_weights(self, D_T, Em_T, approx=None):
        """A + D E_m^T; with approx (an Approx for both sides, whose start may
        be a pair (start for D, start for E_m), or a pair of Approx) the -GKL
        / -RPI variant."""
        a = _csr_struct(D_T, self._keep)
        b = _csr_struct(Em_T, self._keep)
        starts = []
        for ap in (approx if isinstance(approx, (tuple, list)) else [approx]):
            if ap is not None:
                starts += list(ap.start) if isinstance(ap.start, (tuple, list)) else [ap.start]
        self._order_inputs(D_T, Em_T, *starts)
        if approx is None:
            _check(_lib.svlcov_update_weights(self._h, C.byref(a), C.byref(b)),
                   "svlcov_update_weights")
            return
        if isinstance(approx, (tuple, list)):
            aD, aE = approx
        elif isinstance(approx.start, (tuple, list)):
            aD = Approx(approx.method, approx.l, approx.t, approx.start[0])
            aE = Approx(approx.method, approx.l, approx.t, approx.start[1])
        else:
            aD = aE = approx
        sD, sE = aD._struct(self._keep), aE._struct(self._keep)
        _check(_lib.svlcov_update_weights_approx(self._h, C.byref(a), C.byref(b), C.byref(sD),
                                                 C.byref(sE)), "svlcov_update_weights_approx")

    def apply(self, update, approx: "Approx" = None):
        kind = update[0]
        if kind == "rows":
            self.add_rows(update[1], approx)
        elif kind == "cols":
            self.add_cols(update[1], approx)
        elif kind == "weights":
            self.update_weights(update[1], update[2], approx)
        else:
            raise ValueError(kind)

    def sync(self):
        code = _lib.svlcov_sync(self._h)
        self._keep = []
        _check(code, "svlcov_sync")

    @property
    def stream(self) -> int:
        return int(_lib.svlcov_stream(self._h) or 0)

    def shape(self):
        m, n, k = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.svlcov_get_factors(self._h, C.byref(m), C.byref(n), C.byref(k), 1, 0,
                                       None, None, None), "svlcov_get_factors")
        return m.value, n.value

    def factors(self, dtype=np.float64):
        """Realised (U, s, V) as host NumPy arrays."""
        m, n = self.shape()
        U = np.empty((m, self.k), dtype=dtype)
        V = np.empty((n, self.k), dtype=dtype)
        s = np.empty(self.k, dtype=np.float64)
        _check(_lib.svlcov_get_factors(self._h, None, None, None,
                                       1 if dtype == np.float64 else 0, 0, U.ctypes.data,
                                       s.ctypes.data, V.ctypes.data), "svlcov_get_factors")
        self._keep = []
        return U, s, V

    def query(self, side: int, i: int):
        out = np.empty(self.k, dtype=np.float64)
        _check(_lib.svlcov_query_row(self._h, side, i, out.ctypes.data), "svlcov_query_row")
        return out

    def query_rows(self, side: int, idx):
        """Rows idx of U (side 0) or V (side 1) as a (len(idx), k) FP64 CUDA
        tensor (svlcov_query_rows; NaN rows for indices outside the factor)."""
        import torch
        ix = torch.as_tensor(idx, dtype=torch.int64, device="cuda").contiguous()
        out = torch.empty((ix.numel(), self.k), dtype=torch.float64, device="cuda")
        self._follow_torch()
        _check(_lib.svlcov_query_rows(self._h, int(side), ix.numel(), ix.data_ptr(),
                                      out.data_ptr()), "svlcov_query_rows")
        self._keep.append(ix)
        self._lead_torch()
        return out

    def _follow_torch(self):
        """The state's stream waits for torch's current stream (inputs)."""
        import torch
        ext = torch.cuda.ExternalStream(self.stream)
        ext.wait_stream(torch.cuda.current_stream())

    def _lead_torch(self):
        """Torch's current stream waits for the state's stream (outputs)."""
        import torch
        ext = torch.cuda.ExternalStream(self.stream)
        torch.cuda.current_stream().wait_stream(ext)

    def score_pairs(self, i, j, both: bool = False, timing=None):
        """U[i]^T Sigma V[j] per pair (the larger of both directions with
        both) as an FP64 CUDA tensor (svlcov_score_pairs); with a list as
        timing the scoring kernel's device time in ms is appended."""
        import torch
        ti = torch.as_tensor(i, dtype=torch.int64, device="cuda").contiguous()
        tj = torch.as_tensor(j, dtype=torch.int64, device="cuda").contiguous()
        out = torch.empty(ti.numel(), dtype=torch.float64, device="cuda")
        ms = C.c_float(0.0)
        self._follow_torch()
        _check(_lib.svlcov_score_pairs(self._h, ti.numel(), ti.data_ptr(), tj.data_ptr(),
                                       1 if both else 0, out.data_ptr(),
                                       C.byref(ms) if timing is not None else None),
               "svlcov_score_pairs")
        self._keep += [ti, tj]
        self._lead_torch()
        if timing is not None:
            timing.append(float(ms.value))
        return out

    def stats(self) -> dict:
        st = _Stats()
        _check(_lib.svlcov_get_stats(self._h, C.byref(st)), "svlcov_get_stats")
        return {f: getattr(st, f) for f, _ in _Stats._fields_}

    def profile(self, enable: bool = True, phases=None):
        """Time every phase of the following updates, or only the named ones
        (svlcov_profile_phases)."""
        if phases is None or not enable:
            _check(_lib.svlcov_profile(self._h, 1 if enable else 0), "svlcov_profile")
            return
        names = [_lib.svlcov_phase_name(i).decode() for i in range(NUM_PHASES)]
        mask = 0
        for name in phases:
            if name not in names:
                raise ValueError(f"unknown phase {name!r}")
            mask |= 1 << names.index(name)
        _check(_lib.svlcov_profile_phases(self._h, mask), "svlcov_profile_phases")

    def phase_times(self) -> dict:
        """{phase name: (total ms, occurrences)} since the previous call."""
        ms = np.zeros(NUM_PHASES)
        cnt = np.zeros(NUM_PHASES, dtype=np.int64)
        _check(_lib.svlcov_phase_times(self._h, ms.ctypes.data, cnt.ctypes.data, NUM_PHASES),
               "svlcov_phase_times")
        return {_lib.svlcov_phase_name(i).decode(): (float(ms[i]), int(cnt[i]))
                for i in range(NUM_PHASES)}

    def close(self):
        """Destroy the state.  A state attached to a live Server belongs to it
        until the server is closed (the library would refuse the destroy)."""
        if getattr(self, "_h", None):
            srv = getattr(self, "_server", None)
            if srv is not None and getattr(srv, "_h", None):
                raise RuntimeError("TruncatedSVD is attached to a live Server; close the server first")
            _lib.svlcov_destroy(self._h)
            self._h = None
            _LIVE_STATES.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def project_batch(states, sides, Es, stream=None, timing=None):
    """The fused projection C' = E base W of many updates in one launch
    (svlcov_project_batch): states are idle TruncatedSVD objects, sides 0 (U)
    or 1 (V), Es DeviceCSR.  Returns the C' tensors (rows x k FP64 CUDA) and
    the squared row norms of each E; with a list as ``timing`` the launch's
    device time in ms is appended to it."""
    import torch
    n = len(states)
    keep, outs, norms = [], [], []
    csrs = (_Csr * n)()
    for q, (svd, E) in enumerate(zip(states, Es)):
        csrs[q] = _csr_struct(E, keep)
        outs.append(torch.empty((E.rows, svd.k), dtype=torch.float64, device="cuda"))
        norms.append(torch.empty(E.rows, dtype=torch.float64, device="cuda"))
    hs = (C.c_void_p * n)(*[svd._h for svd in states])
    sd = (C.c_int32 * n)(*sides)
    po = (C.c_void_p * n)(*[t.data_ptr() for t in outs])
    pn = (C.c_void_p * n)(*[t.data_ptr() for t in norms])
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    ms = C.c_float(0.0)
    _check(_lib.svlcov_project_batch(n, hs, sd, csrs, po, pn, st,
                                     C.byref(ms) if timing is not None else None),
           "svlcov_project_batch")
    if timing is not None:
        timing.append(float(ms.value))
    return outs, norms


# ---- tile shapes of the fused projection and their tuning table
SPMM_ROW_BINS = (16, 64, 256)   # bin edges in mean nonzeros per row
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spmm_tuning_gfx950.json")


def spmm_variants():
    """[(loads in flight per lane, rows per tile)] of every variant."""
    out = []
    for v in range(_lib.svlcov_spmm_variant_count()):
        u, rb = C.c_int32(), C.c_int32()
        _check(_lib.svlcov_spmm_variant_shape(v, C.byref(u), C.byref(rb)),
               "svlcov_spmm_variant_shape")
        out.append((u.value, rb.value))
    return out


def spmm_row_bin(nnz_per_row: float) -> int:
    return sum(nnz_per_row >= e for e in SPMM_ROW_BINS)


def spmm_tune_set(fp64: int, k: int, row_bin: int, variant: int):
    _check(_lib.svlcov_spmm_tune_set(int(fp64), int(k), int(row_bin), int(variant)),
           "svlcov_spmm_tune_set")


def spmm_tune_get(fp64: int, k: int, row_bin: int) -> int:
    v = C.c_int32()
    _check(_lib.svlcov_spmm_tune_get(int(fp64), int(k), int(row_bin), C.byref(v)),
           "svlcov_spmm_tune_get")
    return v.value


def load_spmm_tuning(path: str = TUNING_PATH) -> int:
    """Apply a tuning cache written by ``paper_2401_09703_amd.autotune``;
    returns the number of entries applied (0 when there is no file)."""
    import json
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for e in data.get("entries", []):
        spmm_tune_set(e["fp64"], e["k"], e["row_bin"], e["variant"])
        n += 1
    return n


load_spmm_tuning(os.environ.get("SVLCOV_SPMM_TUNING", TUNING_PATH))


_OPS = {"rows": 0, "cols": 1, "weights": 2}


class Server:
    """Continuous-batching request server over many matrices on one GPU (the
    svlcov_server_* calls).  attach() hands a TruncatedSVD to the server;
    after that only the server updates it, and its factors may be read once
    drain() has returned.  Close the server before the attached states."""

    def __init__(self, device: int = 0, max_inflight: int = 8, workspace_budget: int = 0):
        opt = _ServerOptions()
        _lib.svlcov_server_default_options(C.byref(opt))
        opt.device, opt.max_inflight = device, max_inflight
        if workspace_budget:
            opt.workspace_budget = workspace_budget
        h = C.c_void_p()
        _check(_lib.svlcov_server_create(C.byref(h), C.byref(opt)), "svlcov_server_create")
        self._h = h
        self._keep = {}
        self._attached = []   # states stay alive while the server drives them
        _LIVE_SERVERS.add(self)

    def attach(self, svd: "TruncatedSVD") -> int:
        mid = C.c_int32()
        _check(_lib.svlcov_server_attach(self._h, svd._h, C.byref(mid)), "svlcov_server_attach")
        self._attached.append(svd)
        svd._server = self
        return int(mid.value)

    def submit(self, matrix_id: int, update) -> int:
        self._order_device_inputs(update)
        keep = []
        a = _csr_struct(update[1], keep)
        b = _csr_struct(update[2], keep) if update[0] == "weights" else None
        t = C.c_int64()
        _check(_lib.svlcov_server_submit(self._h, matrix_id, _OPS[update[0]], C.byref(a),
                                         C.byref(b) if b is not None else None, C.byref(t)),
               "svlcov_server_submit")
        # host inputs were copied; device tensors must outlive the request
        if any(_is_torch(x) for x in keep):
            self._keep[int(t.value)] = keep
        return int(t.value)

    @staticmethod
    def _order_device_inputs(update):
        """The server reads device inputs on its own streams: whatever torch
        enqueued to produce them must have finished first."""
        if any(_is_torch(getattr(x, "row_ptr", None)) for x in update[1:]):
            import torch
            torch.cuda.current_stream().synchronize()

    def wait(self, ticket: int):
        """(status code, latency in ms) of a request; blocks."""
        st, lat = C.c_int32(), C.c_double()
        _check(_lib.svlcov_server_wait(self._h, ticket, C.byref(st), C.byref(lat)),
               "svlcov_server_wait")
        self._keep.pop(ticket, None)
        return int(st.value), float(lat.value)

    def poll(self, ticket: int):
        """None while the request runs, else (status code, latency in ms)."""
        done, st, lat = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.svlcov_server_poll(self._h, ticket, C.byref(done), C.byref(st),
                                       C.byref(lat)), "svlcov_server_poll")
        if not done.value:
            return None
        self._keep.pop(ticket, None)
        return int(st.value), float(lat.value)

    def drain(self):
        _check(_lib.svlcov_server_drain(self._h), "svlcov_server_drain")

    def stats(self) -> dict:
        st = _ServerStats()
        _check(_lib.svlcov_server_get_stats(self._h, C.byref(st)), "svlcov_server_get_stats")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.svlcov_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            for svd in self._attached:
                svd._server = None
            self._attached = []
            _LIVE_SERVERS.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["TruncatedSVD", "DeviceCSR", "rsvd", "SvlcovError", "Server", "project_batch", "Approx",
           "close_all", "spmm_variants", "spmm_tune_set", "spmm_tune_get", "load_spmm_tuning", "spmm_row_bin", "load_library", "LIB_PATH", "EXPORTS",
           "FP64", "FP32", "BF16X3"]
