"""ctypes binding of libspk.so (argument marshalling only).

Every function has the name of the C entry point without the ``spk_`` prefix
and takes torch tensors where the C call takes device pointers; the tensor's
data pointer and the current torch stream are passed through.  There is no
fallback of any kind: if the HIP library is not built, importing this module
raises.
"""

from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime that libspk.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2011_00715_amd.build or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
dbl = ctypes.c_double

# ------------------------------------------------------------------ constants
MEM_HOST, MEM_DEVICE = 0, 1
PREC_FP64, PREC_MIXED, PREC_MIXED_IR = 0, 1, 2
MAT_MIXED, MAT_VALIDATE, MAT_BORROW, MAT_STREAM = 1, 2, 4, 8
KERNEL_AUTO, KERNEL_STREAM, KERNEL_VECTOR, KERNEL_MERGE, KERNEL_SELL, KERNEL_SLICED = 0, 1, 2, 3, 4, 5
KERNEL_SELL_SIGMA = 6
# spk_mat_set_kernel parameter of SPK_KERNEL_SELL: column offsets shared per slice
SELL_SHARED = 1
KERNEL_NAMES = {1: "stream", 2: "vector", 3: "merge", 4: "sell", 5: "sliced", 6: "sell_sigma"}
OK, EINVAL, ENOMEM, EHIP, EZERODIAG, EBUSY, EBUDGET, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
CONVERGED_RTOL, CONVERGED_ATOL = 1, 2
DIVERGED_ITS, DIVERGED_INDEFINITE_MAT, DIVERGED_INDEFINITE_PC = -1, -2, -3
DIVERGED_NANORINF, DIVERGED_BREAKDOWN, DIVERGED_STAGNATION = -4, -5, -6


class MatInfo(ctypes.Structure):
    _fields_ = [
        ("n", i32), ("kernel", i32), ("nnz", i64), ("lanes", i32), ("has_f32", i32),
        ("row_min", i32), ("row_max", i32), ("row_p50", i32), ("row_p99", i32),
        ("row_mean", dbl), ("row_cv", dbl),
        ("bytes_spmv_f64", i64), ("bytes_spmv_f32", i64),
        ("bytes_pcg_iter_f64", i64), ("bytes_pcg_iter_f32", i64),
        ("device_bytes", i64), ("zero_diag_rows", i32), ("cached_loads", i32),
        ("format_bytes_spmv_f64", i64), ("format_bytes_spmv_f32", i64), ("stored_nnz", i64),
        ("gershgorin", dbl), ("sell_sigma", i32), ("pad_", i32),
    ]


class KspOpts(ctypes.Structure):
    _fields_ = [
        ("rtol", dbl), ("atol", dbl), ("maxit", i32), ("precision", i32),
        ("x0_nonzero", i32), ("graph_k", i32), ("inner_rtol", dbl),
        ("inner_maxit", i32), ("max_outer", i32),
        ("hist", ctypes.POINTER(dbl)), ("hist_len", i32), ("single_reduction", i32),
        ("profile", i32),
    ]


class KspResult(ctypes.Structure):
    _fields_ = [
        ("reason", i32), ("iterations", i32), ("inner_iterations", i32),
        ("outer_steps", i32), ("restarts", i32), ("fallback_fp64", i32),
        ("rnorm0", dbl), ("rnorm", dbl), ("bnorm", dbl),
        ("true_rel_residual", dbl), ("seconds", dbl),
        ("product_ms", dbl), ("product_launches", i32), ("pad_", i32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["reason_str"] = reason_str(self.reason)
        return d


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", i64), ("max_slots", i32), ("graph_k", i32),
        ("max_blocks_per_system", i32), ("pad_", i32), ("pinned_bytes", i64),
    ]


class MgOpts(ctypes.Structure):
    _fields_ = [
        ("max_levels", i32), ("coarse_max", i32), ("smooth_steps", i32), ("cycle", i32),
        ("emin_frac", dbl), ("omega", dbl), ("precision", i32), ("pad_", i32),
    ]


class MgInfo(ctypes.Structure):
    _fields_ = [
        ("levels", i32), ("pad_", i32), ("n", i32 * 16), ("nnz", i64 * 16),
        ("shape", (i32 * 3) * 16), ("kernel", i32 * 16), ("emax", dbl * 16),
        ("device_bytes", i64),
    ]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("spk_mat_create_csr", ctypes.c_int, [i32, i64, P, P, P, ctypes.c_int, u32, P,
                                          ctypes.POINTER(P)])
_sig("spk_mat_set_kernel", ctypes.c_int, [P, ctypes.c_int, i32, P])
_sig("spk_mat_mult", ctypes.c_int, [P, P, P, P])
_sig("spk_mat_mult_f32", ctypes.c_int, [P, P, P, P])
_sig("spk_mat_get_info", ctypes.c_int, [P, ctypes.POINTER(MatInfo)])
_sig("spk_pc_jacobi_apply", ctypes.c_int, [P, P, P, P])
_sig("spk_pc_chebyshev", ctypes.c_int, [P, P, P, P, i32, dbl, dbl, i32, P])
_sig("spk_mat_destroy", ctypes.c_int, [P])
_sig("spk_vec_axpy", ctypes.c_int, [i32, dbl, P, P, P])
_sig("spk_vec_aypx", ctypes.c_int, [i32, dbl, P, P, P])
_sig("spk_vec_dot", ctypes.c_int, [i32, P, P, P, P])
_sig("spk_vec_dot2", ctypes.c_int, [i32, P, P, P, P, P])
_sig("spk_vec_dot2_noalloc", ctypes.c_int, [i32, P, P, P, P, P])
_sig("spk_vec_nrm2", ctypes.c_int, [i32, P, P, P])
_sig("spk_ksp_opts_default", None, [ctypes.POINTER(KspOpts)])
_sig("spk_ksp_solve", ctypes.c_int, [P, P, P, ctypes.POINTER(KspOpts),
                                     ctypes.POINTER(KspResult), P])
_sig("spk_mat_mult_multi", ctypes.c_int, [P, i32, P, P, P])
_sig("spk_ksp_solve_multi", ctypes.c_int, [P, i32, P, P, ctypes.POINTER(KspOpts),
                                           ctypes.POINTER(KspResult), P])
_sig("spk_mg_opts_default", None, [ctypes.POINTER(MgOpts)])
_sig("spk_mg_create", ctypes.c_int, [P, i32, P, ctypes.POINTER(MgOpts), P, ctypes.POINTER(P)])
_sig("spk_mg_get_info", ctypes.c_int, [P, ctypes.POINTER(MgInfo)])
_sig("spk_mg_copy_level", ctypes.c_int, [P, i32, P, P, P])
_sig("spk_mg_apply", ctypes.c_int, [P, P, P, P])
_sig("spk_mg_profile", ctypes.c_int, [P, P, P, i32, P, P])
_sig("spk_ksp_solve_mg", ctypes.c_int, [P, P, P, ctypes.POINTER(KspOpts), ctypes.POINTER(KspResult), P])
_sig("spk_mg_destroy", ctypes.c_int, [P])
_sig("spk_server_opts_default", None, [ctypes.POINTER(ServerOpts)])
_sig("spk_server_create", ctypes.c_int, [ctypes.POINTER(ServerOpts), P, ctypes.POINTER(P)])
_sig("spk_server_submit", ctypes.c_int, [P, i32, i64, P, P, P, P, ctypes.POINTER(KspOpts),
                                         ctypes.POINTER(u64)])
_sig("spk_server_progress", ctypes.c_int, [P, i32])
_sig("spk_server_poll", ctypes.c_int, [P, u64, P, ctypes.POINTER(KspResult),
                                       ctypes.POINTER(dbl)])
_sig("spk_server_completed", ctypes.c_int, [P, ctypes.POINTER(u64), i32])
_sig("spk_server_destroy", ctypes.c_int, [P])
_sig("spk_status_str", ctypes.c_char_p, [ctypes.c_int])
_sig("spk_reason_str", ctypes.c_char_p, [ctypes.c_int])
_sig("spk_last_error", ctypes.c_char_p, [])
_sig("spk_now", dbl, [])
_sig("spk_runtime_version", ctypes.c_int, [])
_sig("spk_bw_copy", ctypes.c_int, [i64, P, P, P])
_sig("spk_cache_flush", ctypes.c_int, [P, i64, P])

EXPORTS = [
    "spk_mat_create_csr", "spk_mat_set_kernel", "spk_mat_mult", "spk_mat_mult_f32",
    "spk_mat_get_info", "spk_pc_jacobi_apply", "spk_pc_chebyshev", "spk_mat_destroy", "spk_vec_axpy",
    "spk_vec_aypx", "spk_vec_dot", "spk_vec_dot2", "spk_vec_dot2_noalloc", "spk_vec_nrm2", "spk_ksp_opts_default",
    "spk_ksp_solve", "spk_mat_mult_multi", "spk_ksp_solve_multi", "spk_mg_opts_default",
    "spk_mg_create", "spk_mg_get_info", "spk_mg_copy_level", "spk_mg_apply", "spk_mg_profile",
    "spk_ksp_solve_mg", "spk_mg_destroy", "spk_server_opts_default", "spk_server_create", "spk_server_submit",
    "spk_server_progress", "spk_server_poll", "spk_server_completed", "spk_server_destroy", "spk_status_str",
    "spk_reason_str", "spk_last_error", "spk_now", "spk_runtime_version", "spk_bw_copy",
    "spk_cache_flush",
]


class SpkError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({last_error()})")


def _check(rc, where):
    if rc != OK:
        raise SpkError(rc, where)
    return rc


def status_str(s: int) -> str:
    return _lib.spk_status_str(s).decode()


def reason_str(r: int) -> str:
    return _lib.spk_reason_str(r).decode()


def last_error() -> str:
    return _lib.spk_last_error().decode()


def now() -> float:
    return _lib.spk_now()


def runtime_version() -> int:
    return _lib.spk_runtime_version()


def _stream(stream=None):
    if stream is None:
        return P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return P(stream.cuda_stream)
    return P(int(stream))


def _dev(t: torch.Tensor, dtype, n=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return P(t.data_ptr())


# ------------------------------------------------------------------ matrix
class Mat:
    """Owns an spk_mat handle (and, for borrowed CSR, the device arrays)."""

    def __init__(self, handle: int, keep=()):
        self.handle = P(handle)
        self._keep = keep
        self.info = mat_get_info(self)
        self.n = self.info.n
        self.nnz = self.info.nnz

    def close(self):
        if self.handle:
            mat_destroy(self)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def mat_create_csr(rowptr, colind, values, flags: int = 0, stream=None) -> Mat:
    """Create from torch tensors (all on the GPU: SPK_MEM_DEVICE) or NumPy
    arrays (host: SPK_MEM_HOST, copied through pinned staging)."""
    import numpy as np

    out = P()
    keep = ()
    if isinstance(rowptr, torch.Tensor):
        n = rowptr.numel() - 1
        nnz = colind.numel()
        args = (_dev(rowptr, torch.int32, name="rowptr"), _dev(colind, torch.int32, name="colind"),
                _dev(values, torch.float64, name="values"))
        mem = MEM_DEVICE
        if flags & MAT_BORROW:
            keep = (rowptr, colind, values)
    else:
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=np.float64)
        n = rowptr.size - 1
        nnz = colind.size
        args = tuple(P(a.ctypes.data) for a in (rowptr, colind, values))
        mem = MEM_HOST
    _check(_lib.spk_mat_create_csr(n, nnz, *args, mem, flags, _stream(stream), ctypes.byref(out)),
           "spk_mat_create_csr")
    return Mat(out.value, keep)


def mat_set_kernel(A: Mat, kernel: int, param: int = 0, stream=None):
    _check(_lib.spk_mat_set_kernel(A.handle, kernel, param, _stream(stream)), "spk_mat_set_kernel")
    A.info = mat_get_info(A)


def mat_mult(A: Mat, x: torch.Tensor, y: torch.Tensor, stream=None):
    _check(_lib.spk_mat_mult(A.handle, _dev(x, torch.float64, A.n, "x"),
                             _dev(y, torch.float64, A.n, "y"), _stream(stream)), "spk_mat_mult")


def mat_mult_f32(A: Mat, x: torch.Tensor, y: torch.Tensor, stream=None):
    _check(_lib.spk_mat_mult_f32(A.handle, _dev(x, torch.float32, A.n, "x"),
                                 _dev(y, torch.float32, A.n, "y"), _stream(stream)),
           "spk_mat_mult_f32")


def mat_get_info(A: Mat) -> MatInfo:
    info = MatInfo()
    _check(_lib.spk_mat_get_info(A.handle, ctypes.byref(info)), "spk_mat_get_info")
    return info


def pc_jacobi_apply(A: Mat, r: torch.Tensor, z: torch.Tensor, stream=None):
    _check(_lib.spk_pc_jacobi_apply(A.handle, _dev(r, torch.float64, A.n, "r"),
                                    _dev(z, torch.float64, A.n, "z"), _stream(stream)),
           "spk_pc_jacobi_apply")


def pc_chebyshev(A: Mat, b: torch.Tensor, x: torch.Tensor, steps: int, emin: float = 0.0,
                 emax: float = 0.0, r_out: torch.Tensor = None, x0_nonzero: bool = False,
                 stream=None):
    _check(_lib.spk_pc_chebyshev(A.handle, _dev(b, torch.float64, A.n, "b"),
                                 _dev(x, torch.float64, A.n, "x"),
                                 _dev(r_out, torch.float64, A.n, "r_out") if r_out is not None else None,
                                 int(steps), float(emin), float(emax), int(bool(x0_nonzero)),
                                 _stream(stream)),
           "spk_pc_chebyshev")


def mat_destroy(A: Mat):
    _check(_lib.spk_mat_destroy(A.handle), "spk_mat_destroy")


# ------------------------------------------------------------------ vectors
def vec_axpy(alpha: float, x, y, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_axpy(n, float(alpha), _dev(x, torch.float64, n, "x"),
                             _dev(y, torch.float64, n, "y"), _stream(stream)), "spk_vec_axpy")


def vec_aypx(beta: float, x, y, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_aypx(n, float(beta), _dev(x, torch.float64, n, "x"),
                             _dev(y, torch.float64, n, "y"), _stream(stream)), "spk_vec_aypx")


def vec_dot(x, y, result, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_dot(n, _dev(x, torch.float64, n, "x"), _dev(y, torch.float64, n, "y"),
                            _dev(result, torch.float64, None, "result"), _stream(stream)),
           "spk_vec_dot")


def vec_dot2(x, y, w, result, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_dot2(n, _dev(x, torch.float64, n, "x"), _dev(y, torch.float64, n, "y"),
                             _dev(w, torch.float64, n, "w"),
                             _dev(result, torch.float64, None, "result"), _stream(stream)),
           "spk_vec_dot2")


def vec_dot2_noalloc(x, y, w, result, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_dot2_noalloc(n, _dev(x, torch.float64, n, "x"), _dev(y, torch.float64, n, "y"),
                                     _dev(w, torch.float64, n, "w"),
                                     _dev(result, torch.float64, None, "result"), _stream(stream)),
           "spk_vec_dot2_noalloc")


def vec_nrm2(x, result, stream=None):
    n = x.numel()
    _check(_lib.spk_vec_nrm2(n, _dev(x, torch.float64, n, "x"),
                             _dev(result, torch.float64, None, "result"), _stream(stream)),
           "spk_vec_nrm2")


# ------------------------------------------------------------------ solver
def ksp_opts_default() -> KspOpts:
    o = KspOpts()
    _lib.spk_ksp_opts_default(ctypes.byref(o))
    return o


def ksp_opts(**kw) -> KspOpts:
    o = ksp_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _block(t: torch.Tensor, n: int, name: str):
    """A row-major n x k float64 CUDA block: (pointer, k)."""
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or t.shape[0] != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({n}, k) tensor")
    return P(t.data_ptr()), t.shape[1]


def mat_mult_multi(A: Mat, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Y = A X for the k columns of the row-major (n, k) blocks X and Y."""
    px, k = _block(X, A.n, "X")
    py, k2 = _block(Y, A.n, "Y")
    if k != k2:
        raise ValueError("X and Y must have the same number of columns")
    _check(_lib.spk_mat_mult_multi(A.handle, int(k), px, py, _stream(stream)), "spk_mat_mult_multi")


def ksp_solve_multi(A: Mat, B: torch.Tensor, X: torch.Tensor, opts: KspOpts | None = None,
                    stream=None) -> list:
    """k independent solves A X[:, j] = B[:, j] sharing every SpMM; returns
    one KspResult per column."""
    pb, k = _block(B, A.n, "B")
    px, k2 = _block(X, A.n, "X")
    if k != k2:
        raise ValueError("B and X must have the same number of columns")
    o = opts if opts is not None else ksp_opts_default()
    res = (KspResult * k)()
    _check(_lib.spk_ksp_solve_multi(A.handle, int(k), pb, px, ctypes.byref(o), res, _stream(stream)),
           "spk_ksp_solve_multi")
    return list(res)


def ksp_solve(A: Mat, b, x, opts: KspOpts | None = None, hist=None, stream=None) -> KspResult:
    """Solve A x = b.  ``hist`` (optional NumPy float64 array) receives the
    residual history."""
    o = opts if opts is not None else ksp_opts_default()
    if hist is not None:
        import numpy as np

        assert hist.dtype == np.float64 and hist.flags.c_contiguous
        o.hist = hist.ctypes.data_as(ctypes.POINTER(dbl))
        o.hist_len = hist.size
    res = KspResult()
    _check(_lib.spk_ksp_solve(A.handle, _dev(b, torch.float64, A.n, "b"),
                              _dev(x, torch.float64, A.n, "x"), ctypes.byref(o),
                              ctypes.byref(res), _stream(stream)), "spk_ksp_solve")
    return res


# ------------------------------------------------------------------ multigrid
def mg_opts_default() -> MgOpts:
    o = MgOpts()
    _lib.spk_mg_opts_default(ctypes.byref(o))
    return o


def mg_opts(**kw) -> MgOpts:
    o = mg_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Mg:
    """Owns an spk_mg hierarchy; keeps the finest matrix alive with it."""

    def __init__(self, handle: int, A: Mat):
        self.handle = P(handle)
        self.A = A
        self.info = mg_get_info(self)
        self.levels = self.info.levels

    def close(self):
        if self.handle:
            _lib.spk_mg_destroy(self.handle)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def mg_create(A: Mat, shape, opts: MgOpts | None = None, stream=None) -> Mg:
    """Multigrid hierarchy of A on a grid of the given extents (first fastest)."""
    sh = (i32 * 3)(*[int(v) for v in shape], *([1] * (3 - len(shape))))
    out = P()
    _check(_lib.spk_mg_create(A.handle, len(shape), sh, ctypes.byref(opts) if opts is not None else None,
                              _stream(stream), ctypes.byref(out)), "spk_mg_create")
    return Mg(out.value, A)


def mg_get_info(M: Mg) -> MgInfo:
    info = MgInfo()
    _check(_lib.spk_mg_get_info(M.handle, ctypes.byref(info)), "spk_mg_get_info")
    return info


def mg_copy_level(M: Mg, level: int):
    """(rowptr, col, val) NumPy copies of one level's matrix."""
    import numpy as np

    n, nnz = M.info.n[level], M.info.nnz[level]
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(max(nnz, 1), dtype=np.int32)
    va = np.empty(max(nnz, 1), dtype=np.float64)
    _check(_lib.spk_mg_copy_level(M.handle, level, P(rp.ctypes.data), P(ci.ctypes.data), P(va.ctypes.data)),
           "spk_mg_copy_level")
    return rp, ci[:nnz], va[:nnz]


def mg_apply(M: Mg, b: torch.Tensor, x: torch.Tensor, stream=None):
    n = M.info.n[0]
    _check(_lib.spk_mg_apply(M.handle, _dev(b, torch.float64, n, "b"), _dev(x, torch.float64, n, "x"),
                             _stream(stream)), "spk_mg_apply")


def mg_profile(M: Mg, b: torch.Tensor, x: torch.Tensor, reps: int = 10, stream=None) -> list:
    """Mean milliseconds per cycle spent on each level's own kernels."""
    n = M.info.n[0]
    ms = (dbl * 16)()
    _check(_lib.spk_mg_profile(M.handle, _dev(b, torch.float64, n, "b"), _dev(x, torch.float64, n, "x"),
                               int(reps), ms, _stream(stream)), "spk_mg_profile")
    return [ms[l] for l in range(M.levels)]


def ksp_solve_mg(M: Mg, b, x, opts: KspOpts | None = None, hist=None, stream=None) -> KspResult:
    """CG preconditioned by one multigrid cycle per iteration."""
    n = M.info.n[0]
    o = opts if opts is not None else ksp_opts_default()
    if hist is not None:
        import numpy as np

        assert hist.dtype == np.float64 and hist.flags.c_contiguous
        o.hist = hist.ctypes.data_as(ctypes.POINTER(dbl))
        o.hist_len = hist.size
    res = KspResult()
    _check(_lib.spk_ksp_solve_mg(M.handle, _dev(b, torch.float64, n, "b"), _dev(x, torch.float64, n, "x"),
                                 ctypes.byref(o), ctypes.byref(res), _stream(stream)), "spk_ksp_solve_mg")
    return res


def mg_destroy(M: Mg):
    M.close()


# ------------------------------------------------------------------ server
def server_opts_default() -> ServerOpts:
    o = ServerOpts()
    _lib.spk_server_opts_default(ctypes.byref(o))
    return o


class Server:
    def __init__(self, handle):
        self.handle = P(handle)

    def close(self):
        if self.handle:
            server_destroy(self)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def server_create(opts: ServerOpts | None = None, stream=None) -> Server:
    o = opts if opts is not None else server_opts_default()
    out = P()
    _check(_lib.spk_server_create(ctypes.byref(o), _stream(stream), ctypes.byref(out)),
           "spk_server_create")
    return Server(out.value)


def server_submit(S: Server, rowptr, colind, values, b, opts: KspOpts | None = None) -> int:
    import numpy as np

    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    t = u64()
    o = ctypes.byref(opts) if opts is not None else None
    rc = _lib.spk_server_submit(S.handle, rowptr.size - 1, colind.size, P(rowptr.ctypes.data),
                                P(colind.ctypes.data), P(values.ctypes.data), P(b.ctypes.data),
                                o, ctypes.byref(t))
    _check(rc, "spk_server_submit")
    return t.value


def server_progress(S: Server, max_steps: int = 1) -> int:
    rc = _lib.spk_server_progress(S.handle, max_steps)
    if rc < 0:
        raise SpkError(rc, "spk_server_progress")
    return rc


def server_poll(S: Server, ticket: int, x_host):
    """Returns (KspResult, done_time) when finished, None while in flight."""
    import numpy as np

    assert x_host.dtype == np.float64 and x_host.flags.c_contiguous
    res = KspResult()
    tdone = dbl()
    rc = _lib.spk_server_poll(S.handle, ticket, P(x_host.ctypes.data), ctypes.byref(res),
                              ctypes.byref(tdone))
    if rc == EBUSY:
        return None
    _check(rc, "spk_server_poll")
    return res, tdone.value


def server_completed(S: Server, cap: int = 256) -> list:
    """Tickets of requests finished since the last call (each reported once)."""
    buf = (u64 * cap)()
    k = _lib.spk_server_completed(S.handle, buf, int(cap))
    if k < 0:
        raise SpkError(k, "spk_server_completed")
    return list(buf[:k])


def server_destroy(S: Server):
    _check(_lib.spk_server_destroy(S.handle), "spk_server_destroy")


# ------------------------------------------------------------------ measurement
def bw_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    n = src.numel()
    _check(_lib.spk_bw_copy(n, _dev(src, torch.float64, n, "src"), _dev(dst, torch.float64, n, "dst"),
                            _stream(stream)), "spk_bw_copy")


def cache_flush(scratch: torch.Tensor, stream=None):
    _check(_lib.spk_cache_flush(P(scratch.data_ptr()), scratch.numel() * scratch.element_size(),
                                _stream(stream)), "spk_cache_flush")
