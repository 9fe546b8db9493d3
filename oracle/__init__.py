"""CPU oracle for the CSR SpMV / Jacobi-PCG path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2011_00715_amd``) never imports it, and the two share no code: the
oracle is plain serial C (``oracle.c``, built with gcc ``-O2
-ffp-contract=off``) reached through ctypes.  Inputs come from ``spkgen``.

Every function here is pinned by CPU tests (``tests/test_oracle_pins.py``)
against results fixed by mathematics -- closed-form Laplacian eigenpairs, exact
integer arithmetic, brute-force dense solves, finite termination of CG -- and
not against itself.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REASONS = {
    1: "CONVERGED_RTOL",
    2: "CONVERGED_ATOL",
    -1: "DIVERGED_ITS",
    -2: "DIVERGED_INDEFINITE_MAT",
    -3: "DIVERGED_INDEFINITE_PC",
    -4: "DIVERGED_NANORINF",
    -5: "DIVERGED_BREAKDOWN",
}


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(extra_flags=()) -> str:
    """Compile liboracle.so with gcc (always recompiles), and the same source
    with OpenMP as liboracle_omp.so (used only to time the oracle on all host
    cores)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
           *extra_flags, _SRC, "-o", _LIB, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-fopenmp",
           *extra_flags, _SRC, "-o", _LIB_OMP, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


_lib_omp = None


def load_omp():
    """The OpenMP build of the same oracle (parallel loops, fixed-order
    chunked inner products); threads from OMP_NUM_THREADS or all cores."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build()
        _lib_omp = load(_LIB_OMP)
    return _lib_omp


class _PcgResult(ctypes.Structure):
    _fields_ = [
        ("reason", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("rnorm0", ctypes.c_double),
        ("rnorm", ctypes.c_double),
        ("bnorm", ctypes.c_double),
        ("true_rel_residual", ctypes.c_double),
    ]


_PC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))

_lib = None


def load(path: str | None = None):
    """Load liboracle.so, building it first only if it does not exist."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build()
    lib = ctypes.CDLL(p)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    d = ctypes.c_double
    lib.orc_spmv.argtypes = [i32, P, P, P, P, P]
    lib.orc_spmv_f32.argtypes = [i32, P, P, P, P, P]
    lib.orc_spmv_abs.argtypes = [i32, P, P, P, P, P]
    lib.orc_spmv_rows.argtypes = [i32, P, P, P, P, P, P, P]
    lib.orc_dot.argtypes = [i32, P, P]
    lib.orc_dot.restype = d
    lib.orc_nrm2.argtypes = [i32, P]
    lib.orc_nrm2.restype = d
    lib.orc_axpy.argtypes = [i32, d, P, P]
    lib.orc_aypx.argtypes = [i32, d, P, P]
    lib.orc_diag_inv.argtypes = [i32, P, P, P, P]
    lib.orc_diag_inv.restype = ctypes.c_int
    lib.orc_jacobi_apply.argtypes = [i32, P, P, P]
    lib.orc_pcg.argtypes = [i32, P, P, P, P, P, d, d, i32, i32, P, i32,
                            ctypes.POINTER(_PcgResult)]
    lib.orc_pcg.restype = ctypes.c_int
    lib.orc_pcg_sr.argtypes = [i32, P, P, P, P, P, d, d, i32, i32, P, i32,
                               ctypes.POINTER(_PcgResult)]
    lib.orc_pcg_sr.restype = ctypes.c_int
    lib.orc_dense_cholesky_solve.argtypes = [i32, P, P]
    lib.orc_dense_cholesky_solve.restype = ctypes.c_int
    lib.orc_chebyshev.argtypes = [i32, P, P, P, P, P, P, i32, d, d, i32]
    lib.orc_chebyshev.restype = ctypes.c_int
    lib.orc_gershgorin.argtypes = [i32, P, P, P, P]
    lib.orc_gershgorin.restype = ctypes.c_int
    lib.orc_pcg_pc.argtypes = [i32, P, P, P, P, P, d, d, i32, i32, _PC_FN, P, P, i32,
                               ctypes.POINTER(_PcgResult)]
    lib.orc_pcg_pc.restype = ctypes.c_int
    lib.orc_dense_cholesky_factor.argtypes = [i32, P]
    lib.orc_dense_cholesky_factor.restype = ctypes.c_int
    lib.orc_dense_cholesky_subst.argtypes = [i32, P, P]
    lib.orc_mg_coarse_shape.argtypes = [i32, P, P]
    lib.orc_mg_galerkin.argtypes = [i32, P, P, P, i32, P, P, P, P]
    lib.orc_mg_galerkin.restype = ctypes.c_int64
    lib.orc_mg_restrict.argtypes = [i32, P, P, P]
    lib.orc_mg_prolong.argtypes = [i32, P, d, P, P]
    lib.orc_threads.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def threads(lib=None) -> int:
    """Threads the library's loops run on (1 for the serial build)."""
    return int((lib or load()).orc_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _csr(A):
    return _c(A.rowptr, np.int32), _c(A.col, np.int32)


def spmv(A, x, lib=None) -> np.ndarray:
    """y = A x in FP64 (long-double accumulation, rounded once)."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    x = _c(x, np.float64)
    y = np.empty(A.n, dtype=np.float64)
    lib.orc_spmv(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(x), _ptr(y))
    return y


def spmv_f32(A, x32, val32=None, lib=None) -> np.ndarray:
    """y = A32 x32 with FP32 values and x, exact sum rounded to FP32 once."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val if val32 is None else val32, np.float32)
    x = _c(x32, np.float32)
    y = np.empty(A.n, dtype=np.float32)
    lib.orc_spmv_f32(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(x), _ptr(y))
    return y


def spmv_abs(A, x, lib=None) -> np.ndarray:
    """sum_j |a_ij x_j| per row (the scale of the per-entry tolerance)."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    x = _c(x, np.float64)
    y = np.empty(A.n, dtype=np.float64)
    lib.orc_spmv_abs(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(x), _ptr(y))
    return y


def spmv_rows(A, x, rows, lib=None):
    """(A x)_i and sum_j |a_ij x_j| for the selected rows only."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    x = _c(x, np.float64)
    rows = _c(rows, np.int32)
    y = np.empty(rows.size, dtype=np.float64)
    ya = np.empty(rows.size, dtype=np.float64)
    lib.orc_spmv_rows(rows.size, _ptr(rows), _ptr(rp), _ptr(ci), _ptr(v), _ptr(x),
                      _ptr(y), _ptr(ya))
    return y, ya


def dot(x, y, lib=None) -> float:
    lib = lib or load()
    x = _c(x, np.float64)
    y = _c(y, np.float64)
    return lib.orc_dot(x.size, _ptr(x), _ptr(y))


def nrm2(x, lib=None) -> float:
    lib = lib or load()
    x = _c(x, np.float64)
    return lib.orc_nrm2(x.size, _ptr(x))


def axpy(alpha, x, y, lib=None) -> np.ndarray:
    """Returns alpha x + y (exact, rounded once)."""
    lib = lib or load()
    x = _c(x, np.float64)
    out = np.array(y, dtype=np.float64, copy=True)
    lib.orc_axpy(x.size, float(alpha), _ptr(x), _ptr(out))
    return out


def aypx(beta, x, y, lib=None) -> np.ndarray:
    """Returns x + beta y (exact, rounded once)."""
    lib = lib or load()
    x = _c(x, np.float64)
    out = np.array(y, dtype=np.float64, copy=True)
    lib.orc_aypx(x.size, float(beta), _ptr(x), _ptr(out))
    return out


def diag_inv(A, lib=None):
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    out = np.empty(A.n, dtype=np.float64)
    st = lib.orc_diag_inv(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(out))
    if st:
        raise ValueError("zero or missing diagonal")
    return out


def jacobi_apply(dinv, r, lib=None) -> np.ndarray:
    lib = lib or load()
    dinv = _c(dinv, np.float64)
    r = _c(r, np.float64)
    z = np.empty_like(r)
    lib.orc_jacobi_apply(r.size, _ptr(dinv), _ptr(r), _ptr(z))
    return z


def _pcg_out(res, hist, hist_len):
    out = {f: getattr(res, f) for f, _ in _PcgResult._fields_ if f != "pad_"}
    out["reason_str"] = REASONS.get(res.reason, str(res.reason))
    return out, (hist[: res.iterations + 1] if hist_len > 0 else None)


def pcg(A, b, x0=None, rtol=1e-8, atol=0.0, maxit=10000, hist_len=0, lib=None,
        single_reduction=False):
    """FP64 Jacobi-PCG (textbook, or the single-reduction Chronopoulos-Gear
    form).  Returns (x, result dict, history array or None)."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    b = _c(b, np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = np.full(max(hist_len, 1), np.nan)
    res = _PcgResult()
    fn = lib.orc_pcg_sr if single_reduction else lib.orc_pcg
    st = fn(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(b), _ptr(x), float(rtol),
                     float(atol), int(maxit), int(x0 is not None),
                     _ptr(hist) if hist_len > 0 else None, int(hist_len), ctypes.byref(res))
    if st:
        raise ValueError(f"oracle pcg failed with status {st}")
    out, hh = _pcg_out(res, hist, hist_len)
    return x, out, hh


def dense_cholesky_solve(D, b, lib=None):
    """Solve D x = b for dense SPD D; raises if D is not positive definite."""
    lib = lib or load()
    A = np.array(D, dtype=np.float64, copy=True, order="C")
    x = np.array(b, dtype=np.float64, copy=True)
    st = lib.orc_dense_cholesky_solve(A.shape[0], _ptr(A), _ptr(x))
    if st:
        raise ValueError("matrix is not positive definite")
    return x


def chebyshev(A, b, steps, emin, emax, x0=None, lib=None):
    """Jacobi-preconditioned Chebyshev iteration (`steps` steps on the
    spectral interval [emin, emax] of D^-1 A).  Returns (x, r)."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    b = _c(b, np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = np.empty(A.n)
    st = lib.orc_chebyshev(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(b), _ptr(x), _ptr(r), int(steps),
                           float(emin), float(emax), int(x0 is not None))
    if st:
        raise ValueError(f"oracle chebyshev failed with status {st}")
    return x, r


def gershgorin(A, lib=None) -> float:
    """max_i sum_j |a_ij| / |a_ii|: a bound on the spectrum of D^-1 A."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    out = ctypes.c_double(0.0)
    st = lib.orc_gershgorin(A.n, _ptr(rp), _ptr(ci), _ptr(v), ctypes.byref(out))
    if st:
        raise ValueError("zero or missing diagonal")
    return out.value


# ---------------------------------------------------------------- multigrid
# Geometric multigrid (Sec. 5.3: Jacobi-preconditioned Chebyshev smoothing on
# every level but the coarsest, a direct solve there, V- or W-cycles).  The
# grid transfers and coarse operators are the aggregation reading stated in
# oracle.c; the cycle is composed here from the C functions, in the order the
# method applies them.


def _shape3(shape):
    s = [int(v) for v in shape] + [1] * (3 - len(shape))
    return np.array(s, dtype=np.int32)


def coarse_shape(shape, lib=None):
    lib = lib or load()
    s = _shape3(shape)
    c = np.empty(3, dtype=np.int32)
    lib.orc_mg_coarse_shape(len(shape), _ptr(s), _ptr(c))
    return tuple(int(v) for v in c[: len(shape)])


def galerkin(A, shape, lib=None):
    """A_c = P^T A P for the aggregation prolongation on a grid of `shape`
    (first dimension fastest).  Returns a CSR of the same class as A."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    s = _shape3(shape)
    cs = coarse_shape(shape, lib)
    nc = int(np.prod(cs))
    crp = np.empty(nc + 1, dtype=np.int32)
    cap = max(int(rp[-1]), 1)
    cc = np.empty(cap, dtype=np.int32)
    cv = np.empty(cap, dtype=np.float64)
    nnz = lib.orc_mg_galerkin(A.n, _ptr(rp), _ptr(ci), _ptr(v), len(shape), _ptr(s),
                              _ptr(crp), _ptr(cc), _ptr(cv))
    if nnz < 0:
        raise ValueError(f"oracle galerkin failed with status {nnz}")
    return type(A)(nc, crp, cc[:nnz].copy(), cv[:nnz].copy())


def restrict(shape, r, lib=None):
    """b_c = P^T r: the sum over each aggregate."""
    lib = lib or load()
    s = _shape3(shape)
    r = _c(r, np.float64)
    bc = np.empty(int(np.prod(coarse_shape(shape, lib))))
    lib.orc_mg_restrict(len(shape), _ptr(s), _ptr(r), _ptr(bc))
    return bc


def prolong(shape, omega, xc, x, lib=None):
    """Returns x + omega P x_c."""
    lib = lib or load()
    s = _shape3(shape)
    xc = _c(xc, np.float64)
    out = np.array(x, dtype=np.float64, copy=True)
    lib.orc_mg_prolong(len(shape), _ptr(s), float(omega), _ptr(xc), _ptr(out))
    return out


class MGHierarchy:
    """Levels 0 (finest) .. L-1 (coarsest): matrices, grid shapes, smoother
    intervals and the Cholesky factor of the coarsest matrix."""

    def __init__(self, mats, shapes, steps, emin_frac, omega, cycle, chol):
        self.mats, self.shapes = mats, shapes
        self.steps, self.emin_frac, self.omega, self.cycle = steps, emin_frac, omega, cycle
        self.emax = [gershgorin(A) for A in mats[:-1]]
        self.chol = chol

    @property
    def levels(self):
        return len(self.mats)


def mg_setup(A, shape, max_levels=16, coarse_max=1000, steps=2, emin_frac=0.1, omega=2.0,
             cycle=1, lib=None):
    """Coarsen by aggregation while the level has more than coarse_max rows,
    fewer than max_levels levels exist and the grid can still shrink; the
    last level is factored for the direct solve."""
    lib = lib or load()
    mats, shapes = [A], [tuple(int(v) for v in shape)]
    while len(mats) < max_levels and mats[-1].n > coarse_max:
        cs = coarse_shape(shapes[-1], lib)
        if cs == shapes[-1]:
            break
        mats.append(galerkin(mats[-1], shapes[-1], lib))
        shapes.append(cs)
    Ac = mats[-1]
    D = np.zeros((Ac.n, Ac.n))
    for i in range(Ac.n):
        for k in range(Ac.rowptr[i], Ac.rowptr[i + 1]):
            D[i, Ac.col[k]] = Ac.val[k]
    L = np.ascontiguousarray(D)
    if lib.orc_dense_cholesky_factor(Ac.n, _ptr(L)):
        raise ValueError("coarsest matrix is not positive definite")
    return MGHierarchy(mats, shapes, steps, emin_frac, omega, cycle, L)


def mg_cycle(h, b, level=0, x0=None, lib=None):
    """One multigrid cycle on level `level` for right-hand side b, from x0
    (zero when None):
      pre-smoothing (Chebyshev, `steps` steps on [emin_frac g, g], g the
      Gershgorin bound of D^-1 A), restriction of the residual, the coarse
      cycle (twice for a W-cycle, the second from the first's result; once on
      the directly solved coarsest level), the correction x += omega P x_c,
      and post-smoothing from x."""
    lib = lib or load()
    if level == h.levels - 1:
        x = np.array(b, dtype=np.float64, copy=True)
        lib.orc_dense_cholesky_subst(x.size, _ptr(h.chol), _ptr(x))
        return x
    A, g = h.mats[level], h.emax[level]
    x, r = chebyshev(A, b, h.steps, h.emin_frac * g, g, x0=x0, lib=lib)
    bc = restrict(h.shapes[level], r, lib)
    xc = mg_cycle(h, bc, level + 1, lib=lib)
    if h.cycle == 2 and level + 1 < h.levels - 1:
        xc = mg_cycle(h, bc, level + 1, x0=xc, lib=lib)
    x = prolong(h.shapes[level], h.omega, xc, x, lib)
    x, _ = chebyshev(A, b, h.steps, h.emin_frac * g, g, x0=x, lib=lib)
    return x


def pcg_mg(A, h, b, x0=None, rtol=1e-8, atol=0.0, maxit=10000, hist_len=0, lib=None):
    """PCG (the stopping rules of pcg) preconditioned by one multigrid cycle
    from zero per iteration.  Returns (x, result dict, history or None)."""
    lib = lib or load()
    rp, ci = _csr(A)
    v = _c(A.val, np.float64)
    b = _c(b, np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = np.full(max(hist_len, 1), np.nan)
    res = _PcgResult()
    failed = []

    def pc(ctx, n, r, z):
        try:
            rr = np.ctypeslib.as_array(r, shape=(n,))
            zz = np.ctypeslib.as_array(z, shape=(n,))
            zz[:] = mg_cycle(h, rr.copy(), lib=lib)
            return 0
        except Exception as e:  # noqa: BLE001 - reported after the call
            failed.append(e)
            return -100

    cb = _PC_FN(pc)
    st = lib.orc_pcg_pc(A.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(b), _ptr(x), float(rtol),
                        float(atol), int(maxit), int(x0 is not None), cb, None,
                        _ptr(hist) if hist_len > 0 else None, int(hist_len), ctypes.byref(res))
    if failed:
        raise failed[0]
    if st:
        raise ValueError(f"oracle pcg_mg failed with status {st}")
    out, hh = _pcg_out(res, hist, hist_len)
    return x, out, hh
