"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point the header declares, and rejects bad arguments on the host."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spk.h")
LIB = os.path.join(ROOT, "paper_2011_00715_amd", "libspk.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spk_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libspk.so not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (shares its HIP runtime with the library)

    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("spk_mat_create_csr", "spk_mat_mult", "spk_ksp_solve", "spk_server_create",
                     "spk_server_submit", "spk_server_progress", "spk_server_poll"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    from paper_2011_00715_amd import spk

    assert sorted(spk.EXPORTS) == declared_functions()


def test_host_side_validation_without_gpu(lib):
    from paper_2011_00715_amd import spk

    out = ctypes.c_void_p()
    f = spk._lib.spk_mat_create_csr
    assert f(-1, 0, None, None, None, 0, 0, None, ctypes.byref(out)) == spk.EINVAL
    assert "n = -1" in spk.last_error()
    assert f(4, 1 << 40, None, None, None, 0, 0, None, ctypes.byref(out)) == spk.EINVAL
    assert f(4, 4, None, None, None, 0, 0, None, ctypes.byref(out)) == spk.EINVAL  # NULL rowptr
    assert spk.status_str(spk.EZERODIAG) == "SPK_EZERODIAG"
    assert spk.reason_str(spk.DIVERGED_INDEFINITE_PC) == "DIVERGED_INDEFINITE_PC"
    o = spk.ksp_opts_default()
    assert (o.rtol, o.atol, o.maxit, o.graph_k, o.inner_rtol, o.max_outer) == (1e-8, 0.0, 10000, 8, 0.0, 100)
    so = spk.server_opts_default()
    assert so.max_slots > 0 and so.hbm_budget_bytes > 0
    assert spk.now() > 0
    # the smoother rejects a NULL handle before touching the device
    assert spk._lib.spk_pc_chebyshev(None, None, None, None, 2, 0.0, 0.0, 0, None) == spk.EINVAL
    assert "NULL" in spk.last_error()


def test_multigrid_host_validation_without_gpu(lib):
    from paper_2011_00715_amd import spk

    o = spk.mg_opts_default()
    assert (o.max_levels, o.coarse_max, o.smooth_steps, o.cycle, o.emin_frac, o.omega, o.precision) ==         (16, 1000, 2, 1, 0.1, 2.0, spk.PREC_FP64)
    assert ctypes.sizeof(spk.MgOpts) == 40
    assert ctypes.sizeof(spk.MgInfo) == 592
    out = ctypes.c_void_p()
    shape = (ctypes.c_int32 * 3)(4, 4, 1)
    assert spk._lib.spk_mg_create(None, 2, shape, None, None, ctypes.byref(out)) == spk.EINVAL
    assert "NULL" in spk.last_error() and not out.value
    info = spk.MgInfo()
    assert spk._lib.spk_mg_get_info(None, ctypes.byref(info)) == spk.EINVAL
    res = spk.KspResult()
    assert spk._lib.spk_ksp_solve_mg(None, None, None, None, ctypes.byref(res), None) == spk.EINVAL
    assert spk._lib.spk_mg_apply(None, None, None, None) == spk.EINVAL
    assert spk._lib.spk_mg_destroy(None) == spk.OK
