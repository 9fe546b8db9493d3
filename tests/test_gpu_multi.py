"""Multiple right-hand sides: SpMM parity against the oracle applied column
by column (bit-exact on integer data, the sequential-sum bound elsewhere),
and the multi-RHS solve checked column by column like the single solve
(oracle true residual, iteration counts, solution error), plus independence
of the columns' stopping decisions."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import U64, check_spmv, mat_on_gpu, need_gpu, spmv_bound_rows, to_dev

pytestmark = pytest.mark.gpu


def _mats():
    rng = np.random.default_rng(5)
    D = rng.integers(-9, 10, size=(300, 300)) * (rng.random((300, 300)) < 0.05)
    D[np.arange(300), np.arange(300)] = 40
    yield "int_random_300", spkgen.dense_to_csr(D.astype(np.float64)), True
    yield "lap2d_61", spkgen.laplace2d5(61), True
    yield "lap3d_23", spkgen.laplace3d7(23), True
    yield "diff27_13", spkgen.diffusion3d27_lognormal(13, seed=1), False
    yield "powerlaw_20k", spkgen.powerlaw_spd(20000, seed=3), False
    # 130 diagonal-only rows (slices of one entry per row, no pairs) ahead of
    # a 2D Laplacian (slices of at most two pairs and a tail): on SELL the
    # SpMM takes its general loop for the one-entry slices and the pipelined
    # pairs for the others
    L = spkgen.laplace2d5(21)
    m = 130
    rowptr = np.concatenate([np.arange(m + 1), m + L.rowptr[1:]]).astype(np.int32)
    col = np.concatenate([np.arange(m), L.col + m]).astype(np.int32)
    val = np.concatenate([np.full(m, 3.0), L.val])
    yield "diag_then_lap2d", spkgen.CSR(m + L.n, rowptr, col, val), True


def _dev2(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kernel", ["auto", "sell", "sell16", "sell32"])
@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
def test_spmm_parity(k, kernel):
    """kernel "sell": the SELL-64 walk with the automatic offsets (shared per
    slice on the stencils, int16 per lane on the others; slices of up to
    three pairs gathered in one round, wider ones pipelined; LDS-staged
    stores); "sell16" / "sell32": per-lane int16 / int32 offsets."""
    spk = need_gpu()
    import torch

    for name, A, integer in _mats():
        M = mat_on_gpu(spk, A)
        if kernel != "auto":
            spk.mat_set_kernel(M, spk.KERNEL_SELL, {"sell": 0, "sell16": 16, "sell32": 32}[kernel])
        rng = np.random.default_rng(k)
        if integer:
            X = rng.integers(-50, 50, size=(A.n, k)).astype(np.float64)
        else:
            X = rng.uniform(-1, 1, size=(A.n, k))
        Y = torch.full((A.n, k), np.nan, dtype=torch.float64, device="cuda")
        spk.mat_mult_multi(M, _dev2(X), Y)
        Y = Y.cpu().numpy()
        for j in range(k):
            ref = oracle.spmv(A, X[:, j].copy())
            if integer:
                assert np.array_equal(Y[:, j], ref), f"{name} k={k} column {j}"
            else:
                scale = oracle.spmv_abs(A, X[:, j].copy())
                check_spmv(Y[:, j], ref, scale, spmv_bound_rows(A, "stream", 0, U64), f"{name} k={k} col {j}")
        M.close()


def _cases():
    yield "lap2d_64", spkgen.laplace2d5(64)
    yield "lap3d_24", spkgen.laplace3d7(24)
    yield "diff27_14", spkgen.diffusion3d27_lognormal(14, seed=0)
    yield "powerlaw_20k", spkgen.powerlaw_spd(20000, seed=1)


@pytest.mark.parametrize("kernel", ["auto", "sell", "sell16", "sell32"])
@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_24", "diff27_14", "powerlaw_20k"])
def test_multi_solve_parity(case, kernel):
    """auto: k = 4 on the automatic kernel; sell / sell16 / sell32: k = 8 on
    the SELL-64 layout with automatic (shared on the stencils) / int16 /
    int32 offsets (the pipelined, staged product and its flat p.q
    partials)."""
    spk = need_gpu()
    import torch

    A = dict(_cases())[case]
    M = mat_on_gpu(spk, A)
    k = 4
    if kernel != "auto":
        spk.mat_set_kernel(M, spk.KERNEL_SELL, {"sell": 0, "sell16": 16, "sell32": 32}[kernel])
        k = 8
    B = np.stack([spkgen.rhs_uniform(A.n, s) for s in range(k)], axis=1)
    X = torch.zeros((A.n, k), dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_multi(M, _dev2(B), X)
    X = X.cpu().numpy()
    for j in range(k):
        b = B[:, j].copy()
        xo, ro, _ = oracle.pcg(A, b)
        r = res[j]
        assert r.reason == spk.CONVERGED_RTOL, (j, spk.reason_str(r.reason))
        assert abs(r.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"]), (j, r.iterations, ro)
        x = X[:, j]
        tr = oracle.nrm2(b - oracle.spmv(A, x))
        assert tr <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)
        assert abs(r.true_rel_residual - tr / oracle.nrm2(b)) <= 1e-12
        assert r.bnorm == pytest.approx(ro["bnorm"], rel=1e-14)
        assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)
    M.close()


def test_multi_columns_stop_independently():
    """Column 0: an eigenvector (one iteration); column 1: b = 0 (x = 0 at
    once, whatever x0 was); column 2: the exact solution as x0 (zero
    iterations); column 3: a random right-hand side (full count)."""
    spk = need_gpu()
    import torch

    N = 32
    A = spkgen.laplace2d5(N)
    j = np.arange(1, N + 1)
    v = np.kron(np.sin(np.pi * 3 * j / (N + 1)), np.sin(np.pi * 5 * j / (N + 1)))
    xs = np.random.default_rng(2).integers(-9, 9, A.n).astype(np.float64)
    B = np.stack([oracle.spmv(A, v), np.zeros(A.n), oracle.spmv(A, xs), spkgen.rhs_uniform(A.n, 7)], axis=1)
    X0 = np.stack([np.zeros(A.n), np.ones(A.n), xs, np.zeros(A.n)], axis=1)
    M = mat_on_gpu(spk, A)
    X = _dev2(X0)
    res = spk.ksp_solve_multi(M, _dev2(B), X, spk.ksp_opts(x0_nonzero=1))
    X = X.cpu().numpy()
    assert res[0].reason == spk.CONVERGED_RTOL and res[0].iterations <= 2
    assert np.allclose(X[:, 0], v, rtol=0, atol=1e-8)
    assert res[1].reason == spk.CONVERGED_ATOL and res[1].iterations == 0 and not X[:, 1].any()
    assert res[2].reason == spk.CONVERGED_RTOL and res[2].iterations == 0
    assert np.array_equal(X[:, 2], xs)
    _, ro, _ = oracle.pcg(A, B[:, 3].copy())
    assert abs(res[3].iterations - ro["iterations"]) <= 2
    # maxit stops every column that has not converged
    X = torch.zeros((A.n, 4), dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_multi(M, _dev2(B), X, spk.ksp_opts(maxit=5))
    assert res[3].reason == spk.DIVERGED_ITS and res[3].iterations == 5
    assert res[0].reason == spk.CONVERGED_RTOL


def test_multi_graph_and_direct_identical():
    spk = need_gpu()
    import torch

    A = spkgen.diffusion3d27_lognormal(12, seed=3)
    M = mat_on_gpu(spk, A)
    B = np.stack([spkgen.rhs_uniform(A.n, s) for s in range(8)], axis=1)
    outs = []
    for gk in (8, 0, 3):
        X = torch.zeros((A.n, 8), dtype=torch.float64, device="cuda")
        res = spk.ksp_solve_multi(M, _dev2(B), X, spk.ksp_opts(graph_k=gk))
        outs.append((X.cpu().numpy(), [r.iterations for r in res]))
    for X, its in outs[1:]:
        assert np.array_equal(X, outs[0][0]) and its == outs[0][1]


def test_multi_errors():
    spk = need_gpu()
    import torch

    A = spkgen.laplace2d5(8)
    M = mat_on_gpu(spk, A)
    B = torch.ones((A.n, 3), dtype=torch.float64, device="cuda")
    X = torch.zeros((A.n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(spk.SpkError) as e:
        spk.ksp_solve_multi(M, B, X)
    assert e.value.status == spk.EINVAL
    with pytest.raises(spk.SpkError):
        spk.mat_mult_multi(M, B, X)
    B4 = torch.ones((A.n, 4), dtype=torch.float64, device="cuda")
    X4 = torch.zeros((A.n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(spk.SpkError):
        spk.ksp_solve_multi(M, B4, X4, spk.ksp_opts(precision=spk.PREC_MIXED))
    with pytest.raises(spk.SpkError):
        spk.ksp_solve_multi(M, B4, B4)
