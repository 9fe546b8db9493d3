"""Jacobi-PCG parity: the HIP solver against the oracle on the same seeded
inputs.  CG iterates depend on rounding, so the contract is: the true residual
meets the tolerance for both, the iteration counts agree within max(2, 1%),
the first 20 recursive residual norms agree to 1e-10 relative, and the
solution error against the oracle stays within kappa * rtol."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import mat_on_gpu, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _solve(spk, M, b, **kw):
    import torch

    hist = np.full(kw.pop("hist_len", 64), np.nan)
    x0 = kw.pop("x0", None)
    x = to_dev(x0) if x0 is not None else torch.zeros(M.n, dtype=torch.float64, device="cuda")
    o = spk.ksp_opts(**kw)
    if x0 is not None:
        o.x0_nonzero = 1
    res = spk.ksp_solve(M, to_dev(b), x, o, hist=hist)
    return x.cpu().numpy(), res, hist


def _cases():
    yield "lap2d_64", spkgen.laplace2d5(64), 0
    yield "lap3d_24", spkgen.laplace3d7(24), 1
    yield "diff27_14", spkgen.diffusion3d27_lognormal(14, seed=0), 2
    yield "powerlaw_20k", spkgen.powerlaw_spd(20000, seed=1), 3


@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_24", "diff27_14", "powerlaw_20k"])
@pytest.mark.parametrize("kernel", ["auto", "vector", "merge", "sell", "sell_sigma"])
def test_pcg_fp64_parity(case, kernel):
    spk = need_gpu()
    name, A, seed = [c for c in _cases() if c[0] == case][0]
    M = mat_on_gpu(spk, A)
    if kernel == "vector":
        spk.mat_set_kernel(M, spk.KERNEL_VECTOR, 8)
    elif kernel == "merge":
        spk.mat_set_kernel(M, spk.KERNEL_MERGE, 0)
    elif kernel == "sell":
        spk.mat_set_kernel(M, spk.KERNEL_SELL, 0)
    elif kernel == "sell_sigma":
        spk.mat_set_kernel(M, spk.KERNEL_SELL_SIGMA, 256)
    b = spkgen.rhs_uniform(A.n, seed)
    x, res, hist = _solve(spk, M, b, hist_len=4000)
    xo, ro, ho = oracle.pcg(A, b, rtol=1e-8, hist_len=4000)
    assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
    assert abs(res.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    k = min(20, res.iterations, ro["iterations"])
    assert np.allclose(hist[:k + 1], ho[:k + 1], rtol=1e-10, atol=0), (hist[:k + 1], ho[:k + 1])
    # the oracle recomputes the true residual of the GPU's x
    r = b - oracle.spmv(A, x)
    assert oracle.nrm2(r) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)
    assert abs(res.true_rel_residual - oracle.nrm2(r) / oracle.nrm2(b)) <= 1e-12
    assert res.bnorm == pytest.approx(ro["bnorm"], rel=1e-14)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert err <= 1e-5, err  # both within kappa * 1e-8 of the solution


@pytest.mark.parametrize("width", [16, 32])
def test_pcg_wide_sell_product(width):
    """Rows of about 110 entries forced onto SELL: each lane of the
    persistent grid would stream more than 96 stored entries, so the PCG
    product runs one wavefront per slice and a one-block fold of its partials
    (the path the 160^3 27-point system takes).  int16 column offsets (band
    +-55) and int32 offsets (a +-40000 coupling).  FP64: the first 20
    residual norms within 1e-10 of the oracle's, the iteration count, the
    oracle's true residual; mixed: the oracle's true residual and the
    solution error."""
    spk = need_gpu()
    n = 65536
    offs = list(range(1, 56)) if width == 16 else list(range(1, 55)) + [40000]
    A = spkgen.banded_spd(n, offs, seed=width, negative=True)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    spk.mat_set_kernel(M, spk.KERNEL_SELL, width)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sell" and M.info.lanes == width
    nblk = n // 256  # tiles of 256 rows, one block each (fewer than 2048)
    assert M.info.stored_nnz > 96 * 256 * nblk  # the wide product's rule
    b = spkgen.rhs_uniform(n, 4)
    x, res, hist = _solve(spk, M, b, hist_len=400)
    xo, ro, ho = oracle.pcg(A, b, rtol=1e-8, hist_len=400)
    assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
    assert ro["iterations"] >= 20
    assert abs(res.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    assert np.allclose(hist[:21], ho[:21], rtol=1e-10, atol=0), (hist[:21], ho[:21])
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)
    xm, rm, _ = _solve(spk, M, b, precision=spk.PREC_MIXED)
    assert rm.reason == spk.CONVERGED_RTOL and rm.fallback_fp64 == 0, rm.as_dict()
    assert oracle.nrm2(b - oracle.spmv(A, xm)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(xm - xo) <= 1e-5 * np.linalg.norm(xo)
    assert rm.inner_iterations <= 1.1 * ro["iterations"] + 2


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pcg_profiled_solve_same_result(prec):
    """opts.profile (one iteration per launch batch, an event pair around
    every product) gives the bits of the graph-replayed solve, and times one
    product per counted iteration."""
    spk = need_gpu()
    A = spkgen.diffusion3d27_lognormal(16, seed=2)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    b = spkgen.rhs_uniform(A.n, 1)
    x0, r0, _ = _solve(spk, M, b, precision=p)
    x1, r1, _ = _solve(spk, M, b, precision=p, profile=1)
    assert np.array_equal(x0, x1)
    assert (r0.iterations, r0.inner_iterations, r0.outer_steps) == (r1.iterations, r1.inner_iterations,
                                                                    r1.outer_steps)
    counted = r1.inner_iterations if p == spk.PREC_MIXED else r1.iterations
    assert r1.product_launches == counted > 0
    assert 0 < r1.product_ms < 1e3 * r1.seconds
    assert r0.product_launches == 0 and r0.product_ms == 0.0
    # a fixed number of iterations (rtol 0): every launch is an iteration
    _, r2, _ = _solve(spk, M, b, rtol=0.0, maxit=37, profile=1)
    assert r2.reason == spk.DIVERGED_ITS and r2.iterations == 37 and r2.product_launches == 37
    with pytest.raises(spk.SpkError):
        _solve(spk, M, b, profile=1, single_reduction=1)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_ir"])
@pytest.mark.parametrize("case", ["lap3d_30", "lap2d_90", "diff27_14"])
def test_pcg_fused_iteration_equals_three_kernels(case, prec):
    """SELL on the persistent grid takes the fused iteration (B, then F: the
    p/x pass fused into the next product, p in two alternating buffers); a
    profiled solve runs the three-kernel iteration on the same matrix.  Both
    give the same bits, iteration counts and refinement steps, in FP64 and
    in both mixed-precision readings, and meet the oracle's true residual."""
    spk = need_gpu()
    A = {"lap3d_30": spkgen.laplace3d7(30, shift=0.05), "lap2d_90": spkgen.laplace2d5(90),
         "diff27_14": spkgen.diffusion3d27_lognormal(14, seed=4)}[case]
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    spk.mat_set_kernel(M, spk.KERNEL_SELL, 0)
    p = {"fp64": spk.PREC_FP64, "mixed": spk.PREC_MIXED, "mixed_ir": spk.PREC_MIXED_IR}[prec]
    b = spkgen.rhs_uniform(A.n, 7)
    xf, rf, hf = _solve(spk, M, b, precision=p, hist_len=64)
    xt, rt, ht = _solve(spk, M, b, precision=p, hist_len=64, profile=1)
    assert rf.reason == spk.CONVERGED_RTOL, rf.as_dict()
    assert np.array_equal(xf, xt)
    assert (rf.iterations, rf.inner_iterations, rf.outer_steps, rf.restarts) == \
        (rt.iterations, rt.inner_iterations, rt.outer_steps, rt.restarts)
    assert np.array_equal(hf, ht, equal_nan=True)
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, xf)) <= 1e-8 * bn * (1 + 1e-6)
    # and a second solve on the same handle (buffers left by the first)
    xf2, rf2, _ = _solve(spk, M, b, precision=p, hist_len=64)
    assert np.array_equal(xf2, xf) and rf2.iterations == rf.iterations


@pytest.mark.parametrize("case", ["lap3d_30", "lap2d_90", "diff27_14", "diff27_100_wide"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pcg_shared_offsets_same_bits(case, prec):
    """The shared-offset SELL layout (the automatic choice on stencils) and
    per-lane int16 offsets give the same solves bit for bit, in FP64 and
    mixed precision, on the fused iteration, the three-kernel one and (27-point
    100^3: more stored entries than 1024 blocks' lanes take 96 each) the wide
    product."""
    spk = need_gpu()
    A = {"lap3d_30": spkgen.laplace3d7(30, shift=0.05), "lap2d_90": spkgen.laplace2d5(90),
         "diff27_14": spkgen.diffusion3d27_lognormal(14, seed=4),
         "diff27_100_wide": spkgen.diffusion3d27_lognormal(100, seed=2)}[case]
    p = {"fp64": spk.PREC_FP64, "mixed": spk.PREC_MIXED}[prec]
    b = spkgen.rhs_uniform(A.n, 3)
    res = []
    for param in (spk.SELL_SHARED, 16):
        M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
        spk.mat_set_kernel(M, spk.KERNEL_SELL, param)
        assert (M.info.lanes == 0) == (param == spk.SELL_SHARED)
        if case.endswith("_wide"):
            assert M.info.stored_nnz > 96 * 256 * 1024  # the wide product's rule
        for prof in (0, 1):
            x, r, h = _solve(spk, M, b, precision=p, hist_len=64, profile=prof)
            res.append((x, (r.reason, r.iterations, r.inner_iterations, r.outer_steps), h))
        M.close()
    x0, r0, h0 = res[0]
    assert r0[0] == spk.CONVERGED_RTOL
    for x, r, h in res[1:]:
        assert np.array_equal(x, x0) and r == r0
        assert np.array_equal(h, h0, equal_nan=True)
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, x0)) <= 1e-8 * bn * (1 + 1e-6)


@pytest.mark.parametrize("edge", ["maxit_5", "restarts", "x0"])
def test_pcg_fused_iteration_edge_cases(edge):
    """The fused and three-kernel iterations agree bit for bit where a solve
    stops inside a batch (maxit), through the true-residual restarts (an
    unreachable rtol: the fused start kernel after every re-setup), and from
    a nonzero initial guess."""
    spk = need_gpu()
    A = spkgen.laplace2d5(32)
    M = mat_on_gpu(spk, A)
    spk.mat_set_kernel(M, spk.KERNEL_SELL, 0)
    b = spkgen.rhs_uniform(A.n, 0)
    kw = {"maxit_5": dict(maxit=5), "restarts": dict(rtol=1e-17, maxit=100000),
          "x0": dict(x0=spkgen.rhs_uniform(A.n, 5))}[edge]
    xf, rf, hf = _solve(spk, M, b, hist_len=4000, **dict(kw))
    xt, rt, ht = _solve(spk, M, b, hist_len=4000, profile=1, **dict(kw))
    assert np.array_equal(xf, xt)
    assert (rf.reason, rf.iterations, rf.restarts) == (rt.reason, rt.iterations, rt.restarts)
    assert np.array_equal(hf, ht, equal_nan=True)
    if edge == "maxit_5":
        assert rf.reason == spk.DIVERGED_ITS and rf.iterations == 5
        xo, _, _ = oracle.pcg(A, b, maxit=5)
        assert np.allclose(xf, xo, rtol=1e-12, atol=1e-14)
    if edge == "restarts":
        assert rf.restarts >= 1


def test_pcg_graph_and_direct_launch_identical():
    spk = need_gpu()
    A = spkgen.diffusion3d27_lognormal(12, seed=3)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    outs = []
    for gk in (8, 0, 3, 8):
        x, res, _ = _solve(spk, M, b, graph_k=gk)
        outs.append((x, res.iterations, res.rnorm))
    for x, it, rn in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and it == outs[0][1] and rn == outs[0][2]


def test_pcg_reasons():
    spk = need_gpu()
    A = spkgen.laplace2d5(10)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    x, res, _ = _solve(spk, M, b, maxit=3)
    xo, ro, _ = oracle.pcg(A, b, maxit=3)
    assert res.reason == spk.DIVERGED_ITS and res.iterations == 3
    assert np.allclose(x, xo, rtol=1e-12, atol=1e-14)
    x, res, _ = _solve(spk, M, b, maxit=0)
    assert res.reason == spk.DIVERGED_ITS and res.iterations == 0 and not x.any()
    x, res, _ = _solve(spk, M, np.zeros(A.n))
    assert res.reason == spk.CONVERGED_ATOL and res.iterations == 0 and not x.any()
    x, res, _ = _solve(spk, M, np.zeros(A.n), x0=np.ones(A.n))
    assert res.reason == spk.CONVERGED_ATOL and not x.any()
    bn = b.copy()
    bn[3] = np.nan
    _, res, _ = _solve(spk, M, bn)
    assert res.reason == spk.DIVERGED_NANORINF
    An = spkgen.CSR(A.n, A.rowptr, A.col, -A.val)
    _, res, _ = _solve(spk, mat_on_gpu(spk, An), b)
    assert res.reason == spk.DIVERGED_INDEFINITE_PC
    Ai = spkgen.dense_to_csr(np.array([[1.0, 2.0], [2.0, 1.0]]))
    x, res, _ = _solve(spk, mat_on_gpu(spk, Ai), np.array([1.0, -1.0]))
    assert res.reason == spk.DIVERGED_INDEFINITE_MAT and res.iterations == 0 and not x.any()
    _, res, _ = _solve(spk, M, b, rtol=0.0, atol=1e-3)
    _, ro, _ = oracle.pcg(A, b, rtol=0.0, atol=1e-3)
    assert res.reason == spk.CONVERGED_ATOL and res.iterations == ro["iterations"]
    xs = np.linalg.solve(spkgen.to_dense(A), b)
    _, res, _ = _solve(spk, M, b, x0=xs)
    assert res.iterations == 0 and res.reason > 0
    Z = spkgen.dense_to_csr(np.array([[1.0, 2.0], [2.0, 0.0]]))
    MZ = mat_on_gpu(spk, Z)
    with pytest.raises(spk.SpkError) as e:
        _solve(spk, MZ, np.ones(2))
    assert e.value.status == spk.EZERODIAG


def test_pcg_x0_nonzero_matches_oracle():
    spk = need_gpu()
    A = spkgen.laplace3d7(16)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 2)
    x0 = spkgen.rhs_uniform(A.n, 3)
    x, res, hist = _solve(spk, M, b, x0=x0, hist_len=400)
    xo, ro, ho = oracle.pcg(A, b, x0=x0, hist_len=400)
    assert abs(res.iterations - ro["iterations"]) <= 2
    assert np.allclose(hist[:21], ho[:21], rtol=1e-10)


def test_pcg_true_residual_restart_rule():
    spk = need_gpu()
    A = spkgen.laplace2d5(32)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    _, res, _ = _solve(spk, M, b, rtol=1e-17, maxit=100000)
    assert res.reason in (spk.DIVERGED_BREAKDOWN, spk.CONVERGED_RTOL)
    if res.reason == spk.DIVERGED_BREAKDOWN:
        assert res.restarts == 3
    assert res.true_rel_residual < 1e-13


@pytest.mark.parametrize("case", ["lap2d_64", "diff27_14", "powerlaw_20k", "diff27_14/sell"])
@pytest.mark.parametrize("mode", ["mixed", "mixed_ir"])
def test_pcg_mixed_precision(case, mode):
    spk = need_gpu()
    case, _, kern = case.partition("/")
    name, A, seed = [c for c in _cases() if c[0] == case][0]
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    if kern == "sell":
        spk.mat_set_kernel(M, spk.KERNEL_SELL, 0)
    b = spkgen.rhs_uniform(A.n, seed)
    prec = spk.PREC_MIXED if mode == "mixed" else spk.PREC_MIXED_IR
    x, res, hist = _solve(spk, M, b, precision=prec)
    assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
    assert res.fallback_fp64 == 0
    if mode == "mixed":  # reliable updates keep CG's iteration count close to FP64's
        _, ro, _ = oracle.pcg(A, b, rtol=1e-8)
        assert res.inner_iterations <= 1.25 * ro["iterations"] + 10, (res.inner_iterations, ro["iterations"])
    assert res.outer_steps >= 1 and res.inner_iterations > 0
    r = b - oracle.spmv(A, x)
    rel = oracle.nrm2(r) / oracle.nrm2(b)
    assert rel <= 1e-8 * (1 + 1e-6), rel
    xo, _, _ = oracle.pcg(A, b, rtol=1e-8)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert err <= 1e-5, err
    # outer residuals decrease
    h = hist[: res.outer_steps + 1]
    assert np.all(np.diff(h) < 0)


@pytest.mark.parametrize("kernel", ["auto", "sell"])
def test_pcg_mixed_without_flag_converts_lazily(kernel):
    spk = need_gpu()
    A = spkgen.laplace2d5(40)
    M = mat_on_gpu(spk, A)
    if kernel == "sell":
        spk.mat_set_kernel(M, spk.KERNEL_SELL, 0)
        _, r64, _ = _solve(spk, M, spkgen.rhs_uniform(A.n, 0))  # FP64 workspace first
        assert r64.reason == spk.CONVERGED_RTOL
    assert M.info.has_f32 == 0
    b = spkgen.rhs_uniform(A.n, 0)
    _, res, _ = _solve(spk, M, b, precision=spk.PREC_MIXED)
    assert res.reason == spk.CONVERGED_RTOL
    assert spk.mat_get_info(M).has_f32 == 1


def test_pcg_repeat_bitwise():
    spk = need_gpu()
    A = spkgen.powerlaw_spd(20000, seed=2)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 9)
    x1, r1, _ = _solve(spk, M, b)
    x2, r2, _ = _solve(spk, M, b)
    assert np.array_equal(x1, x2) and r1.iterations == r2.iterations
    x3, r3, _ = _solve(spk, M, b, precision=spk.PREC_MIXED)
    x4, r4, _ = _solve(spk, M, b, precision=spk.PREC_MIXED)
    assert np.array_equal(x3, x4) and r3.inner_iterations == r4.inner_iterations


@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_24", "diff27_14", "powerlaw_20k"])
@pytest.mark.parametrize("kernel", ["auto", "stream", "vector", "merge"])
def test_pcg_single_reduction_parity(case, kernel):
    """Single-reduction (Chronopoulos-Gear) solve against the single-reduction
    oracle, with the same contract as the textbook solve."""
    spk = need_gpu()
    name, A, seed = [c for c in _cases() if c[0] == case][0]
    M = mat_on_gpu(spk, A)
    if kernel == "stream":
        spk.mat_set_kernel(M, spk.KERNEL_STREAM, 0)
    elif kernel == "vector":
        spk.mat_set_kernel(M, spk.KERNEL_VECTOR, 8)
    elif kernel == "merge":
        spk.mat_set_kernel(M, spk.KERNEL_MERGE, 0)
    b = spkgen.rhs_uniform(A.n, seed)
    x, res, hist = _solve(spk, M, b, hist_len=4000, single_reduction=1)
    xo, ro, ho = oracle.pcg(A, b, rtol=1e-8, hist_len=4000, single_reduction=True)
    assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
    assert abs(res.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    k = min(20, res.iterations, ro["iterations"])
    assert np.allclose(hist[:k + 1], ho[:k + 1], rtol=1e-10, atol=0), (hist[:k + 1], ho[:k + 1])
    r = b - oracle.spmv(A, x)
    assert oracle.nrm2(r) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)
    assert abs(res.true_rel_residual - oracle.nrm2(r) / oracle.nrm2(b)) <= 1e-12
    assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)


def test_pcg_single_reduction_graph_direct_and_reasons():
    spk = need_gpu()
    A = spkgen.diffusion3d27_lognormal(12, seed=3)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    outs = []
    for gk in (8, 0, 5):
        x, res, _ = _solve(spk, M, b, graph_k=gk, single_reduction=1)
        outs.append((x, res.iterations, res.rnorm))
    for x, it, rn in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and it == outs[0][1] and rn == outs[0][2]
    # the same matrix and right-hand side through the textbook solve
    xt, rt, _ = _solve(spk, M, b)
    assert abs(rt.iterations - outs[0][1]) <= 2
    # maxit, b = 0, exact start
    _, r, _ = _solve(spk, M, b, maxit=7, single_reduction=1)
    assert r.reason == spk.DIVERGED_ITS and r.iterations == 7
    x, r, _ = _solve(spk, M, np.zeros(A.n), single_reduction=1)
    assert r.reason == spk.CONVERGED_ATOL and r.iterations == 0 and not x.any()
    A2 = spkgen.laplace2d5(20)
    M2 = mat_on_gpu(spk, A2)
    xs = np.random.default_rng(0).integers(-5, 5, A2.n).astype(np.float64)
    x, r, _ = _solve(spk, M2, oracle.spmv(A2, xs), x0=xs, single_reduction=1)
    assert r.iterations == 0 and np.array_equal(x, xs)
    with pytest.raises(spk.SpkError):
        _solve(spk, M2, xs, single_reduction=1, precision=spk.PREC_MIXED)
