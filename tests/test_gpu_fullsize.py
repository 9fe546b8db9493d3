"""Parity at the configurations' full sizes, in the launch configuration the
bench times: every row of every SpMV compared with the oracle's product,
solves checked through the oracle's own true residual of the GPU solution and
its FP64 iteration counts."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import mat_on_gpu, need_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


class _Ref:
    """The oracle's product y = A x and its per-row scale sum_j |a_ij x_j|,
    computed once per (A, x) and compared with every kernel run on them."""

    def __init__(self, A, x):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = oracle.spmv(A, self.x)
        self.scale = oracle.spmv_abs(A, self.x)


def _spmv_all(spk, M, A, ref, tol=1e-14):
    """Every row of the FP64 product against the oracle: |dy_i| <= tol * sum_j
    |a_ij x_j| (tol = 0: bit-exact)."""
    import torch

    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    spk.mat_mult(M, to_dev(ref.x), y)
    yg = y.cpu().numpy()
    err = np.abs(yg - ref.y)
    bad = err > tol * ref.scale
    if bad.any():
        i = int(np.argmax(err / np.maximum(ref.scale, 1e-300)))
        raise AssertionError(f"{int(bad.sum())} of {A.n} rows exceed {tol}; worst row {i}: "
                             f"gpu {yg[i]!r} oracle {ref.y[i]!r} scale {ref.scale[i]!r}")
    return yg


def _spmv_f32_all(spk, M, A, x32, yo32, scale, ulps):
    """Every row of the FP32-value product against the oracle's exact product
    of the FP32-rounded values and x: |dy_i| <= ulps * 2^-24 * sum_j |a_ij x_j|
    (ulps = 0: bit-exact)."""
    import torch

    y32 = torch.empty(A.n, dtype=torch.float32, device="cuda")
    spk.mat_mult_f32(M, to_dev(x32), y32)
    yg = y32.cpu().numpy().astype(np.float64)
    err = np.abs(yg - yo32)
    bad = err > ulps * 2.0**-24 * scale
    assert not bad.any(), (int(bad.sum()), float(np.max(err / np.maximum(scale, 1e-300))))


def _solve(spk, M, b, **kw):
    import torch

    x = torch.zeros(M.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve(M, to_dev(b), x, spk.ksp_opts(**kw))
    return x.cpu().numpy(), res


@pytest.mark.parametrize("seed", range(5))
def test_c1_all_seeds(seed):
    spk = need_gpu()
    A = spkgen.laplace2d5(64)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, seed)
    x, res = _solve(spk, M, b)
    _, ro, _ = oracle.pcg(A, b)
    assert res.reason == spk.CONVERGED_RTOL
    assert abs(res.iterations - ro["iterations"]) <= 2
    assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)


def test_c2_spmv_and_pcg():
    spk = need_gpu()
    import torch

    A = spkgen.laplace3d7(128)
    assert (A.n, A.nnz) == (2097152, 14581760)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sell" and M.info.lanes == 0  # offsets shared per slice
    # bit-exact on integer data, 1e-14 on the bench's x (rhs of seed 0); FP32
    # values bit-exact on integers, 16 FP32 ulps of the row scale on the rhs
    xi = np.random.default_rng(3).integers(-100, 100, A.n).astype(np.float64)
    b = spkgen.rhs_uniform(A.n, 0)
    ri, rb = _Ref(A, xi), _Ref(A, b)
    b32 = b.astype(np.float32)
    yo32, sc32 = oracle.spmv_f32(A, b32), oracle.spmv_abs(A, b32.astype(np.float64))

    def check_all():
        _spmv_all(spk, M, A, ri, tol=0.0)
        _spmv_all(spk, M, A, rb)
        _spmv_f32_all(spk, M, A, xi.astype(np.float32), ri.y, ri.scale, 0)
        _spmv_f32_all(spk, M, A, b32, yo32, sc32, 16)

    check_all()
    # the stream family on the same matrix, then back to the selected one
    spk.mat_set_kernel(M, spk.KERNEL_STREAM, 0)
    check_all()
    spk.mat_set_kernel(M, spk.KERNEL_AUTO, 0)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sell"
    check_all()
    x64, r64 = _solve(spk, M, b)
    xo, ro, ho = oracle.pcg(A, b, hist_len=40)
    assert r64.reason == spk.CONVERGED_RTOL
    assert abs(r64.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, x64)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(x64 - xo) <= 1e-5 * np.linalg.norm(xo)
    xm, rm = _solve(spk, M, b, precision=spk.PREC_MIXED)
    assert rm.reason == spk.CONVERGED_RTOL and rm.fallback_fp64 == 0
    assert oracle.nrm2(b - oracle.spmv(A, xm)) <= 1e-8 * bn * (1 + 1e-6)
    assert rm.inner_iterations <= 1.1 * ro["iterations"]
    # the fused FP32 inner iteration at this size against the three-kernel
    # iteration of a profiled solve: the same bits (FP64 runs three kernels
    # here either way: its fused working set would not fit the cache)
    for prec, xf, rf in ((spk.PREC_FP64, x64, r64), (spk.PREC_MIXED, xm, rm)):
        xt, rt = _solve(spk, M, b, precision=prec, profile=1)
        assert np.array_equal(xt, xf)
        assert (rt.iterations, rt.inner_iterations, rt.outer_steps) == (rf.iterations, rf.inner_iterations,
                                                                        rf.outer_steps)



def _cached_bits(A, vectors, budget):
    """The load-policy bits the library documents: ordinary loads when the
    SELL layout and `vectors` n-vectors fit `budget` bytes (per precision)."""
    lens = np.diff(A.rowptr)
    lens = np.concatenate([lens, np.zeros(-A.n % 64, lens.dtype)])
    stored = 64 * int(lens.reshape(-1, 64).max(axis=1).sum())
    fixed = 4 * ((A.n + 63) // 64 + 1) + A.n
    b64 = 10 * stored + fixed + 8 * vectors * A.n <= budget
    b32 = 6 * stored + fixed + 4 * vectors * A.n <= budget
    return int(b64) | int(b32) << 1


def test_sell_load_policy_split_by_precision():
    """150^3 7-point: with the 6 vectors of a Krylov iteration the FP64
    layout (236 MB) does not fit the 256 MiB budget and the FP32 one does;
    with the x and y of a standalone product both fit 288 MiB.  Both products
    are bit-exact on integer data and within 1e-14 (FP64) of the oracle on the
    rhs, and the FP32 product matches the oracle's FP32 product to 16 FP32
    ulps of the row's absolute sum."""
    spk = need_gpu()
    import torch

    A = spkgen.laplace3d7(150)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sell"
    it, sp = _cached_bits(A, 6, 256 << 20), _cached_bits(A, 2, 288 << 20)
    assert (it, sp) == (2, 3)
    assert M.info.cached_loads == it | sp << 2
    xi = np.random.default_rng(5).integers(-100, 100, A.n).astype(np.float64)
    b = spkgen.rhs_uniform(A.n, 1)
    ri = _Ref(A, xi)
    _spmv_all(spk, M, A, ri, tol=0.0)
    _spmv_all(spk, M, A, _Ref(A, b))
    _spmv_f32_all(spk, M, A, xi.astype(np.float32), ri.y, ri.scale, 0)
    b32 = b.astype(np.float32)
    _spmv_f32_all(spk, M, A, b32, oracle.spmv_f32(A, b32), oracle.spmv_abs(A, b32.astype(np.float64)), 16)


def test_c3_fp64_and_mixed():
    spk = need_gpu()
    A = spkgen.diffusion3d27_lognormal(160, seed=0)
    assert (A.n, A.nnz) == (4096000, 109215352)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sell"
    b = spkgen.rhs_uniform(A.n, 0)
    _spmv_all(spk, M, A, _Ref(A, b))
    b32 = b.astype(np.float32)
    # a sequential FMA chain over a 27-entry row: at most 28 FP32 units of
    # the row scale (the FP64 check's 1e-14 has the same origin)
    _spmv_f32_all(spk, M, A, b32, oracle.spmv_f32(A, b32), oracle.spmv_abs(A, b32.astype(np.float64)),
                  int(A.row_lengths().max()) + 1)
    bn = oracle.nrm2(b)
    x64, r64 = _solve(spk, M, b)
    xm, rm = _solve(spk, M, b, precision=spk.PREC_MIXED)
    for x, r in ((x64, r64), (xm, rm)):
        assert r.reason == spk.CONVERGED_RTOL
        assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * bn * (1 + 1e-6)
    assert rm.inner_iterations <= 1.1 * r64.iterations
    assert np.linalg.norm(xm - x64) <= 1e-5 * np.linalg.norm(x64)


def test_c4_powerlaw_spmv_all_kernels():
    spk = need_gpu()
    import torch

    A = spkgen.powerlaw_spd(4_000_000, seed=0)
    M = mat_on_gpu(spk, A, flags=spk.MAT_MIXED)
    assert spk.KERNEL_NAMES[M.info.kernel] == "sliced"
    assert M.info.lanes == 2048  # skewed rows: merge path over the slices
    assert M.info.row_max == A.row_lengths().max()
    x = spkgen.rhs_uniform(A.n, 0)
    ref = _Ref(A, x)
    _spmv_all(spk, M, A, ref)  # the selected kernel meets 1e-14
    x32 = x.astype(np.float32)
    Af = spkgen.CSR(A.n, A.rowptr, A.col, A.val.astype(np.float32).astype(np.float64))
    yo32 = oracle.spmv(Af, x32.astype(np.float64))
    sc32 = oracle.spmv_abs(Af, x32.astype(np.float64))

    def check_f32():  # per-row bound of the merge / sliced orders in FP32
        _spmv_f32_all(spk, M, A, x32, yo32, sc32, 30)

    check_f32()
    for k, p, tol in ((spk.KERNEL_MERGE, 0, 1e-14), (spk.KERNEL_VECTOR, 32, 1e-14),
                      (spk.KERNEL_VECTOR, 64, 1e-14), (spk.KERNEL_SLICED, 2, 1e-14),
                      (spk.KERNEL_SLICED, 4, 1e-14)):
        spk.mat_set_kernel(M, k, p)
        _spmv_all(spk, M, A, ref, tol)
    spk.mat_set_kernel(M, spk.KERNEL_MERGE, 0)
    check_f32()


def test_c5_served_requests_full_sizes():
    """The first 16 requests of the seed-0 stream at their real sizes."""
    spk = need_gpu()
    reqs = spkgen.serve_stream(seed=0, count=16)
    S = spk.server_create()
    o = spk.ksp_opts(precision=spk.PREC_MIXED)
    items = []
    for r in reqs:
        A = spkgen.serve_matrix(r)
        b = spkgen.rhs_uniform(A.n, r.rhs_seed % (2**31))
        items.append((A, b, spk.server_submit(S, A.rowptr, A.col, A.val, b, o)))
    done = {}
    for _ in range(100000):
        spk.server_progress(S, 4)
        for A, b, t in items:
            if t not in done:
                x = np.empty(A.n)
                got = spk.server_poll(S, t, x)
                if got is not None:
                    done[t] = (x, got[0])
        if len(done) == len(items):
            break
    assert len(done) == len(items)
    for A, b, t in items:
        x, res = done[t]
        assert res.reason == spk.CONVERGED_RTOL
        assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)
    S.close()


def test_c2_single_reduction_chebyshev_and_multi():
    """The bench's extra C2 legs at full size: the single-reduction solve
    against its oracle, the 8-step Chebyshev smoother against its oracle,
    and 8 right-hand sides sharing each SpMM (oracle true residual of every
    column; column 0 is the bench's right-hand side, 446 oracle iterations)."""
    spk = need_gpu()
    import torch

    A = spkgen.laplace3d7(128)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    bn = oracle.nrm2(b)
    # single reduction
    xs, rs = _solve(spk, M, b, single_reduction=1)
    xo, ro, _ = oracle.pcg(A, b, single_reduction=True)
    assert rs.reason == spk.CONVERGED_RTOL
    assert abs(rs.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    assert oracle.nrm2(b - oracle.spmv(A, xs)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(xs - xo) <= 1e-5 * np.linalg.norm(xo)
    # Chebyshev, default interval [g/10, g]
    g = oracle.gershgorin(A)
    assert M.info.gershgorin == pytest.approx(g, rel=1e-14)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.pc_chebyshev(M, to_dev(b), x, 8)
    xc, _ = oracle.chebyshev(A, b, 8, g / 10, g)
    assert np.max(np.abs(x.cpu().numpy() - xc)) <= 1e-11 * np.max(np.abs(xc))
    # 8 right-hand sides
    k = 8
    B = np.stack([spkgen.rhs_uniform(A.n, s) for s in range(k)], axis=1)
    X = torch.zeros((A.n, k), dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_multi(M, torch.from_numpy(B).cuda(), X)
    X = X.cpu().numpy()
    # column 0 is the right-hand side of the textbook oracle solve above the
    # single-reduction one: its count is pinned (446, SciPy agrees)
    _, r0, _ = oracle.pcg(A, b)
    assert abs(res[0].iterations - r0["iterations"]) <= max(2, 0.01 * r0["iterations"])
    for j in range(k):
        bj = B[:, j].copy()
        assert res[j].reason == spk.CONVERGED_RTOL
        assert oracle.nrm2(bj - oracle.spmv(A, X[:, j].copy())) <= 1e-8 * oracle.nrm2(bj) * (1 + 1e-6)


def test_c2_multigrid_pcg():
    """The bench's multigrid leg at full size: every coarse level bit-exact
    against the oracle's Galerkin products (integer Laplacian), one V-cycle
    against the oracle's cycle, and the V-cycle PCG solve (iterations within
    one of the oracle's, the oracle's true residual of the GPU solution)."""
    spk = need_gpu()
    import torch

    A = spkgen.laplace3d7(128)
    M = mat_on_gpu(spk, A)
    G = spk.mg_create(M, (128, 128, 128))
    h = oracle.mg_setup(A, (128, 128, 128))
    assert [G.info.n[l] for l in range(G.levels)] == [m.n for m in h.mats] == [128**3, 64**3, 32**3, 16**3, 8**3]
    for l in range(1, G.levels):
        rp, ci, va = spk.mg_copy_level(G, l)
        assert np.array_equal(rp, h.mats[l].rowptr) and np.array_equal(ci, h.mats[l].col)
        assert np.array_equal(va, h.mats[l].val)
    b = spkgen.rhs_uniform(A.n, 0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.mg_apply(G, to_dev(b), x)
    xc = oracle.mg_cycle(h, b)
    assert np.max(np.abs(x.cpu().numpy() - xc)) <= 1e-11 * np.max(np.abs(xc))
    x.zero_()
    res = spk.ksp_solve_mg(G, to_dev(b), x, spk.ksp_opts(graph_k=1))
    xo, ro, _ = oracle.pcg_mg(A, h, b)
    assert res.reason == spk.CONVERGED_RTOL and abs(res.iterations - ro["iterations"]) <= 1
    xg = x.cpu().numpy()
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, xg)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_c2_multigrid_fp32_cycle():
    """The bench's FP32-cycle leg: V-cycle PCG with the cycle in FP32 inside
    FP64 CG on the 128^3 Laplacian; iterations within two of the oracle's
    FP64-cycle solve (14), the oracle's true residual of the solution."""
    spk = need_gpu()
    import torch

    A = spkgen.laplace3d7(128)
    M = mat_on_gpu(spk, A)
    G = spk.mg_create(M, (128, 128, 128), spk.mg_opts(precision=spk.PREC_MIXED))
    h = oracle.mg_setup(A, (128, 128, 128))
    b = spkgen.rhs_uniform(A.n, 0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.mg_apply(G, to_dev(b), x)
    xc = oracle.mg_cycle(h, b)
    assert np.max(np.abs(x.cpu().numpy() - xc)) <= 1e-4 * np.max(np.abs(xc))
    x.zero_()
    res = spk.ksp_solve_mg(G, to_dev(b), x, spk.ksp_opts(graph_k=1))
    _, ro, _ = oracle.pcg_mg(A, h, b)
    assert res.reason == spk.CONVERGED_RTOL
    assert ro["iterations"] - 1 <= res.iterations <= ro["iterations"] + 2
    assert oracle.nrm2(b - oracle.spmv(A, x.cpu().numpy())) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)


def test_c3_multigrid_pcg():
    """Multigrid on the 27-point lognormal 160^3 system: the first coarse
    level against the oracle's Galerkin product (within 1e-14 of the summed
    |terms|), one V-cycle against the oracle's cycle, and the FP64- and
    FP32-cycle solves through the oracle's true residual."""
    spk = need_gpu()
    import torch

    A = spkgen.diffusion3d27_lognormal(160, seed=0)
    M = mat_on_gpu(spk, A)
    G = spk.mg_create(M, (160, 160, 160))
    assert [G.info.n[l] for l in range(G.levels)] == [160**3, 80**3, 40**3, 20**3, 10**3]
    A1 = oracle.galerkin(A, (160, 160, 160))
    rp, ci, va = spk.mg_copy_level(G, 1)
    assert np.array_equal(rp, A1.rowptr) and np.array_equal(ci, A1.col)
    scale = oracle.galerkin(spkgen.CSR(A.n, A.rowptr, A.col, np.abs(A.val)), (160, 160, 160)).val
    assert np.all(np.abs(va - A1.val) <= 1e-14 * scale)
    h = oracle.mg_setup(A, (160, 160, 160))
    b = spkgen.rhs_uniform(A.n, 0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.mg_apply(G, to_dev(b), x)
    xc = oracle.mg_cycle(h, b)
    assert np.max(np.abs(x.cpu().numpy() - xc)) <= 1e-11 * np.max(np.abs(xc))
    bn = oracle.nrm2(b)
    for prec in (spk.PREC_FP64, spk.PREC_MIXED):
        Gp = G if prec == spk.PREC_FP64 else spk.mg_create(M, (160, 160, 160), spk.mg_opts(precision=prec))
        x.zero_()
        res = spk.ksp_solve_mg(Gp, to_dev(b), x, spk.ksp_opts(graph_k=1))
        assert res.reason == spk.CONVERGED_RTOL and res.iterations <= 30
        assert oracle.nrm2(b - oracle.spmv(A, x.cpu().numpy())) <= 1e-8 * bn * (1 + 1e-6)
