"""Multigrid parity: the HIP hierarchy, cycle and MG-preconditioned CG
against the oracle's on the same seeded inputs.

Bounds: the Galerkin products are bit-exact on the integer Laplacians and
within 1e-14 of the per-entry sum of |terms| otherwise (a sequential double
sum of at most 216 terms per coarse entry); the cycle is a fixed linear map
whose rounding differences pass through a few SpMVs and the coarsest inverse
(condition number below 1e3 here), so 1e-11 of the largest |x| bounds them;
CG with the cycle follows the Jacobi solve's contract (iterations within one,
the oracle's true residual of the GPU solution at most 1e-8, the first eight
residual norms within 1e-10 relative: later ones drift apart by the rounding
CG amplifies, up to 1e-8 relative after 20 iterations on the 1D grid)."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import mat_on_gpu, need_gpu, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (matrix, grid shape, coarse_max)
    "lap2d_64": (lambda: spkgen.laplace2d5(64), (64, 64), 300),
    "lap2d_45x37": (lambda: spkgen.laplace_grid((45, 37), 0.25), (45, 37), 64),
    "lap3d_24": (lambda: spkgen.laplace3d7(24), (24, 24, 24), 100),
    "lap3d_13x9x11": (lambda: spkgen.laplace_grid((13, 9, 11)), (13, 9, 11), 30),
    "diff27_15": (lambda: spkgen.diffusion3d27_lognormal(15, seed=3), (15, 15, 15), 64),
    "line_1000": (lambda: spkgen.laplace_grid((1000,)), (1000,), 20),
}


def _hier(spk, case, kernel="auto", **kw):
    make, shape, cmax = CASES[case]
    A = make()
    M = mat_on_gpu(spk, A)
    if kernel != "auto":
        k = {"stream": spk.KERNEL_STREAM, "vector": spk.KERNEL_VECTOR, "merge": spk.KERNEL_MERGE,
             "sell": spk.KERNEL_SELL}[kernel]
        spk.mat_set_kernel(M, k, 8 if kernel == "vector" else 0)
    opts = spk.mg_opts(coarse_max=cmax, **kw)
    G = spk.mg_create(M, shape, opts)
    okw = dict(kw)
    okw.pop("precision", None)  # the oracle is FP64
    if "smooth_steps" in okw:
        okw["steps"] = okw.pop("smooth_steps")
    h = oracle.mg_setup(A, shape, coarse_max=cmax, **okw)
    return A, M, G, h


def _close(a, ref, tol, what):
    scale = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(a - ref))
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("case", list(CASES))
def test_hierarchy_matches_oracle(case):
    spk = need_gpu()
    A, M, G, h = _hier(spk, case)
    assert G.levels == h.levels >= 3
    exact = "diff27" not in case
    for l in range(G.levels):
        assert tuple(G.info.shape[l])[: len(h.shapes[l])] == h.shapes[l]
        assert G.info.n[l] == h.mats[l].n and G.info.nnz[l] == h.mats[l].nnz
        rp, ci, va = spk.mg_copy_level(G, l)
        Ao = h.mats[l]
        assert np.array_equal(rp, Ao.rowptr) and np.array_equal(ci, Ao.col)
        if exact or l == 0:
            assert np.array_equal(va, Ao.val), f"level {l}"
        else:
            prev = h.mats[l - 1]
            scale = oracle.galerkin(spkgen.CSR(prev.n, prev.rowptr, prev.col, np.abs(prev.val)),
                                    h.shapes[l - 1]).val
            assert np.all(np.abs(va - Ao.val) <= 1e-14 * scale), f"level {l}"
        if l < G.levels - 1:
            assert G.info.emax[l] == pytest.approx(oracle.gershgorin(Ao), rel=1e-14)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("steps,omega,cycle", [(2, 2.0, 1), (1, 1.0, 1), (3, 1.5, 2), (0, 1.0, 1)])
def test_cycle_matches_oracle(case, steps, omega, cycle):
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, case, smooth_steps=steps, omega=omega, cycle=cycle)
    for seed in (0, 1):
        b = spkgen.rhs_uniform(A.n, seed)
        x = torch.full((A.n,), np.nan, dtype=torch.float64, device="cuda")
        spk.mg_apply(G, to_dev(b), x)
        _close(x.cpu().numpy(), oracle.mg_cycle(h, b), 1e-11, f"{case} seed {seed}")


@pytest.mark.parametrize("kernel", ["stream", "vector", "merge", "sell"])
def test_cycle_every_fine_family(kernel):
    """The fine level's SpMV family (the coarse levels choose their own)."""
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, "lap3d_24", kernel=kernel)
    assert spk.KERNEL_NAMES[G.info.kernel[0]] == kernel
    b = spkgen.rhs_uniform(A.n, 5)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.mg_apply(G, to_dev(b), x)
    _close(x.cpu().numpy(), oracle.mg_cycle(h, b), 1e-11, kernel)
    xs = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_mg(G, to_dev(b), xs)
    _, ro, _ = oracle.pcg_mg(A, h, b)
    assert res.reason == spk.CONVERGED_RTOL and abs(res.iterations - ro["iterations"]) <= 1


@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_13x9x11", "diff27_15", "line_1000"])
@pytest.mark.parametrize("cycle", [1, 2])
def test_pcg_mg_matches_oracle(case, cycle):
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, case, cycle=cycle)
    b = spkgen.rhs_uniform(A.n, 2)
    hist = np.full(64, np.nan)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_mg(G, to_dev(b), x, hist=hist)
    xo, ro, ho = oracle.pcg_mg(A, h, b, hist_len=64)
    assert res.reason == spk.CONVERGED_RTOL
    assert abs(res.iterations - ro["iterations"]) <= 1
    k = min(res.iterations, ro["iterations"], 8) + 1
    assert np.all(np.abs(hist[:k] - ho[:k]) <= 1e-10 * ho[:k])
    xg = x.cpu().numpy()
    bn = oracle.nrm2(b)
    assert oracle.nrm2(b - oracle.spmv(A, xg)) <= 1e-8 * bn * (1 + 1e-6)
    assert res.true_rel_residual == pytest.approx(oracle.nrm2(b - oracle.spmv(A, xg)) / bn, rel=1e-6)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_pcg_mg_graph_depths_and_determinism():
    """Graphs of 1 or 4 iterations and direct launches run the same kernels:
    identical bits; a repeated solve too."""
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, "lap3d_24")
    b = to_dev(spkgen.rhs_uniform(A.n, 7))
    out = []
    for gk in (0, 1, 4, 4):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = spk.ksp_solve_mg(G, b, x, spk.ksp_opts(graph_k=gk))
        out.append((res.iterations, x.cpu().numpy()))
    for it, xv in out[1:]:
        assert it == out[0][0] and np.array_equal(xv, out[0][1])


def test_pcg_mg_reasons_and_starts():
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, "lap2d_45x37")
    b = spkgen.rhs_uniform(A.n, 0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_mg(G, to_dev(b), x, spk.ksp_opts(maxit=2))
    assert res.reason == spk.DIVERGED_ITS and res.iterations == 2
    _, ro, _ = oracle.pcg_mg(A, h, b, maxit=2)
    assert res.true_rel_residual == pytest.approx(ro["true_rel_residual"], rel=1e-8)
    # b = 0 returns x = 0 even from a nonzero start
    x = to_dev(spkgen.rhs_uniform(A.n, 1))
    res = spk.ksp_solve_mg(G, to_dev(np.zeros(A.n)), x, spk.ksp_opts(x0_nonzero=1))
    assert res.reason == spk.CONVERGED_ATOL and res.iterations == 0 and not x.cpu().numpy().any()
    # starting from an exact integer solution: no iteration
    xs = np.random.default_rng(0).integers(-9, 9, A.n).astype(np.float64)
    bs = oracle.spmv(spkgen.laplace_grid((45, 37)), xs)
    x = to_dev(xs)
    Ai = spkgen.laplace_grid((45, 37))
    Mi = mat_on_gpu(spk, Ai)
    Gi = spk.mg_create(Mi, (45, 37), spk.mg_opts(coarse_max=64))
    res = spk.ksp_solve_mg(Gi, to_dev(bs), x, spk.ksp_opts(x0_nonzero=1))
    assert res.reason == spk.CONVERGED_RTOL and res.iterations == 0
    assert np.array_equal(x.cpu().numpy(), xs)
    # a nonzero start converges to the same tolerance as the oracle's
    x0 = spkgen.rhs_uniform(A.n, 9)
    x = to_dev(x0)
    res = spk.ksp_solve_mg(G, to_dev(b), x, spk.ksp_opts(x0_nonzero=1))
    _, ro, _ = oracle.pcg_mg(A, h, b, x0=x0)
    assert res.reason == spk.CONVERGED_RTOL and abs(res.iterations - ro["iterations"]) <= 1
    # a NaN in b
    bn = b.copy()
    bn[17] = np.nan
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_mg(G, to_dev(bn), x)
    assert res.reason == spk.DIVERGED_NANORINF
    with pytest.raises(spk.SpkError):
        spk.ksp_solve_mg(G, to_dev(b), x, spk.ksp_opts(precision=spk.PREC_MIXED))


def test_mg_create_rejects():
    spk = need_gpu()
    A = spkgen.laplace2d5(20)
    M = mat_on_gpu(spk, A)
    with pytest.raises(spk.SpkError, match="grid"):
        spk.mg_create(M, (20, 21))
    # a 2D matrix read as 1D: couplings 20 rows apart
    with pytest.raises(spk.SpkError, match="stencil"):
        spk.mg_create(M, (400,))
    M70 = mat_on_gpu(spk, spkgen.laplace2d5(70))  # 4900 rows: above the dense limit
    with pytest.raises(spk.SpkError, match="coarsest"):
        spk.mg_create(M70, (70, 70), spk.mg_opts(max_levels=1, coarse_max=100))
    G1 = spk.mg_create(M, (20, 20), spk.mg_opts(max_levels=1, coarse_max=100))
    assert G1.levels == 1  # 400 rows: one directly solved level
    with pytest.raises(spk.SpkError, match="omega"):
        spk.mg_create(M, (20, 20), spk.mg_opts(omega=0.0))
    # symmetric indefinite (negated diagonal): the coarsest inverse has no positive pivot
    D = spkgen.to_dense(A)
    D[np.diag_indices(A.n)] *= -1
    Mi = mat_on_gpu(spk, spkgen.dense_to_csr(D))
    with pytest.raises(spk.SpkError, match="positive definite"):
        spk.mg_create(Mi, (20, 20), spk.mg_opts(coarse_max=400))


def test_mg_profile_levels():
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, "lap3d_24")
    b = to_dev(spkgen.rhs_uniform(A.n, 0))
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ms = spk.mg_profile(G, b, x, reps=3)
    assert len(ms) == G.levels and all(t > 0 for t in ms)
    _close(x.cpu().numpy(), oracle.mg_cycle(h, b.cpu().numpy()), 1e-11, "profiled cycle")


# ---------------------------------------------------------------- FP32 cycle inside FP64 CG
# The FP32 cycle is the FP64 cycle's arithmetic in single precision: each
# step is backward stable with u32 = 6e-8 per operation, and the result's
# error relative to the FP64 cycle is that rounding amplified by at most the
# coarsest matrix's condition number (below 1e3 here), hence 1e-4 of the
# largest |x|.  CG stays FP64: the FP32 preconditioner may cost an iteration
# or two, and the oracle's true residual of the solution is still 1e-8.

@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_13x9x11", "diff27_15", "line_1000"])
@pytest.mark.parametrize("cycle", [1, 2])
def test_fp32_cycle_and_solve(case, cycle):
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, case, cycle=cycle, precision=spk.PREC_MIXED)
    for seed in (0, 1):
        b = spkgen.rhs_uniform(A.n, seed)
        x = torch.full((A.n,), np.nan, dtype=torch.float64, device="cuda")
        spk.mg_apply(G, to_dev(b), x)
        _close(x.cpu().numpy(), oracle.mg_cycle(h, b), 1e-4, f"fp32 {case} seed {seed}")
    b = spkgen.rhs_uniform(A.n, 2)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = spk.ksp_solve_mg(G, to_dev(b), x)
    _, ro, _ = oracle.pcg_mg(A, h, b)
    assert res.reason == spk.CONVERGED_RTOL
    assert ro["iterations"] - 1 <= res.iterations <= ro["iterations"] + 2
    xg = x.cpu().numpy()
    assert oracle.nrm2(b - oracle.spmv(A, xg)) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)


@pytest.mark.parametrize("kernel", ["stream", "vector", "merge"])
def test_fp32_cycle_fine_families(kernel):
    spk = need_gpu()
    import torch

    A, M, G, h = _hier(spk, "lap3d_24", kernel=kernel, precision=spk.PREC_MIXED)
    b = spkgen.rhs_uniform(A.n, 5)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    spk.mg_apply(G, to_dev(b), x)
    _close(x.cpu().numpy(), oracle.mg_cycle(h, b), 1e-4, kernel)
