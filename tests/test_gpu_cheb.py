"""Chebyshev-Jacobi smoother parity: the HIP smoother against the oracle's
three-term recurrence on the same seeded inputs, every SpMV family, with and
without a starting guess and a residual output.  The recurrence has no inner
product, so rounding differences grow only through the few steps: the bound
is 1e-11 of the largest |x| (bit-exact where the arithmetic is exact)."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import mat_on_gpu, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _cases():
    yield "lap2d_61", spkgen.laplace2d5(61)
    yield "lap3d_23", spkgen.laplace3d7(23, 0.1)
    yield "diff27_13", spkgen.diffusion3d27_lognormal(13, seed=2)
    yield "powerlaw_20k", spkgen.powerlaw_spd(20000, seed=4)


def _run(spk, M, b, steps, emin, emax, x0=None, want_r=True):
    import torch

    x = to_dev(x0) if x0 is not None else torch.full((M.n,), np.nan, dtype=torch.float64, device="cuda")
    r = torch.full((M.n,), np.nan, dtype=torch.float64, device="cuda") if want_r else None
    spk.pc_chebyshev(M, to_dev(b), x, steps, emin, emax, r_out=r, x0_nonzero=x0 is not None)
    return x.cpu().numpy(), (r.cpu().numpy() if want_r else None)


def _close(a, ref, what):
    scale = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(a - ref))
    assert err <= 1e-11 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("case", ["lap2d_61", "lap3d_23", "diff27_13", "powerlaw_20k"])
@pytest.mark.parametrize("kernel", ["auto", "stream", "vector", "merge", "sell"])
def test_chebyshev_parity(case, kernel):
    spk = need_gpu()
    A = dict(_cases())[case]
    M = mat_on_gpu(spk, A)
    if kernel != "auto":
        k = {"stream": spk.KERNEL_STREAM, "vector": spk.KERNEL_VECTOR, "merge": spk.KERNEL_MERGE,
             "sell": spk.KERNEL_SELL}[kernel]
        spk.mat_set_kernel(M, k, 8 if kernel == "vector" else 0)
    g = oracle.gershgorin(A)
    assert M.info.gershgorin == pytest.approx(g, rel=1e-14)
    b = spkgen.rhs_uniform(A.n, 3)
    x0 = spkgen.rhs_uniform(A.n, 4)
    for steps in (0, 1, 2, 5):
        for start in (None, x0):
            xo, ro = oracle.chebyshev(A, b, steps, 0.1 * g, g, x0=start)
            x, r = _run(spk, M, b, steps, 0.0, 0.0, x0=start)  # defaults: [g/10, g]
            _close(x, xo, f"{case}/{kernel} steps {steps} x")
            _close(r, ro, f"{case}/{kernel} steps {steps} r")
            x2, _ = _run(spk, M, b, steps, 0.1 * g, g, x0=start, want_r=False)
            _close(x2, xo, f"{case}/{kernel} steps {steps} x (no residual)")
    M.close()


def test_chebyshev_explicit_interval_and_exact_start():
    spk = need_gpu()
    A = spkgen.laplace3d7(20)
    M = mat_on_gpu(spk, A)
    b = spkgen.rhs_uniform(A.n, 0)
    xo, ro = oracle.chebyshev(A, b, 6, 0.05, 1.95)
    x, r = _run(spk, M, b, 6, 0.05, 1.95)
    _close(x, xo, "explicit interval")
    _close(r, ro, "explicit interval r")
    # exact integer start: r = 0 exactly and x never moves
    xs = np.random.default_rng(1).integers(-50, 50, A.n).astype(np.float64)
    bi = oracle.spmv(A, xs)
    x, r = _run(spk, M, bi, 4, 0.2, 2.0, x0=xs)
    assert np.array_equal(x, xs) and not r.any()


def test_chebyshev_errors():
    spk = need_gpu()
    import torch

    A = spkgen.laplace2d5(8)
    M = mat_on_gpu(spk, A)
    b = to_dev(np.ones(A.n))
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    for steps, emin, emax in ((-1, 0.1, 1.0), (2, 1.0, 1.0), (2, 2.0, 1.0)):
        with pytest.raises(spk.SpkError) as e:
            spk.pc_chebyshev(M, b, x, steps, emin, emax)
        assert e.value.status == spk.EINVAL
    with pytest.raises(spk.SpkError):
        spk.pc_chebyshev(M, x, x, 2)  # b overlaps x
    Z = spkgen.CSR(3, np.array([0, 1, 1, 2], np.int32), np.array([0, 2], np.int32), np.array([1.0, 1.0]))
    MZ = mat_on_gpu(spk, Z)
    assert MZ.info.gershgorin == 0.0
    with pytest.raises(spk.SpkError) as e:
        spk.pc_chebyshev(MZ, to_dev(np.ones(3)), torch.zeros(3, dtype=torch.float64, device="cuda"), 2)
    assert e.value.status == spk.EZERODIAG
    E = spkgen.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    ME = mat_on_gpu(spk, E)
    e0 = torch.zeros(0, dtype=torch.float64, device="cuda")
    spk.pc_chebyshev(ME, e0, e0.clone(), 3, 0.1, 1.0)


def test_chebyshev_smooths_high_frequencies():
    """Smoother property on the GPU result: with [g/10, g] an oscillatory
    error mode (eigenvalue inside the interval) shrinks by at least
    1/T_k(sigma) while the smoothest mode barely moves."""
    spk = need_gpu()
    N = 48
    A = spkgen.laplace2d5(N)
    M = mat_on_gpu(spk, A)
    j = np.arange(1, N + 1)
    smooth = np.kron(np.sin(np.pi * j / (N + 1)), np.sin(np.pi * j / (N + 1)))
    rough = np.kron(np.sin(np.pi * j * N / (N + 1)), np.sin(np.pi * j * (N - 3) / (N + 1)))
    sigma = 1.1 / 0.9  # theta / delta for [0.2, 2]
    y = sigma
    bound = 1.0 / (8 * y**4 - 8 * y**2 + 1)  # 1 / T_4(sigma)
    for e0, shrinks in ((rough, True), (smooth, False)):
        b = oracle.spmv(A, e0)
        x, _ = _run(spk, M, b, 4, 0.0, 0.0)
        red = np.linalg.norm(e0 - x) / np.linalg.norm(e0)
        assert (red <= bound * (1 + 1e-9)) if shrinks else (red > 0.9), (red, bound)
