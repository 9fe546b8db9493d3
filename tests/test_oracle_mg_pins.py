"""Pins of the oracle's geometric multigrid (Sec. 5.3: Chebyshev-Jacobi
smoothing on every level but the coarsest, a direct coarsest solve, V- and
W-cycles) against results fixed independently of its code: the Galerkin
product of the Laplacian in closed form, SciPy's sparse triple product with a
prolongation built here from grid coordinates, and the cycle's error operator
assembled from dense matrices, with the smoother's error polynomial evaluated
on an eigendecomposition (not by the recurrence)."""

import numpy as np
import pytest

import oracle
import spkgen
from test_oracle_pins import cheb_P


def agg_P(shape):
    """Dense piecewise-constant prolongation for the 2 x 2 (x 2) aggregates
    of a grid (x fastest), built from coordinates."""
    dims = list(shape)
    cs = [(s + 1) // 2 for s in dims]
    coords = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]
    agg = np.zeros(coords.shape[1], dtype=np.int64)
    stride = 1
    for d in range(len(dims)):
        agg += (coords[d] // 2) * stride
        stride *= cs[d]
    P = np.zeros((coords.shape[1], stride))
    P[np.arange(coords.shape[1]), agg] = 1.0
    return P, tuple(cs)


def same_csr(a, b):
    return (a.n == b.n and np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.col, b.col)
            and np.array_equal(a.val, b.val))


def scaled(A, c, shift=0.0):
    v = A.val * c
    out = spkgen.CSR(A.n, A.rowptr.copy(), A.col.copy(), v)
    if shift:
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        out.val[rows == A.col] += shift
    return out


# ---------------------------------------------------------------- Galerkin product

@pytest.mark.parametrize("N", [4, 8, 16])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_galerkin_laplacian_closed_form(orc, N, shift):
    """Aggregating 2^d points of the unscaled Dirichlet Laplacian: each
    coarse off-diagonal collects 2^(d-1) fine couplings of -1, each coarse
    diagonal 2^d fine diagonals minus the 2 d 2^(d-1) internal couplings, so
    A_c = 2^(d-1) A(N/2) exactly, plus 2^d times the fine shift."""
    A2 = oracle.galerkin(spkgen.laplace2d5(N, shift), (N, N))
    assert same_csr(A2, scaled(spkgen.laplace2d5(N // 2), 2.0, 4 * shift))
    A3 = oracle.galerkin(spkgen.laplace3d7(N, shift), (N, N, N))
    assert same_csr(A3, scaled(spkgen.laplace3d7(N // 2), 4.0, 8 * shift))


@pytest.mark.parametrize("case", ["lap2d_7x5", "lap3d_5x3x4", "lognormal27_5", "lognormal27_7", "line_9"])
def test_galerkin_vs_scipy_triple_product(orc, case):
    """Ragged aggregates (odd extents), 27-point variable coefficients and a
    1D grid: the oracle's A_c equals SciPy's P^T A P (P from coordinates);
    the stored pattern is every coarse pair with a fine coupling."""
    import scipy.sparse as sp

    if case == "lap2d_7x5":
        shape = (7, 5)
        A = spkgen.laplace_grid(shape, 0.25)
    elif case == "lap3d_5x3x4":
        shape = (5, 3, 4)
        A = spkgen.laplace_grid(shape)
    elif case == "line_9":
        shape = (9,)
        A = spkgen.dense_to_csr(2 * np.eye(9) - np.eye(9, k=1) - np.eye(9, k=-1))
    else:
        N = int(case.split("_")[1])
        shape = (N, N, N)
        A = spkgen.diffusion3d27_lognormal(N, seed=1)
    Ac = oracle.galerkin(A, shape)
    P, cs = agg_P(shape)
    assert cs == oracle.coarse_shape(shape)
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    Ps = sp.csr_matrix(P)
    ref = (Ps.T @ S @ Ps).toarray()
    got = spkgen.to_dense(Ac)
    assert np.allclose(got, ref, rtol=1e-15, atol=1e-15 * np.abs(ref).max())
    pattern = (Ps.T @ abs(S) @ Ps).toarray() > 0
    rows = np.repeat(np.arange(Ac.n), np.diff(Ac.rowptr))
    mask = np.zeros_like(pattern)
    mask[rows, Ac.col] = True
    assert np.array_equal(mask, pattern)
    assert all(np.all(np.diff(Ac.col[Ac.rowptr[i]:Ac.rowptr[i + 1]]) > 0) for i in range(Ac.n))
    # aggregation keeps row sums: A_c 1 = P^T (A 1)
    assert np.allclose(got.sum(axis=1), P.T @ spkgen.to_dense(A).sum(axis=1), rtol=1e-14, atol=1e-12)


def test_restrict_prolong_definitions(orc):
    rng = np.random.default_rng(0)
    for shape in [(7, 5), (5, 3, 4), (8, 8, 8), (9,)]:
        P, cs = agg_P(shape)
        r = rng.integers(-50, 50, P.shape[0]).astype(np.float64)
        assert np.array_equal(oracle.restrict(shape, r), P.T @ r)
        xc = rng.integers(-50, 50, P.shape[1]).astype(np.float64)
        x = rng.integers(-50, 50, P.shape[0]).astype(np.float64)
        assert np.array_equal(oracle.prolong(shape, 0.5, xc, x), x + 0.5 * (P @ xc))


# ---------------------------------------------------------------- the cycle

def smoother_error(A, steps, emin_frac):
    """Error operator of `steps` Chebyshev-Jacobi steps on [f g, g] (g the
    Gershgorin bound of D^-1 A): P_k(D^-1 A) from the eigendecomposition of
    the symmetric D^-1/2 A D^-1/2."""
    d = np.diag(A)
    g = float(np.max(np.abs(A).sum(axis=1) / np.abs(d)))
    s = 1.0 / np.sqrt(d)
    lam, Q = np.linalg.eigh(A * s[:, None] * s[None, :])
    p = np.array([cheb_P(steps, t, emin_frac * g, g) for t in lam])
    return (s[:, None] * (Q * p) @ Q.T) / s[None, :]


def cycle_operator(mats, shapes, steps, emin_frac, omega, cycle):
    """B_0 with x = B_0 b for one cycle from zero, built top-down from
    E_l = S_l (I - omega P_l C_{l+1} P_l^T A_l) S_l, B_l = (I - E_l) A_l^-1;
    C is A^-1 on the coarsest level, B for a V-cycle, (I - E^2) A^-1 for a
    W-cycle (two cycles, the second from the first's result)."""
    L = len(mats)
    B = [None] * L
    E = [None] * L
    B[L - 1] = np.linalg.inv(mats[L - 1])
    for l in range(L - 2, -1, -1):
        A = mats[l]
        P, _ = agg_P(shapes[l])
        if l + 1 == L - 1:
            C = B[l + 1]
        elif cycle == 1:
            C = B[l + 1]
        else:
            C = (np.eye(len(mats[l + 1])) - E[l + 1] @ E[l + 1]) @ np.linalg.inv(mats[l + 1])
        S = smoother_error(A, steps, emin_frac)
        E[l] = S @ (np.eye(len(A)) - omega * P @ C @ P.T @ A) @ S
        B[l] = (np.eye(len(A)) - E[l]) @ np.linalg.inv(A)
    return B[0]


CASES = {
    "lap2d_12": (lambda: spkgen.laplace2d5(12), (12, 12), 9),
    "lap2d_11x7": (lambda: spkgen.laplace_grid((11, 7), 0.125), (11, 7), 4),
    "lap3d_6x5x4": (lambda: spkgen.laplace_grid((6, 5, 4)), (6, 5, 4), 4),
    "lognormal27_6": (lambda: spkgen.diffusion3d27_lognormal(6, seed=2), (6, 6, 6), 8),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("steps,omega,cycle", [(1, 1.0, 1), (2, 2.0, 1), (3, 1.5, 2), (2, 2.0, 2)])
def test_cycle_matches_dense_error_operator(orc, case, steps, omega, cycle):
    make, shape, coarse_max = CASES[case]
    A = make()
    h = oracle.mg_setup(A, shape, coarse_max=coarse_max, steps=steps, omega=omega, cycle=cycle)
    assert h.levels >= 3 and h.mats[-1].n <= coarse_max
    mats = [spkgen.to_dense(m) for m in h.mats]
    B0 = cycle_operator(mats, h.shapes, steps, 0.1, omega, cycle)
    for seed in range(2):
        b = spkgen.rhs_uniform(A.n, seed)
        x = oracle.mg_cycle(h, b)
        ref = B0 @ b
        assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
    # from a nonzero start the cycle is x0 + B_0 (b - A x0)
    x0 = spkgen.rhs_uniform(A.n, 7)
    x = oracle.mg_cycle(h, b, x0=x0)
    ref = x0 + B0 @ (b - mats[0] @ x0)
    assert np.max(np.abs(x - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("omega", [1.0, 2.0])
def test_v_cycle_is_symmetric_positive_definite(orc, omega):
    """B_0 = (A^-1 - S A^-1 S^T) + omega S P B_1 P^T S^T with |P_k| < 1 on
    the spectrum: symmetric positive definite for every omega > 0, so PCG
    may use it."""
    A = spkgen.diffusion3d27_lognormal(6, seed=3)
    h = oracle.mg_setup(A, (6, 6, 6), coarse_max=8, steps=2, omega=omega)
    B = np.stack([oracle.mg_cycle(h, e) for e in np.eye(A.n)], axis=1)
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_hierarchy_shapes_and_limits(orc):
    A = spkgen.laplace3d7(16)
    h = oracle.mg_setup(A, (16, 16, 16), coarse_max=100)
    assert h.shapes == [(16, 16, 16), (8, 8, 8), (4, 4, 4)] and h.mats[-1].n == 64
    h = oracle.mg_setup(A, (16, 16, 16), coarse_max=100, max_levels=2)
    assert h.levels == 2 and h.mats[-1].n == 512
    h = oracle.mg_setup(spkgen.laplace_grid((9,)), (9,), coarse_max=1)
    assert h.shapes == [(9,), (5,), (3,), (2,), (1,)]


# ---------------------------------------------------------------- multigrid PCG

def test_pcg_mg_single_level_is_a_direct_solve(orc):
    A = spkgen.laplace2d5(10)
    h = oracle.mg_setup(A, (10, 10), coarse_max=100)
    assert h.levels == 1
    b = spkgen.rhs_uniform(A.n, 0)
    x, res, _ = oracle.pcg_mg(A, h, b, rtol=1e-10)
    assert res["reason_str"] == "CONVERGED_RTOL" and res["iterations"] == 1
    assert np.allclose(x, np.linalg.solve(spkgen.to_dense(A), b), rtol=0, atol=1e-12)


@pytest.mark.parametrize("case,cycle", [("lap2d_12", 1), ("lognormal27_6", 1), ("lap3d_6x5x4", 2)])
def test_pcg_mg_vs_scipy_with_dense_preconditioner(orc, case, cycle):
    """The PCG loop with the cycle as preconditioner agrees with SciPy's CG
    given the dense B_0 of the closed form (iterations within 1, solution
    to the solve's accuracy)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    make, shape, coarse_max = CASES[case]
    A = make()
    h = oracle.mg_setup(A, shape, coarse_max=coarse_max, cycle=cycle)
    B0 = cycle_operator([spkgen.to_dense(m) for m in h.mats], h.shapes, 2, 0.1, 2.0, cycle)
    b = spkgen.rhs_uniform(A.n, 3)
    x, res, _ = oracle.pcg_mg(A, h, b, rtol=1e-10)
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    it = [0]

    def cb(_):
        it[0] += 1

    xs, info = sla.cg(S, b, rtol=1e-10, atol=0.0, M=sla.aslinearoperator(B0), callback=cb)
    assert info == 0 and res["reason_str"] == "CONVERGED_RTOL"
    assert abs(res["iterations"] - it[0]) <= 1
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_pcg_mg_c1_and_reasons(orc):
    """The 64^2 system: the cycle cuts the Jacobi-PCG count (193) to about
    a tenth; the stopping rules are those of the Jacobi solve."""
    A = spkgen.laplace2d5(64)
    h = oracle.mg_setup(A, (64, 64), coarse_max=300)
    assert [m.n for m in h.mats] == [4096, 1024, 256]
    b = spkgen.rhs_uniform(A.n, 0)
    x, res, hist = oracle.pcg_mg(A, h, b, hist_len=64)
    assert res["reason_str"] == "CONVERGED_RTOL" and res["iterations"] <= 20
    assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * oracle.nrm2(b)
    assert hist[0] == pytest.approx(oracle.nrm2(b), rel=1e-15)
    _, res, _ = oracle.pcg_mg(A, h, b, maxit=3)
    assert res["reason_str"] == "DIVERGED_ITS" and res["iterations"] == 3
    x, res, _ = oracle.pcg_mg(A, h, np.zeros(A.n))
    assert res["reason_str"] == "CONVERGED_ATOL" and not x.any()
