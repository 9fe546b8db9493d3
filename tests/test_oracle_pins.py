"""Pins for the CPU oracle: each check compares the oracle with something
other than itself -- exact integer / rational arithmetic, closed-form
eigenpairs of the Dirichlet Laplacians, brute-force dense solves, the finite
termination property of CG, and third-party library routines."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import spkgen


# ---------------------------------------------------------------- helpers

def lap_eigpair(N, dim, ks, shift=0.0):
    """Closed-form eigenpair of the unscaled Dirichlet Laplacian on N^dim
    interior points: v = prod_d sin(pi j_d k_d / (N+1)),
    lambda = sum_d (2 - 2 cos(pi k_d / (N+1))) + shift."""
    j = np.arange(1, N + 1)
    v = np.ones(1)
    lam = shift
    for d in range(dim):  # x fastest: kron(slowest, ..., fastest)
        k = ks[d]
        s = np.sin(np.pi * j * k / (N + 1))
        v = np.kron(s, v)
        lam += 2.0 - 2.0 * np.cos(np.pi * k / (N + 1))
    return v, lam


def lap_kappa(N, dim):
    lmin = dim * (2 - 2 * math.cos(math.pi / (N + 1)))
    lmax = dim * (2 - 2 * math.cos(math.pi * N / (N + 1)))
    return lmax / lmin


def random_int_csr(n, seed, density=0.3, lo=-9, hi=9):
    rng = np.random.default_rng(seed)
    D = rng.integers(lo, hi + 1, size=(n, n)) * (rng.random((n, n)) < density)
    D[np.arange(n), np.arange(n)] = rng.integers(1, 20, size=n)
    return spkgen.dense_to_csr(D.astype(np.float64)), D


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("seed", range(4))
def test_spmv_exact_on_integers(orc, seed):
    """Nonsymmetric integer matrix, integer x: the result is exact, so it must
    equal Python's exact integer arithmetic bit for bit (a dropped term, a
    wrong index or a transposed operand all change it)."""
    n = 37
    A, D = random_int_csr(n, seed)
    x = np.random.default_rng(100 + seed).integers(-1000, 1000, size=n).astype(np.float64)
    y = oracle.spmv(A, x)
    exact = [sum(int(D[i, j]) * int(x[j]) for j in range(n)) for i in range(n)]
    assert np.array_equal(y, np.array(exact, dtype=np.float64))
    assert not np.array_equal(y, D.T @ x)  # the test can tell A from A^T


def test_spmv_f32_exact_on_integers(orc):
    n = 41
    A, D = random_int_csr(n, 9)
    x = np.random.default_rng(5).integers(-2000, 2000, size=n).astype(np.float32)
    y = oracle.spmv_f32(A, x)
    exact = [sum(int(D[i, j]) * int(x[j]) for j in range(n)) for i in range(n)]
    assert y.dtype == np.float32
    assert np.array_equal(y, np.array(exact, dtype=np.float32))


def test_spmv_f32_rounded_once(orc):
    """Random FP32 data: the oracle equals the exact (fsum) sum of the exact
    float products, rounded to float32 (within one float32 ulp: fsum rounds to
    double first)."""
    A = spkgen.powerlaw_spd(3000, seed=4)
    x = np.random.default_rng(2).standard_normal(A.n).astype(np.float32)
    v32 = A.val.astype(np.float32)
    y = oracle.spmv_f32(A, x, val32=v32)
    for i in range(0, A.n, 37):
        ks = range(A.rowptr[i], A.rowptr[i + 1])
        ex = math.fsum(float(v32[k]) * float(x[A.col[k]]) for k in ks)
        assert abs(float(y[i]) - ex) <= np.spacing(np.float32(abs(ex))) * 1.0001


@pytest.mark.parametrize("seed", range(3))
def test_spmv_abs_exact_on_integers(orc, seed):
    """The tolerance scale sum_j |a_ij| |x_j| against Python's exact integer
    arithmetic on a nonsymmetric integer matrix and x of both signs.  The
    same data tells the absolute sum from |A x| (rows cancel), from
    |A|^T |x| (a transposed operand) and from sum_j |a_ij| (x dropped), so
    a scale that is inflated, deflated or taken over the wrong operand fails."""
    n = 37
    A, D = random_int_csr(n, seed)
    x = np.random.default_rng(200 + seed).integers(-1000, 1000, size=n).astype(np.float64)
    ya = oracle.spmv_abs(A, x)
    exact = [sum(abs(int(D[i, j])) * abs(int(x[j])) for j in range(n)) for i in range(n)]
    assert np.array_equal(ya, np.array(exact, dtype=np.float64))
    assert not np.array_equal(ya, np.abs(oracle.spmv(A, x)))
    assert not np.array_equal(ya, np.abs(D).T @ np.abs(x))
    assert not np.array_equal(ya, np.abs(D).sum(axis=1).astype(np.float64))


@pytest.mark.parametrize("case", ["powerlaw", "diff27"])
def test_spmv_abs_vs_dense_and_fsum(orc, case):
    """Real data: the oracle's scale equals numpy's dense |A| @ |x| within
    the error of an n-term sum of nonnegative terms ((n - 1) u relative, no
    cancellation is possible), and math.fsum's exactly rounded sum of the
    exact products within one ulp on sampled rows."""
    A = spkgen.powerlaw_spd(700, seed=3) if case == "powerlaw" else spkgen.diffusion3d27_lognormal(9, seed=2)
    x = spkgen.rhs_uniform(A.n, 7) * 1e3
    ya = oracle.spmv_abs(A, x)
    D = spkgen.to_dense(A)
    dense = np.abs(D) @ np.abs(x)
    assert np.all(np.abs(ya - dense) <= (A.n - 1) * 2.0 ** -53 * dense)
    for i in range(0, A.n, 13):
        ks = range(A.rowptr[i], A.rowptr[i + 1])
        ex = math.fsum(abs(float(A.val[k]) * float(x[A.col[k]])) for k in ks)
        assert abs(ya[i] - ex) <= np.spacing(ex)
    # a row sum of |a_ij x_j| is at least |(A x)_i| and equals it only without cancellation
    assert np.all(ya >= np.abs(oracle.spmv(A, x)))


@pytest.mark.parametrize("dim,N,ks", [(2, 64, (1, 1)), (2, 64, (7, 40)), (3, 12, (1, 2, 3)),
                                      (3, 16, (16, 1, 9))])
def test_spmv_closed_form_eigenpairs(orc, dim, N, ks):
    A = spkgen.laplace2d5(N, 0.25) if dim == 2 else spkgen.laplace3d7(N, 0.25)
    v, lam = lap_eigpair(N, dim, ks, shift=0.25)
    y = oracle.spmv(A, v)
    scale = oracle.spmv_abs(A, v)
    assert np.all(np.abs(y - lam * v) <= 1e-14 * scale + 1e-300)


def test_spmv_ones_gives_boundary_counts(orc):
    """A 1 for the unscaled Dirichlet Laplacian = number of neighbours that
    fall off the grid (an integer, exact)."""
    N = 9
    A = spkgen.laplace3d7(N)
    y = oracle.spmv(A, np.ones(A.n))
    idx = np.arange(A.n)
    c = [(idx // N ** d) % N for d in range(3)]
    missing = sum((cd == 0).astype(int) + (cd == N - 1).astype(int) for cd in c)
    assert np.array_equal(y, missing.astype(np.float64))


def test_spmv_scipy_crosscheck(orc):
    import scipy.sparse as sp

    A = spkgen.diffusion3d27_lognormal(7, seed=1)
    x = spkgen.rhs_uniform(A.n, 3)
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    y = oracle.spmv(A, x)
    assert np.all(np.abs(y - S @ x) <= 1e-14 * oracle.spmv_abs(A, x))


def test_spmv_rows_matches_full(orc):
    A = spkgen.powerlaw_spd(5000, seed=1)
    x = spkgen.rhs_uniform(A.n, 1)
    rows = np.array([0, 17, 4999, 2500, 17])
    y, ya = oracle.spmv_rows(A, x, rows)
    assert np.array_equal(y, oracle.spmv(A, x)[rows])
    assert np.array_equal(ya, oracle.spmv_abs(A, x)[rows])


def test_spmv_empty_rows(orc):
    D = np.zeros((6, 6))
    D[1, 2] = 3.0
    D[4, 0] = -2.0
    A = spkgen.dense_to_csr(D)
    y = oracle.spmv(A, np.arange(1.0, 7.0))
    assert np.array_equal(y, np.array([0, 9.0, 0, 0, -2.0, 0]))


# ---------------------------------------------------------------- vectors

def test_dot_nrm2_exact_integers(orc):
    rng = np.random.default_rng(0)
    x = rng.integers(-10**6, 10**6, size=5000)
    y = rng.integers(-10**6, 10**6, size=5000)
    assert oracle.dot(x.astype(float), y.astype(float)) == float(int(np.dot(x.astype(object), y.astype(object))))
    ss = int(np.dot(x.astype(object), x.astype(object)))
    assert oracle.nrm2(x.astype(float)) == pytest.approx(math.isqrt(ss), rel=1e-15, abs=1.0)


@pytest.mark.parametrize("dim,N", [(2, 31), (3, 10)])
def test_dot_closed_form_sine(orc, dim, N):
    """|v|^2 = ((N+1)/2)^dim for the sine eigenvector with all k_d = 1."""
    v, _ = lap_eigpair(N, dim, (1,) * dim)
    assert oracle.dot(v, v) == pytest.approx(((N + 1) / 2) ** dim, rel=1e-15)


def test_dot_fsum_crosscheck(orc):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(20001) * 10 ** rng.uniform(-5, 5, 20001)
    y = rng.standard_normal(20001)
    ex = math.fsum(float(a) * float(b) for a, b in zip(x, y))
    # products are rounded in fsum's input; allow their rounding
    tol = 2 ** -52 * float(np.sum(np.abs(x * y)))
    assert abs(oracle.dot(x, y) - ex) <= tol


def test_axpy_aypx_rounded_once(orc):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(200)
    y = rng.standard_normal(200)
    a = 0.7318237
    out1 = oracle.axpy(a, x, y)
    out2 = oracle.aypx(a, x, y)
    for i in range(200):
        ex1 = Fraction(a) * Fraction(x[i]) + Fraction(y[i])
        ex2 = Fraction(x[i]) + Fraction(a) * Fraction(y[i])
        assert out1[i] == float(ex1)  # float(Fraction) rounds correctly
        assert out2[i] == float(ex2)


def test_diag_inv_and_jacobi(orc):
    A = spkgen.diffusion3d27_lognormal(4, seed=2)
    dinv = oracle.diag_inv(A)
    D = spkgen.to_dense(A)
    for i in range(A.n):
        assert dinv[i] == float(Fraction(1) / Fraction(D[i, i]))
    r = spkgen.rhs_uniform(A.n, 0)
    assert np.array_equal(oracle.jacobi_apply(dinv, r), dinv * r)
    Z = spkgen.dense_to_csr(np.array([[1.0, 2.0], [2.0, 0.0]]))
    with pytest.raises(ValueError):
        oracle.diag_inv(Z)


def test_dense_cholesky_vs_numpy(orc):
    A = spkgen.random_spd_dense_csr(120, seed=5, density=0.2)
    D = spkgen.to_dense(A)
    b = spkgen.rhs_uniform(A.n, 1)
    x = oracle.dense_cholesky_solve(D, b)
    assert np.allclose(x, np.linalg.solve(D, b), rtol=1e-12, atol=1e-14)
    with pytest.raises(ValueError):
        oracle.dense_cholesky_solve(np.array([[1.0, 2.0], [2.0, 1.0]]), np.ones(2))


# ---------------------------------------------------------------- PCG

@pytest.mark.parametrize("dim,N,ks", [(2, 20, (3, 5)), (3, 8, (2, 1, 4))])
def test_pcg_eigenvector_rhs_one_iteration(orc, dim, N, ks):
    """b = eigenvector v with a constant diagonal: Jacobi-PCG is plain CG and
    finishes in exactly one iteration with x = v / lambda."""
    A = spkgen.laplace2d5(N) if dim == 2 else spkgen.laplace3d7(N)
    v, lam = lap_eigpair(N, dim, ks)
    x, res, hist = oracle.pcg(A, v, rtol=1e-12, hist_len=10)
    assert res["reason_str"] == "CONVERGED_RTOL"
    assert res["iterations"] == 1
    assert np.allclose(x, v / lam, rtol=1e-12, atol=1e-13 * np.abs(v).max() / lam)


@pytest.mark.parametrize("m", [2, 3, 4, 6])
def test_pcg_finite_termination(orc, m):
    """b = sum of m eigenvectors with distinct eigenvalues: CG converges in at
    most m iterations (Krylov space of dimension m)."""
    N = 24
    A = spkgen.laplace2d5(N)
    ks = [(1, 1), (2, 3), (5, 5), (7, 2), (11, 13), (20, 4)][:m]
    b = np.zeros(A.n)
    lams = []
    for k in ks:
        v, lam = lap_eigpair(N, 2, k)
        b += v
        lams.append(lam)
    assert len(set(np.round(lams, 12))) == m
    x, res, hist = oracle.pcg(A, b, rtol=1e-9, hist_len=20)
    # the residual collapses to rounding level at step m, not before
    assert res["reason"] > 0 and res["iterations"] == m
    assert hist[m] / hist[0] < 1e-9 and hist[m - 1] / hist[0] > 1e-3
    xs = sum(lap_eigpair(N, 2, k)[0] / lam for k, lam in zip(ks, lams))
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_pcg_exact_rational_iterates(orc):
    """Jacobi-PCG carried out in exact rational arithmetic on a tiny SPD
    system (brute force): the oracle's residual history and iterates after
    k = 1..n steps agree with it to rounding level."""
    D = np.array([[4, -1, 0, -2, 0], [-1, 5, -1, 0, 1], [0, -1, 3, -1, 0],
                  [-2, 0, -1, 6, -1], [0, 1, 0, -1, 2]], dtype=np.float64)
    n = D.shape[0]
    b = np.array([1.0, -2.0, 0.5, 3.0, -1.0])
    A = spkgen.dense_to_csr(D)
    F = [[Fraction(int(D[i, j])) for j in range(n)] for i in range(n)]
    fb = [Fraction(v) for v in b]
    x = [Fraction(0)] * n
    r = fb[:]
    z = [r[i] / F[i][i] for i in range(n)]
    p = z[:]
    rho = sum(r[i] * z[i] for i in range(n))
    ex_hist = [math.sqrt(sum(float(v) ** 2 for v in r))]
    ex_x = []
    for _ in range(n):
        q = [sum(F[i][j] * p[j] for j in range(n)) for i in range(n)]
        eta = sum(p[i] * q[i] for i in range(n))
        alpha = rho / eta
        x = [x[i] + alpha * p[i] for i in range(n)]
        r = [r[i] - alpha * q[i] for i in range(n)]
        ex_hist.append(math.sqrt(float(sum(v * v for v in r))))
        ex_x.append([float(v) for v in x])
        if all(v == 0 for v in r):
            break
        z = [r[i] / F[i][i] for i in range(n)]
        rho_new = sum(r[i] * z[i] for i in range(n))
        p = [z[i] + (rho_new / rho) * p[i] for i in range(n)]
        rho = rho_new
    _, res, hist = oracle.pcg(A, b, rtol=1e-14, hist_len=20)
    assert res["iterations"] <= n
    k = min(len(hist), len(ex_hist)) - 1
    assert np.allclose(hist[:k], ex_hist[:k], rtol=1e-10)
    for kk in range(1, len(ex_x) + 1):
        xk, rk, _ = oracle.pcg(A, b, rtol=0.0, maxit=kk)
        if rk["reason_str"] != "DIVERGED_ITS":
            break
        assert np.allclose(xk, ex_x[kk - 1], rtol=1e-10, atol=1e-12)


def test_pcg_manufactured_solution_c1(orc):
    """Integer x*, b = A x* exact: the error obeys the condition-number bound
    ||x - x*|| / ||x*|| <= kappa ||r|| / ||b||, kappa in closed form."""
    N = 64
    A = spkgen.laplace2d5(N)
    xs = np.random.default_rng(0).integers(-5, 6, size=A.n).astype(np.float64)
    b = oracle.spmv(A, xs)
    assert np.array_equal(b, np.rint(b))
    x, res, _ = oracle.pcg(A, b, rtol=1e-8)
    kappa = lap_kappa(N, 2)
    assert kappa == pytest.approx(1711.66, abs=0.01)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err <= kappa * res["true_rel_residual"] * 1.0001
    assert res["true_rel_residual"] <= 1e-8


@pytest.mark.parametrize("case", ["lap2d_8", "lap2d_16", "lap3d_4", "lap3d_8", "rand_200", "rand_500"])
def test_pcg_vs_dense_solves(orc, case):
    if case.startswith("lap2d"):
        A = spkgen.laplace2d5(int(case.split("_")[1]))
    elif case.startswith("lap3d"):
        A = spkgen.laplace3d7(int(case.split("_")[1]))
    else:
        A = spkgen.random_spd_dense_csr(int(case.split("_")[1]), seed=1, density=0.05)
    D = spkgen.to_dense(A)
    b = spkgen.rhs_uniform(A.n, 4)
    x, res, _ = oracle.pcg(A, b, rtol=1e-8)
    assert res["reason"] > 0
    x_chol = oracle.dense_cholesky_solve(D, b)
    x_np = np.linalg.solve(D, b)
    ev = np.linalg.eigvalsh(D)
    kappa = ev[-1] / ev[0]
    assert np.linalg.norm(x_chol - x_np) <= 1e-12 * np.linalg.norm(x_np) * kappa
    assert np.linalg.norm(x - x_np) <= kappa * 1e-8 * np.linalg.norm(x_np)


def test_pcg_a_norm_error_monotone(orc):
    """||x* - x_k||_A is non-increasing in k (the CG minimisation property);
    a wrong sign in alpha or beta breaks it."""
    A = spkgen.diffusion3d27_lognormal(5, seed=0)
    D = spkgen.to_dense(A)
    b = spkgen.rhs_uniform(A.n, 2)
    xs = np.linalg.solve(D, b)
    errs = []
    for k in range(0, 25):
        xk, _, _ = oracle.pcg(A, b, rtol=0.0, maxit=k)
        e = xs - xk
        errs.append(math.sqrt(e @ D @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-3 * errs[0]


def test_pcg_iteration_count_vs_scipy_c1(orc):
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    A = spkgen.laplace2d5(64)
    for seed in range(3):
        b = spkgen.rhs_uniform(A.n, seed)
        _, res, _ = oracle.pcg(A, b, rtol=1e-8)
        S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
        it = [0]

        def cb(_):
            it[0] += 1

        sla.cg(S, b, rtol=1e-8, atol=0.0, M=sp.diags(1.0 / S.diagonal()), callback=cb, maxiter=10000)
        assert abs(res["iterations"] - it[0]) <= 2
    b = spkgen.rhs_uniform(A.n, 0)
    _, res, _ = oracle.pcg(A, b, rtol=1e-8)
    assert res["iterations"] == 193


def test_pcg_iteration_count_vs_scipy_c2(orc):
    """3D 7-point 128^3 with the rhs of seed 0 (the configuration the bench
    solves): the oracle takes 446 iterations, and SciPy's Jacobi-preconditioned
    CG with the same stopping rule (rtol 1e-8 on the unpreconditioned
    residual, atol 0) agrees within 2."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    A = spkgen.laplace3d7(128)
    b = spkgen.rhs_uniform(A.n, 0)
    _, res, _ = oracle.pcg(A, b, rtol=1e-8)
    assert res["reason_str"] == "CONVERGED_RTOL" and res["iterations"] == 446
    assert res["true_rel_residual"] <= 1e-8
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    it = [0]

    def cb(_):
        it[0] += 1

    _, info = sla.cg(S, b, rtol=1e-8, atol=0.0, M=sp.diags(1.0 / S.diagonal()), callback=cb, maxiter=10000)
    assert info == 0 and abs(res["iterations"] - it[0]) <= 2


def test_pcg_manufactured_solution_c2(orc):
    """128^3 7-point, integer x*, b = A x* exact: the error obeys
    ||x - x*|| / ||x*|| <= kappa ||b - A x|| / ||b|| with the closed-form
    condition number of the 3D Dirichlet Laplacian (6743.68)."""
    N = 128
    A = spkgen.laplace3d7(N)
    xs = np.random.default_rng(1).integers(-5, 6, size=A.n).astype(np.float64)
    b = oracle.spmv(A, xs)
    assert np.array_equal(b, np.rint(b))
    x, res, _ = oracle.pcg(A, b, rtol=1e-8)
    kappa = lap_kappa(N, 3)
    assert kappa == pytest.approx(6743.68, abs=0.01)
    assert res["reason_str"] == "CONVERGED_RTOL" and res["true_rel_residual"] <= 1e-8
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err <= kappa * res["true_rel_residual"] * 1.0001


def test_pcg_variable_diagonal_vs_scipy(orc):
    """Non-constant diagonal (Jacobi really acts): solution and iteration
    count agree with SciPy's preconditioned CG."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    A = spkgen.diffusion3d27_lognormal(12, seed=0)
    b = spkgen.rhs_uniform(A.n, 0)
    x, res, _ = oracle.pcg(A, b, rtol=1e-8)
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    it = [0]

    def cb(_):
        it[0] += 1

    xs, info = sla.cg(S, b, rtol=1e-8, atol=0.0, M=sp.diags(1.0 / S.diagonal()), callback=cb)
    assert info == 0 and abs(res["iterations"] - it[0]) <= 2
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


# ---------------------------------------------------------------- PCG failure modes

def test_pcg_reasons(orc):
    A = spkgen.laplace2d5(10)
    b = spkgen.rhs_uniform(A.n, 0)
    # maxit
    x, res, _ = oracle.pcg(A, b, maxit=3)
    assert res["reason_str"] == "DIVERGED_ITS" and res["iterations"] == 3
    # zero rhs
    x, res, _ = oracle.pcg(A, np.zeros(A.n))
    assert res["reason_str"] == "CONVERGED_ATOL" and res["iterations"] == 0 and not x.any()
    # NaN rhs
    bn = b.copy()
    bn[5] = np.nan
    _, res, _ = oracle.pcg(A, bn)
    assert res["reason_str"] == "DIVERGED_NANORINF"
    # negative definite: Jacobi gives r.z < 0 at the start
    An = spkgen.CSR(A.n, A.rowptr, A.col, -A.val)
    _, res, _ = oracle.pcg(An, b)
    assert res["reason_str"] == "DIVERGED_INDEFINITE_PC"
    # indefinite with positive diagonal: p.Ap < 0 on the first step
    Ai = spkgen.dense_to_csr(np.array([[1.0, 2.0], [2.0, 1.0]]))
    x, res, _ = oracle.pcg(Ai, np.array([1.0, -1.0]))
    assert res["reason_str"] == "DIVERGED_INDEFINITE_MAT" and res["iterations"] == 0
    assert not x.any()
    # atol
    _, res, _ = oracle.pcg(A, b, rtol=0.0, atol=1e-3)
    assert res["reason_str"] == "CONVERGED_ATOL" and res["rnorm"] <= 1e-3
    # x0 already the solution
    xs = np.linalg.solve(spkgen.to_dense(A), b)
    _, res, _ = oracle.pcg(A, b, x0=xs, rtol=1e-8)
    assert res["iterations"] == 0 and res["reason"] > 0


def test_pcg_true_residual_restart_rule(orc):
    """An unreachable rtol makes the recursive residual pass while the true
    residual cannot: the oracle restarts from the true residual, at most three
    times, then reports BREAKDOWN."""
    A = spkgen.laplace2d5(32)
    b = spkgen.rhs_uniform(A.n, 0)
    _, res, _ = oracle.pcg(A, b, rtol=1e-17, maxit=100000)
    assert res["reason_str"] in ("DIVERGED_BREAKDOWN", "CONVERGED_RTOL")
    if res["reason_str"] == "DIVERGED_BREAKDOWN":
        assert res["restarts"] == 3
    assert res["true_rel_residual"] < 1e-13


# ---------------------------------------------------------------- Chebyshev smoother

def cheb_T(k, y):
    """Chebyshev polynomial of the first kind, T_k(y), from its closed forms
    (cos(k arccos y) inside [-1, 1], cosh(k arccosh |y|) with sign (+-1)^k
    outside)."""
    if abs(y) <= 1.0:
        return math.cos(k * math.acos(y))
    v = math.cosh(k * math.acosh(abs(y)))
    return v if y > 0 or k % 2 == 0 else -v


def cheb_P(k, t, emin, emax):
    """Error polynomial of k Chebyshev steps on [emin, emax]:
    T_k((theta - t)/delta) / T_k(theta/delta)."""
    theta, delta = (emax + emin) / 2, (emax - emin) / 2
    return cheb_T(k, (theta - t) / delta) / cheb_T(k, theta / delta)


@pytest.mark.parametrize("steps", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("ks", [(1, 1), (3, 5), (10, 2), (16, 16)])
def test_chebyshev_eigenvector_error_polynomial(orc, steps, ks):
    """With b = A v for an eigenvector v of D^-1 A (constant diagonal) and
    x0 = 0, the error after k steps is exactly P_k(mu) v, so x_k =
    (1 - P_k(mu)) v; mu inside and outside [emin, emax]."""
    N = 16
    A = spkgen.laplace2d5(N)
    v, lam = lap_eigpair(N, 2, ks)
    mu = lam / 4.0
    b = spkgen.to_dense(A) @ v
    emin, emax = 0.3, 1.9
    x, r = oracle.chebyshev(A, b, steps, emin, emax)
    expect = (1.0 - cheb_P(steps, mu, emin, emax)) * v
    assert np.allclose(x, expect, rtol=0, atol=1e-13 * (1 + abs(cheb_P(steps, mu, emin, emax))))
    # the recursive residual is the true one
    assert np.allclose(r, b - spkgen.to_dense(A) @ x, rtol=0, atol=1e-12)


def test_chebyshev_linear_in_eigencomponents(orc):
    N = 12
    A = spkgen.laplace2d5(N, 0.5)
    Ad = spkgen.to_dense(A)
    comps = [lap_eigpair(N, 2, ks, shift=0.5) for ks in ((1, 2), (6, 6), (12, 11))]
    v = sum(c[0] for c in comps)
    b = Ad @ v
    emin, emax = 0.25, 2.2
    x, _ = oracle.chebyshev(A, b, 4, emin, emax)
    expect = sum((1 - cheb_P(4, lam / 4.5, emin, emax)) * w for w, lam in comps)
    assert np.allclose(x, expect, rtol=0, atol=1e-12)


def test_chebyshev_one_step_is_damped_jacobi(orc):
    A, _ = random_int_csr(40, 3)
    b = spkgen.rhs_uniform(A.n, 1)
    d = np.diag(spkgen.to_dense(A))
    x, r = oracle.chebyshev(A, b, 1, 0.5, 1.5)
    assert np.allclose(x, b / d / 1.0, rtol=1e-15, atol=0)  # theta = (0.5 + 1.5) / 2 = 1
    x, r = oracle.chebyshev(A, b, 0, 0.5, 1.5)
    assert np.array_equal(x, np.zeros(A.n)) and np.array_equal(r, b)


def test_chebyshev_exact_start_stays_exact(orc):
    """x0 = integer exact solution of an integer system: r0 = 0 exactly and
    every step adds exact zeros."""
    A = spkgen.laplace3d7(6)
    xs = np.random.default_rng(0).integers(-20, 20, A.n).astype(np.float64)
    b = spkgen.to_dense(A) @ xs
    x, r = oracle.chebyshev(A, b, 5, 0.1, 2.0, x0=xs)
    assert np.array_equal(x, xs) and not r.any()


def test_chebyshev_converges_at_chebyshev_rate(orc):
    """On the exact spectral interval [mu_min, mu_max] every eigencomponent
    of the error shrinks by at least 1/T_k(sigma), hence so does the
    Euclidean error norm (A symmetric, D constant)."""
    N = 10
    A = spkgen.laplace2d5(N)
    Ad = spkgen.to_dense(A)
    mus = np.linalg.eigvalsh(Ad) / 4.0
    emin, emax = float(mus.min()), float(mus.max())
    xs = spkgen.rhs_uniform(A.n, 4)
    b = Ad @ xs
    for k in (2, 5, 9):
        x, _ = oracle.chebyshev(A, b, k, emin, emax)
        bound = 1.0 / cheb_T(k, (emax + emin) / (emax - emin))
        assert np.linalg.norm(x - xs) <= bound * np.linalg.norm(xs) * (1 + 1e-9)


def test_chebyshev_rejects_bad_interval(orc):
    A = spkgen.laplace2d5(4)
    b = np.ones(A.n)
    for emin, emax in ((0.0, 1.0), (1.0, 1.0), (2.0, 1.0), (-1.0, 1.0)):
        with pytest.raises(ValueError):
            oracle.chebyshev(A, b, 2, emin, emax)


def test_gershgorin_bound(orc):
    A = spkgen.laplace2d5(9)
    assert oracle.gershgorin(A) == 2.0  # interior rows: (4 + 4) / 4
    for seed in range(3):
        A, D = random_int_csr(30, seed)
        direct = max(np.abs(D[i]).sum() / abs(D[i, i]) for i in range(30))
        g = oracle.gershgorin(A)
        assert g == pytest.approx(direct, rel=1e-15)
        M = D / np.diag(D)[:, None]
        assert np.abs(np.linalg.eigvals(M)).max() <= g * (1 + 1e-12)
    A = spkgen.diffusion3d27_lognormal(6, seed=1)
    assert 1.0 < oracle.gershgorin(A) <= 2.0 + 1e-15


# ---------------------------------------------------------------- single-reduction PCG

SR = {"single_reduction": True}


@pytest.mark.parametrize("dim,N,ks", [(2, 16, (1, 1)), (2, 30, (4, 9)), (3, 8, (2, 3, 5))])
def test_pcg_sr_eigenvector_rhs_one_iteration(orc, dim, N, ks):
    A = spkgen.laplace2d5(N) if dim == 2 else spkgen.laplace3d7(N)
    v, lam = lap_eigpair(N, dim, ks)
    x, res, _ = oracle.pcg(A, v, rtol=1e-12, hist_len=10, **SR)
    assert res["reason_str"] == "CONVERGED_RTOL" and res["iterations"] == 1
    assert np.allclose(x, v / lam, rtol=1e-12, atol=1e-13 * np.abs(v).max() / lam)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_pcg_sr_finite_termination(orc, m):
    N = 24
    A = spkgen.laplace2d5(N)
    ks = [(1, 1), (2, 3), (5, 5), (7, 2), (11, 13)][:m]
    pairs = [lap_eigpair(N, 2, k) for k in ks]
    b = sum(v for v, _ in pairs)
    x, res, hist = oracle.pcg(A, b, rtol=1e-9, hist_len=20, **SR)
    assert res["reason"] > 0 and res["iterations"] == m
    assert hist[m] / hist[0] < 1e-9 and hist[m - 1] / hist[0] > 1e-3
    xs = sum(v / lam for v, lam in pairs)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_pcg_sr_exact_rational_iterates(orc):
    """The single-reduction recurrences produce CG's iterates: compared with
    Jacobi-PCG carried out in exact rational arithmetic (brute force)."""
    D = np.array([[4, -1, 0, -2, 0], [-1, 5, -1, 0, 1], [0, -1, 3, -1, 0],
                  [-2, 0, -1, 6, -1], [0, 1, 0, -1, 2]], dtype=np.float64)
    n = D.shape[0]
    b = np.array([1.0, -2.0, 0.5, 3.0, -1.0])
    A = spkgen.dense_to_csr(D)
    F = [[Fraction(int(D[i, j])) for j in range(n)] for i in range(n)]
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    z = [r[i] / F[i][i] for i in range(n)]
    p = z[:]
    rho = sum(r[i] * z[i] for i in range(n))
    ex_x = []
    for _ in range(n):
        q = [sum(F[i][j] * p[j] for j in range(n)) for i in range(n)]
        alpha = rho / sum(p[i] * q[i] for i in range(n))
        x = [x[i] + alpha * p[i] for i in range(n)]
        r = [r[i] - alpha * q[i] for i in range(n)]
        ex_x.append([float(v) for v in x])
        if all(v == 0 for v in r):
            break
        z = [r[i] / F[i][i] for i in range(n)]
        rho_new = sum(r[i] * z[i] for i in range(n))
        p = [z[i] + (rho_new / rho) * p[i] for i in range(n)]
        rho = rho_new
    for kk in range(1, len(ex_x) + 1):
        xk, rk, _ = oracle.pcg(A, b, rtol=0.0, maxit=kk, **SR)
        if rk["reason_str"] != "DIVERGED_ITS":
            break
        assert np.allclose(xk, ex_x[kk - 1], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("case", ["lap2d_64", "lap3d_16", "diff27_8", "powerlaw_3k"])
def test_pcg_sr_matches_textbook_cg(orc, case):
    """Same Krylov method: residual histories agree with the (pinned)
    textbook oracle to 1e-10 for 20 steps, counts within one."""
    A = {"lap2d_64": lambda: spkgen.laplace2d5(64), "lap3d_16": lambda: spkgen.laplace3d7(16),
         "diff27_8": lambda: spkgen.diffusion3d27_lognormal(8, seed=3),
         "powerlaw_3k": lambda: spkgen.powerlaw_spd(3000, seed=2)}[case]()
    b = spkgen.rhs_uniform(A.n, 1)
    x1, r1, h1 = oracle.pcg(A, b, hist_len=2000)
    x2, r2, h2 = oracle.pcg(A, b, hist_len=2000, **SR)
    assert r1["reason"] == r2["reason"] == 1
    assert abs(r1["iterations"] - r2["iterations"]) <= 1
    assert np.allclose(h2[:21], h1[:21], rtol=1e-10, atol=0)
    assert r2["true_rel_residual"] <= 1e-8
    assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x1)


def test_pcg_sr_a_norm_error_monotone(orc):
    A = spkgen.diffusion3d27_lognormal(5, seed=0)
    D = spkgen.to_dense(A)
    b = spkgen.rhs_uniform(A.n, 2)
    xs = np.linalg.solve(D, b)
    errs = []
    for k in range(0, 25):
        xk, _, _ = oracle.pcg(A, b, rtol=0.0, maxit=k, **SR)
        e = xs - xk
        errs.append(math.sqrt(e @ D @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-3 * errs[0]


def test_pcg_sr_reasons(orc):
    A = spkgen.laplace2d5(10)
    b = spkgen.rhs_uniform(A.n, 0)
    _, r, _ = oracle.pcg(A, b, maxit=5, **SR)
    assert r["reason_str"] == "DIVERGED_ITS" and r["iterations"] == 5
    x, r, _ = oracle.pcg(A, np.zeros(A.n), **SR)
    assert r["reason_str"] == "CONVERGED_ATOL" and r["iterations"] == 0 and not x.any()
    xs = np.random.default_rng(0).integers(-5, 5, A.n).astype(np.float64)
    x, r, _ = oracle.pcg(A, oracle.spmv(A, xs), x0=xs, **SR)
    assert r["iterations"] == 0 and np.array_equal(x, xs)
    # symmetric indefinite: negative diagonal entries
    Dm = spkgen.to_dense(A)
    Dm[np.arange(0, A.n, 2), np.arange(0, A.n, 2)] *= -1
    _, r, _ = oracle.pcg(spkgen.dense_to_csr(Dm), b, **SR)
    assert r["reason_str"] in ("DIVERGED_INDEFINITE_PC", "DIVERGED_INDEFINITE_MAT")


def test_parallel_oracle_build_matches_serial():
    """The OpenMP build (used only to time the oracle on all host cores) runs
    the same loops: products bit-identical to the serial build, inner products
    equal up to the long-double rounding of its fixed chunks, and the same
    PCG iteration count and solution on the 64^2 Laplacian."""
    import oracle

    lo = oracle.load_omp()
    A = spkgen.laplace3d7(40)
    x = spkgen.rhs_uniform(A.n, 3)
    assert np.array_equal(oracle.spmv(A, x), oracle.spmv(A, x, lib=lo))
    y = spkgen.rhs_uniform(A.n, 4)
    d0, d1 = oracle.dot(x, y), oracle.dot(x, y, lib=lo)
    assert abs(d0 - d1) <= 1e-15 * float(np.abs(x) @ np.abs(y))
    assert oracle.nrm2(x, lib=lo) == pytest.approx(oracle.nrm2(x), rel=1e-15)
    B = spkgen.laplace2d5(64)
    b = spkgen.rhs_uniform(B.n, 0)
    xs, rs, _ = oracle.pcg(B, b)
    xp, rp, _ = oracle.pcg(B, b, lib=lo)
    assert rp["iterations"] == rs["iterations"] == 193
    assert np.linalg.norm(xp - xs) <= 1e-12 * np.linalg.norm(xs)
