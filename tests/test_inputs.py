"""Seeded input generators: sizes, symmetry, definiteness, reproducibility."""

import numpy as np
import pytest

import spkgen


@pytest.mark.parametrize("N", [1, 2, 5, 64])
def test_laplace2d5_nnz_and_values(N):
    A = spkgen.laplace2d5(N)
    assert A.n == N * N
    assert A.nnz == 5 * N * N - 4 * N
    assert A.rowptr.dtype == np.int32 and A.col.dtype == np.int32
    D = spkgen.to_dense(A) if N <= 8 else None
    if D is not None:
        assert np.array_equal(D, D.T)
        assert set(np.unique(A.val)) <= {4.0, -1.0}


@pytest.mark.parametrize("N", [1, 3, 6])
def test_laplace3d7_nnz(N):
    A = spkgen.laplace3d7(N)
    assert A.nnz == 7 * N ** 3 - 6 * N ** 2
    D = spkgen.to_dense(A)
    assert np.array_equal(D, D.T)
    np.linalg.cholesky(D)


def test_config_sizes_c1_c2():
    A = spkgen.laplace2d5(64)
    assert (A.n, A.nnz) == (4096, 20224)
    # C2's nnz by the closed form 7N^3 - 6N^2 (the full matrix is built in GPU tests)
    assert 7 * 128 ** 3 - 6 * 128 ** 2 == 14581760


def test_csr_structure_sorted_with_diagonal():
    for A in (spkgen.laplace2d5(7), spkgen.laplace3d7(4), spkgen.diffusion3d27_lognormal(4, 1),
              spkgen.powerlaw_spd(3000, 2)):
        for i in range(A.n):
            c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
            assert np.all(np.diff(c) > 0)
            assert i in c
        assert A.rowptr[0] == 0 and A.rowptr[-1] == A.nnz


@pytest.mark.parametrize("N", [2, 4, 9])
def test_diffusion27_nnz_symmetry_spd(N):
    A = spkgen.diffusion3d27_lognormal(N, seed=3)
    assert A.nnz == (3 * N - 2) ** 3
    D = spkgen.to_dense(A)
    assert np.array_equal(D, D.T)          # bitwise symmetric
    np.linalg.cholesky(D)                  # SPD
    # diagonal = sum of all 26 connection weights >= sum of |off-diagonals|
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) >= off * (1 - 1e-14))  # equality on interior rows
    assert np.any(np.diag(D) > off * 1.01)           # strict on boundary rows


def test_diffusion27_reproducible():
    a = spkgen.diffusion3d27_lognormal(5, seed=7)
    b = spkgen.diffusion3d27_lognormal(5, seed=7)
    c = spkgen.diffusion3d27_lognormal(5, seed=8)
    assert np.array_equal(a.val, b.val)
    assert not np.array_equal(a.val, c.val)


def test_powerlaw_symmetric_dominant_and_skewed():
    A = spkgen.powerlaw_spd(20000, seed=0)
    import scipy.sparse as sp

    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    assert (S != S.T).nnz == 0
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d - off > 0.999)          # diagonal = abs-sum + 1 (Gershgorin)
    L = A.row_lengths()
    assert L.min() >= 4                      # at least 3 picks + diagonal
    assert L.max() > 10 * L.mean()           # heavy tail
    B = spkgen.powerlaw_spd(20000, seed=0)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_serve_stream_statistics():
    reqs = spkgen.serve_stream(seed=0, rate=200.0, duration=60.0)
    assert 11000 < len(reqs) < 13000
    gaps = np.diff([0.0] + [r.t_arrival for r in reqs])
    assert abs(gaps.mean() - 0.005) < 0.0003
    dims = np.array([r.dim for r in reqs])
    assert 0.45 < (dims == 2).mean() < 0.55
    s2 = np.array([r.side for r in reqs if r.dim == 2])
    s3 = np.array([r.side for r in reqs if r.dim == 3])
    assert s2.min() >= 32 and s2.max() <= 256 and s3.min() >= 16 and s3.max() <= 96
    A = spkgen.serve_matrix(reqs[0])
    base = spkgen.laplace2d5(reqs[0].side) if reqs[0].dim == 2 else spkgen.laplace3d7(reqs[0].side)
    assert np.array_equal(A.col, base.col)
    diff = A.val - base.val
    assert np.count_nonzero(diff) == A.n and np.allclose(diff[diff != 0], reqs[0].shift)


def test_rhs_uniform():
    b = spkgen.rhs_uniform(100000, 0)
    assert b.min() >= -1 and b.max() < 1 and abs(b.mean()) < 0.01
    assert np.array_equal(b, spkgen.rhs_uniform(100000, 0))
