"""Seeded synthetic inputs for the CSR SpMV / Jacobi-PCG path.

This module builds the matrices and right-hand sides that both the CPU oracle
and the HIP library are run on.  It holds none of the solver's arithmetic: no
product, no reduction, no Krylov step -- only matrix assembly and random draws.
Everything is NumPy with ``numpy.random.default_rng(seed)`` (PCG64) and a fixed
draw order, so the same seed gives the same bits on every machine.

Conventions (the paper does not fix them, Sec. 4 "Progress on PETSc's back-end"
only names the CSR format MATAIJ):

* CSR with int32 ``rowptr`` (n+1) and int32 ``col`` (nnz), float64 ``val``.
* Grid unknowns are ordered lexicographically, x fastest:
  ``i + N*j + N*N*k``.  Columns are ascending within a row, no duplicates, and
  every row stores its diagonal.
* Dirichlet boundaries are eliminated: the unknowns are the N**dim interior
  points and neighbours that fall off the grid are dropped.
* Stencils are unscaled integers (2D: 4/-1, 3D 7-point: 6/-1); no h**-2 factor.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np

__all__ = [
    "CSR",
    "laplace2d5",
    "laplace3d7",
    "diffusion3d27_lognormal",
    "powerlaw_spd",
    "rhs_uniform",
    "ServeRequest",
    "serve_stream",
    "serve_matrix",
    "to_dense",
    "random_spd_dense_csr",
]


@dataclasses.dataclass
class CSR:
    """A square CSR matrix: int32 rowptr[n+1], int32 col[nnz], float64 val[nnz]."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)


def _stencil_csr(N, dim: int, offsets, weights) -> CSR:
    """Assemble a stencil on an N**dim grid (or a grid of shape N = (s_x, s_y
    [, s_z]), x fastest) with Dirichlet elimination.

    ``offsets`` are integer tuples (dx, dy[, dz]); ``weights[m]`` is a scalar or
    an array of length n giving the entry of row i for offset m.  Offsets are
    sorted by their linear displacement so that columns come out ascending.
    """
    ext = tuple(int(v) for v in N) if hasattr(N, "__len__") else (int(N),) * dim
    assert len(ext) == dim
    n = int(np.prod(ext))
    if n >= 2**31:
        raise ValueError("n does not fit int32 indices")
    stride = [int(np.prod(ext[:d])) for d in range(dim)]
    lin = [sum(o[d] * stride[d] for d in range(dim)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    m = len(offsets)
    shape = ext[::-1]  # C order: the last axis is x (fastest)
    mask = np.empty((n, m), dtype=bool)
    cols = np.empty((n, m), dtype=np.int32)
    vals = np.empty((n, m), dtype=np.float64)
    idx = np.arange(n, dtype=np.int32)
    for slot, o_i in enumerate(order):
        o = offsets[o_i]
        ok = np.ones(shape, dtype=bool)
        for d in range(dim):
            ax = dim - 1 - d
            sl = [slice(None)] * dim
            if o[d] > 0:
                sl[ax] = slice(ext[d] - o[d], None)
            elif o[d] < 0:
                sl[ax] = slice(0, -o[d])
            else:
                continue
            ok[tuple(sl)] = False
        mask[:, slot] = ok.ravel()
        np.add(idx, np.int32(lin[o_i]), out=cols[:, slot])
        vals[:, slot] = weights[o_i]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, rowptr.astype(np.int32), cols[mask], vals[mask])


def laplace2d5(N: int, shift: float = 0.0) -> CSR:
    """2D 5-point Laplacian on N x N interior points: diagonal 4 (+shift), off -1.

    nnz = 5N^2 - 4N.
    """
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    w = [4.0 + shift, -1.0, -1.0, -1.0, -1.0]
    return _stencil_csr(N, 2, offs, w)


def laplace3d7(N: int, shift: float = 0.0) -> CSR:
    """3D 7-point Laplacian on N^3 interior points: diagonal 6 (+shift), off -1.

    nnz = 7N^3 - 6N^2.
    """
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    w = [6.0 + shift] + [-1.0] * 6
    return _stencil_csr(N, 3, offs, w)


def laplace_grid(shape, shift: float = 0.0) -> CSR:
    """5-point (2D) or 7-point (3D) Laplacian on a grid of the given shape
    (x fastest): diagonal 2 dim (+shift), off-diagonal -1, Dirichlet
    elimination as in laplace2d5 / laplace3d7."""
    dim = len(shape)
    offs = [tuple(0 for _ in range(dim))]
    for d in range(dim):
        for sgn in (-1, 1):
            offs.append(tuple(sgn if e == d else 0 for e in range(dim)))
    w = [2.0 * dim + shift] + [-1.0] * (2 * dim)
    return _stencil_csr(tuple(shape), dim, offs, w)


def _canonical_dirs27():
    """The 13 neighbour directions of the 26-neighbourhood with positive
    linear displacement (x fastest), in a fixed order."""
    dirs = []
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        if (dx, dy, dz) == (0, 0, 0):
            continue
        key = (dz, dy, dx)
        if key > (0, 0, 0):
            dirs.append((dx, dy, dz))
    assert len(dirs) == 13
    return dirs


def diffusion3d27_lognormal(N: int, seed: int = 0) -> CSR:
    """27-point variable-coefficient diffusion on N^3 interior points.

    Reading of "face coefficients lognormal exp(N(0,1))": a weighted graph
    Laplacian over the 26-neighbourhood.  Every undirected connection between
    two interior points gets one weight w = exp(g), g ~ N(0,1), and
    A_ij = A_ji = -w; a connection that leaves the grid gets its own weight,
    which only adds to the diagonal (Dirichlet).  A_ii = sum of the weights of
    all 26 connections of i.  The matrix is symmetric and irreducibly
    diagonally dominant, hence SPD; nnz = (3N-2)^3.

    Draw order: one (26, n) standard-normal array.  Rows 0..12 are the weights
    of the connection from point i in canonical direction d (the shared edge
    weight when the neighbour is interior); rows 13..25 are the weights of the
    connection in direction -d, used only when point i - d is off the grid.
    """
    n = N ** 3
    rng = np.random.default_rng(seed)
    W = np.exp(rng.standard_normal((26, n)))
    dirs = _canonical_dirs27()
    idx = np.arange(n, dtype=np.int64)
    coord = [(idx // N ** d) % N for d in range(3)]

    def inside(o, sign):
        ok = np.ones(n, dtype=bool)
        for d in range(3):
            c = coord[d] + sign * o[d]
            ok &= (c >= 0) & (c < N)
        return ok

    offsets = [(0, 0, 0)]
    weights = [None]
    diag = np.zeros(n, dtype=np.float64)
    for m, o in enumerate(dirs):
        lin = o[0] + N * o[1] + N * N * o[2]
        wp = W[m]
        # connection i -> i + d: shared weight wp[i] (boundary weight if off-grid)
        diag += wp
        offsets.append(o)
        weights.append(-wp)
        # connection i -> i - d: shared weight wp[i - d] if i - d is interior,
        # otherwise the independent boundary weight W[13 + m][i]
        back_in = inside(o, -1)
        wm = np.where(back_in, np.roll(wp, lin), W[13 + m])
        diag += wm
        offsets.append((-o[0], -o[1], -o[2]))
        weights.append(-np.roll(wp, lin))
    weights[0] = diag
    return _stencil_csr(N, 3, offsets, weights)


def powerlaw_spd(n: int, seed: int = 0, a: float = 1.8, lo: int = 3, hi: int = 4000,
                 band: int | None = None) -> CSR:
    """Random SPD matrix with power-law row lengths and a symmetric pattern.

    Reading of "nnz/row Zipf(a) clipped to [lo, hi], symmetric pattern,
    values N(0,1) off-diagonal, diagonal = row abs-sum + 1":
    row i draws d_i = clip(zipf(a), lo, hi) off-diagonal picks, each column
    uniform over [0, n) without i; the pattern is the union of (i, j) and
    (j, i); one N(0,1) value is drawn per unordered pair (in ascending
    (lo, hi) order); A_ii = sum_j |A_ij| + 1 (strictly diagonally dominant,
    hence SPD).

    Draw order: zipf(n), integers(total picks), standard_normal(#pairs).

    band: the banded variant (a diagnostic that separates load balance from
    gather locality): each pick is uniform over [i - band, i + band] without
    i, reflected into [0, n) at the ends; same row-length law.
    """
    rng = np.random.default_rng(seed)
    d = np.clip(rng.zipf(a, n), lo, hi).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), d)
    if band is None:
        cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
        cols += cols >= rows
    else:
        off = rng.integers(1, band + 1, size=rows.size, dtype=np.int64)
        off = np.where(rng.integers(0, 2, size=rows.size) == 0, -off, off)
        cols = rows + off
        cols = np.where(cols < 0, -cols, cols)
        cols = np.where(cols >= n, 2 * (n - 1) - cols, cols)
        cols = np.where(cols == rows, (rows + 1) % n, cols)
    key = np.minimum(rows, cols) * n + np.maximum(rows, cols)
    del rows, cols
    key = np.unique(key)
    v = rng.standard_normal(key.size)
    up_r = key // n          # row of the upper-triangle entry (ascending)
    up_c = key % n           # its column (> up_r, ascending within a row)
    del key
    cnt_up = np.bincount(up_r, minlength=n)
    cnt_lo = np.bincount(up_c, minlength=n)
    absv = np.abs(v)
    diag = np.bincount(up_r, weights=absv, minlength=n)
    diag += np.bincount(up_c, weights=absv, minlength=n)
    diag += 1.0
    del absv
    counts = cnt_lo + 1 + cnt_up
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    # Within a row: lower entries (cols < i, ascending), the diagonal, then
    # upper entries (cols > i, ascending).
    lo_start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_lo, out=lo_start[1:])
    up_start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_up, out=up_start[1:])
    # upper entries, already sorted by (row, col)
    rank_up = np.arange(up_r.size, dtype=np.int64) - up_start[up_r]
    pos = rowptr[up_r] + cnt_lo[up_r] + 1 + rank_up
    col[pos] = up_c
    val[pos] = v
    del rank_up, pos
    # lower entries: entry (up_c, up_r); stable sort by up_c keeps up_r ascending
    perm = np.argsort(up_c, kind="stable")
    lr = up_c[perm]
    lc = up_r[perm]
    lv = v[perm]
    del perm
    rank_lo = np.arange(lr.size, dtype=np.int64) - lo_start[lr]
    pos = rowptr[lr] + rank_lo
    col[pos] = lc
    val[pos] = lv
    del lr, lc, lv, rank_lo, pos
    ar = np.arange(n, dtype=np.int64)
    pos = rowptr[:-1] + cnt_lo
    col[pos] = ar
    val[pos] = diag
    return CSR(n, rowptr.astype(np.int32), col, val)


def banded_spd(n: int, offsets, seed: int = 0, margin: float = 1.0, negative: bool = False) -> CSR:
    """SPD matrix whose row i couples to i + d for every positive d in
    ``offsets`` that stays inside [0, n) and, by symmetry, to i - d: one
    N(0,1) value g per coupled pair (-|g| with ``negative``: a weighted graph
    Laplacian, whose near-constant vectors make it ill-conditioned),
    diagonal = row abs-sum + ``margin`` (strictly diagonally dominant for
    margin > 0, hence SPD).  Columns are
    ascending within a row.  Draw order: standard_normal(n * len(offsets)),
    entry (i, i + d_k) takes draw i * len(offsets) + k."""
    d = np.unique(np.asarray(offsets, dtype=np.int64))
    if d.size == 0 or d[0] <= 0:
        raise ValueError("offsets must be positive")
    rng = np.random.default_rng(seed)
    draws = rng.standard_normal(n * d.size).reshape(n, d.size)
    if negative:
        draws = -np.abs(draws)
    i = np.arange(n, dtype=np.int64)
    up_ok = (i[:, None] + d[None, :]) < n          # entry (i, i + d_k) exists
    up = np.where(up_ok, draws, 0.0)
    # lower entry (i, i - d_k) holds the value of (i - d_k, i)
    lo_ok = (i[:, None] - d[None, :]) >= 0
    lo = np.zeros_like(up)
    for k, dk in enumerate(d):
        lo[dk:, k] = up[: n - dk, k]
    diag = np.abs(up).sum(axis=1) + np.abs(lo).sum(axis=1) + margin
    # row layout: lower entries by descending d (ascending column), diagonal,
    # upper entries by ascending d
    cols = np.concatenate([i[:, None] - d[None, ::-1], i[:, None], i[:, None] + d[None, :]], axis=1)
    vals = np.concatenate([lo[:, ::-1], diag[:, None], up], axis=1)
    keep = np.concatenate([lo_ok[:, ::-1], np.ones((n, 1), bool), up_ok], axis=1)
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), cols[keep].astype(np.int32), vals[keep].astype(np.float64))


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side with entries uniform in [-1, 1), float64."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def random_spd_dense_csr(n: int, seed: int, density: float = 1.0) -> CSR:
    """Small random SPD matrix (for brute-force checks): symmetric N(0,1)
    off-diagonal entries kept with probability ``density`` and a diagonal of
    row abs-sum + 1, stored as CSR (explicit zeros are not stored)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    keep = rng.random((n, n)) < density
    U = np.triu(G * keep, 1)
    A = U + U.T
    A[np.diag_indices(n)] = np.abs(A).sum(axis=1) + 1.0
    return dense_to_csr(A)


def dense_to_csr(A: np.ndarray) -> CSR:
    n = A.shape[0]
    nzmask = A != 0
    counts = nzmask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(counts, out=rowptr[1:])
    r, c = np.nonzero(nzmask)
    return CSR(n, rowptr, c.astype(np.int32), A[r, c].astype(np.float64))


def to_dense(A: CSR) -> np.ndarray:
    D = np.zeros((A.n, A.n))
    r = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    D[r, A.col] = A.val
    return D


@dataclasses.dataclass
class ServeRequest:
    """One request of the served solve stream."""

    t_arrival: float   # seconds after the start of the stream
    dim: int           # 2 or 3
    side: int          # grid side N
    shift: float       # added to the diagonal
    rhs_seed: int

    @property
    def n(self) -> int:
        return self.side ** self.dim


def serve_stream(seed: int = 0, rate: float = 200.0, duration: float = 60.0,
                 side2d=(32, 256), side3d=(16, 96), count: int | None = None):
    """Poisson arrivals of Laplacian solves (open-loop stream).

    Reading: inter-arrival times exponential with mean 1/rate; each request is
    2D 5-point or 3D 7-point with probability 1/2 each; the grid side is a
    uniform integer in the inclusive range; a diagonal shift uniform in [0, 1);
    rhs uniform in [-1, 1) from its own seed.  ``count`` (if given) takes the
    first ``count`` requests regardless of ``duration``.
    Draw order per request: exponential, random, integers, uniform, integers.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if count is None and t >= duration:
            break
        dim = 2 if rng.random() < 0.5 else 3
        lo, hi = side2d if dim == 2 else side3d
        side = int(rng.integers(lo, hi + 1))
        shift = float(rng.uniform(0.0, 1.0))
        rseed = int(rng.integers(0, 2**62))
        out.append(ServeRequest(t, dim, side, shift, rseed))
        if count is not None and len(out) >= count:
            break
    return out


_PATTERN_CACHE: dict = {}


def serve_matrix(req: ServeRequest, cache: bool = True) -> CSR:
    """The matrix of a served request: Laplacian of its dim/side plus the
    shift on the diagonal.  The unshifted pattern is cached per (dim, side)."""
    key = (req.dim, req.side)
    base = _PATTERN_CACHE.get(key) if cache else None
    if base is None:
        base = laplace2d5(req.side) if req.dim == 2 else laplace3d7(req.side)
        r = np.repeat(np.arange(base.n, dtype=np.int64), np.diff(base.rowptr))
        dpos = np.nonzero(base.col == r)[0]
        base = (base, dpos)
        if cache:
            _PATTERN_CACHE[key] = base
    A, dpos = base
    val = A.val.copy()
    val[dpos] += req.shift
    return CSR(A.n, A.rowptr, A.col, val)
