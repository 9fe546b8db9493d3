"""Continuous-batching server: each request's result matches the oracle, is
bitwise the same alone and inside a mixed batch, and admission honours the
HBM budget."""

import numpy as np
import pytest

import oracle
import spkgen
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def _requests(count, seed=0):
    reqs = spkgen.serve_stream(seed=seed, count=count, side2d=(8, 40), side3d=(6, 14))
    out = []
    for r in reqs:
        A = spkgen.serve_matrix(r)
        out.append((r, A, spkgen.rhs_uniform(A.n, r.rhs_seed % (2**31))))
    return out


def _run(spk, S, items, prec, max_rounds=100000):
    tickets = []
    for _, A, b in items:
        o = spk.ksp_opts(precision=prec)
        tickets.append(spk.server_submit(S, A.rowptr, A.col, A.val, b, o))
    results = [None] * len(items)
    rounds = 0
    while any(r is None for r in results):
        spk.server_progress(S, 4)
        for i, t in enumerate(tickets):
            if results[i] is None:
                x = np.empty(items[i][1].n)
                got = spk.server_poll(S, t, x)
                if got is not None:
                    results[i] = (x, got[0])
        rounds += 1
        assert rounds < max_rounds
    return results


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_results_match_oracle(prec):
    spk = need_gpu()
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    items = _requests(12, seed=1)
    opts = spk.server_opts_default()
    opts.max_slots = 5  # fewer slots than requests: continuous admission
    opts.graph_k = 4
    S = spk.server_create(opts)
    results = _run(spk, S, items, p)
    for (req, A, b), (x, res) in zip(items, results):
        assert res.reason == spk.CONVERGED_RTOL, (req, res.as_dict())
        rel = oracle.nrm2(b - oracle.spmv(A, x)) / oracle.nrm2(b)
        assert rel <= 1e-8 * (1 + 1e-6), (req, rel)
        assert res.true_rel_residual == pytest.approx(rel, rel=1e-6, abs=1e-16)
        xo, ro, _ = oracle.pcg(A, b, rtol=1e-8)
        assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)
        if p == spk.PREC_FP64:
            assert abs(res.iterations - ro["iterations"]) <= max(2, 0.01 * ro["iterations"])
    S.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_alone_equals_mixed_batch(prec):
    spk = need_gpu()
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    items = _requests(8, seed=2)
    S = spk.server_create()
    mixed = _run(spk, S, items, p)
    S.close()
    for i, item in enumerate(items):
        S1 = spk.server_create()
        (x1, r1), = _run(spk, S1, [item], p)
        S1.close()
        x, r = mixed[i]
        assert np.array_equal(x1, x), f"request {i} differs alone vs in the batch"
        assert (r1.iterations, r1.inner_iterations, r1.outer_steps) == \
            (r.iterations, r.inner_iterations, r.outer_steps)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_midflight_admission_alone_equals_batch(prec):
    """Continuous admission: 10 requests submitted one at a time between
    server_progress calls, with 3 slots, so each one enters while earlier
    ones are still iterating (checked) and, once the slots are taken, waits
    for and takes a slot another request has just freed.  Every result is
    bitwise the one the same request gets alone, with the same iteration
    counts."""
    spk = need_gpu()
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    items = _requests(10, seed=5)
    opts = spk.server_opts_default()
    opts.max_slots = 3
    opts.graph_k = 2
    S = spk.server_create(opts)
    tickets, results = [], [None] * len(items)

    def collect():
        for i, t in enumerate(tickets):
            if results[i] is None:
                x = np.empty(items[i][1].n)
                got = spk.server_poll(S, t, x)
                if got is not None:
                    results[i] = (x, got[0])

    in_flight_at_submit = []
    for _, A, b in items:
        collect()
        in_flight_at_submit.append(sum(r is None for r in results[:len(tickets)]))
        tickets.append(spk.server_submit(S, A.rowptr, A.col, A.val, b, spk.ksp_opts(precision=p)))
        spk.server_progress(S, 1)
    rounds = 0
    while any(r is None for r in results):
        spk.server_progress(S, 1)
        collect()
        rounds += 1
        assert rounds < 100000
    S.close()
    # every request after the first arrived while others were on the GPU, and
    # more arrived than there are slots
    assert all(k > 0 for k in in_flight_at_submit[1:]), in_flight_at_submit
    assert max(in_flight_at_submit) >= opts.max_slots, in_flight_at_submit
    for i, item in enumerate(items):
        S1 = spk.server_create()
        (x1, r1), = _run(spk, S1, [item], p)
        S1.close()
        x, r = results[i]
        assert r.reason == spk.CONVERGED_RTOL
        assert np.array_equal(x1, x), f"request {i} differs alone vs admitted mid-flight"
        assert (r1.iterations, r1.inner_iterations, r1.outer_steps) == \
            (r.iterations, r.inner_iterations, r.outer_steps)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_large_systems_sell_product(prec):
    """Systems with short rows take the SELL-64 product (layout built on the
    device at admission), whatever their size; a power-law system (rows far
    over 64 entries) takes the stream-tile product in the same batch, so
    both product sections run in one step.  Every result meets the oracle's
    true residual and is bitwise the one the same request gets alone."""
    spk = need_gpu()
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    items = [(None, spkgen.laplace2d5(260, shift=0.3), None), (None, spkgen.laplace3d7(42, shift=0.2), None),
             (None, spkgen.laplace2d5(30, shift=0.1), None), (None, spkgen.laplace3d7(12, shift=0.5), None),
             (None, spkgen.powerlaw_spd(20000, seed=2), None)]
    items = [(r, A, spkgen.rhs_uniform(A.n, 11 + i)) for i, (r, A, _) in enumerate(items)]
    S = spk.server_create()
    mixed = _run(spk, S, items, p)
    S.close()
    for i, ((_, A, b), (x, res)) in enumerate(zip(items, mixed)):
        assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
        assert oracle.nrm2(b - oracle.spmv(A, x)) <= 1e-8 * oracle.nrm2(b) * (1 + 1e-6)
        S1 = spk.server_create()
        (x1, r1), = _run(spk, S1, [items[i]], p)
        S1.close()
        assert np.array_equal(x1, x), f"request {i} differs alone vs in the batch"
        assert (r1.iterations, r1.inner_iterations) == (res.iterations, res.inner_iterations)


def test_server_budget_and_errors():
    spk = need_gpu()
    opts = spk.server_opts_default()
    opts.hbm_budget_bytes = 4 << 20
    S = spk.server_create(opts)
    big = spkgen.laplace3d7(40)  # ~64k rows: does not fit 4 MiB
    with pytest.raises(spk.SpkError) as e:
        spk.server_submit(S, big.rowptr, big.col, big.val, np.ones(big.n))
    assert e.value.status == spk.EBUDGET
    # requests that fit only one or two at a time still all complete (queueing)
    items = [(None, spkgen.laplace2d5(100), spkgen.rhs_uniform(10000, s)) for s in range(4)]
    results = _run(spk, S, items, spk.PREC_FP64)
    for (_, A, b), (x, res) in zip(items, results):
        assert res.reason == spk.CONVERGED_RTOL
    Z = spkgen.dense_to_csr(np.array([[1.0, 2.0], [2.0, 0.0]]))
    with pytest.raises(spk.SpkError) as e:
        spk.server_submit(S, Z.rowptr, Z.col, Z.val, np.ones(2))
    assert e.value.status == spk.EZERODIAG
    A = spkgen.laplace2d5(5)
    bad = A.col.copy()
    bad[3] = 99
    with pytest.raises(spk.SpkError) as e:
        spk.server_submit(S, A.rowptr, bad, A.val, np.ones(A.n))
    assert e.value.status == spk.EINVAL
    with pytest.raises(spk.SpkError) as e:
        spk.server_poll(S, 123456789, np.empty(1))
    assert e.value.status == spk.ENOTFOUND
    S.close()


def test_server_failure_isolated():
    """A failing system (indefinite) finishes with its reason while the other
    systems of the batch converge unaffected."""
    spk = need_gpu()
    good = [(None, spkgen.laplace2d5(30), spkgen.rhs_uniform(900, 1)),
            (None, spkgen.laplace3d7(9), spkgen.rhs_uniform(729, 2))]
    A = spkgen.laplace2d5(20)
    bad = (None, spkgen.CSR(A.n, A.rowptr, A.col, -A.val), spkgen.rhs_uniform(A.n, 3))
    S = spk.server_create()
    res = _run(spk, S, [good[0], bad, good[1]], spk.PREC_FP64)
    assert res[1][1].reason == spk.DIVERGED_INDEFINITE_PC
    assert res[0][1].reason == spk.CONVERGED_RTOL and res[2][1].reason == spk.CONVERGED_RTOL
    S1 = spk.server_create()
    alone = _run(spk, S1, [good[0]], spk.PREC_FP64)
    assert np.array_equal(alone[0][0], res[0][0])


def test_server_completion_queue():
    """spk_server_completed reports every finished ticket exactly once, and
    only finished ones (each reported ticket can be collected at once)."""
    spk = need_gpu()
    items = _requests(10, seed=4)
    opts = spk.server_opts_default()
    opts.max_slots = 3
    S = spk.server_create(opts)
    tickets = [spk.server_submit(S, A.rowptr, A.col, A.val, b, spk.ksp_opts()) for _, A, b in items]
    n_of = {t: A.n for t, (_, A, _) in zip(tickets, items)}
    seen = []
    for _ in range(100000):
        spk.server_progress(S, 2)
        for t in spk.server_completed(S, cap=4):
            assert t in n_of and t not in seen
            got = spk.server_poll(S, t, np.empty(n_of[t]))
            assert got is not None and got[0].reason == spk.CONVERGED_RTOL
            seen.append(t)
        if len(seen) == len(tickets):
            break
    assert sorted(seen) == sorted(tickets)
    assert spk.server_completed(S) == []
    S.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_system_over_more_blocks_than_one_partial_chunk(prec):
    """max_blocks_per_system above 2048 (allowed up to 8192): a 760^2 system
    then spans 2256 blocks, more partials than the update pass loads in one
    chunk per thread, so every block takes the looped partial sum.  The
    result matches the oracle, and the same system over 256
    blocks converges in the same number of iterations within one."""
    spk = need_gpu()
    p = spk.PREC_FP64 if prec == "fp64" else spk.PREC_MIXED
    A = spkgen.laplace2d5(760, shift=0.5)
    b = spkgen.rhs_uniform(A.n, 9)
    xo, _, _ = oracle.pcg(A, b, rtol=1e-8)
    its = []
    for blocks in (4096, 256):
        opts = spk.server_opts_default()
        opts.max_blocks_per_system = blocks
        S = spk.server_create(opts)
        (x, res), = _run(spk, S, [(None, A, b)], p)
        assert res.reason == spk.CONVERGED_RTOL, res.as_dict()
        rel = oracle.nrm2(b - oracle.spmv(A, x)) / oracle.nrm2(b)
        assert rel <= 1e-8 * (1 + 1e-6), rel
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
        its.append(res.iterations)
        S.close()
    assert abs(its[0] - its[1]) <= 1, its
