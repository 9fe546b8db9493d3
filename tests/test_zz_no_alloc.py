"""The allocation-free fused dot (spk_vec_dot2_noalloc) against spk_vec_dot2:
the same bits on two calls in a row, the second on a smaller input, so that
the second call reuses the partials the first one left in the shared static
scratch."""

import numpy as np
import pytest

from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _pair(spk, n, seed):
    import torch

    rng = np.random.default_rng(seed)
    x, y, w = (to_dev(rng.uniform(-1, 1, n)) for _ in range(3))
    ref = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    got = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    spk.vec_dot2(x, y, w, ref)
    spk.vec_dot2_noalloc(x, y, w, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy(), (x, y, w)


def test_noalloc_dot2_matches_allocating_entry_point():
    spk = need_gpu()
    import torch

    # large first (2048 blocks of partials), then smaller (fewer blocks, the
    # rest of the scratch still holding the first call's partials), then a
    # ragged tail of one block and the empty vector
    for n, seed in ((5_000_000, 0), (123_457, 1), (77, 2)):
        ref, got, (x, y, w) = _pair(spk, n, seed)
        assert np.array_equal(ref, got), (n, ref, got)
        xs, ys, ws = (t.cpu().numpy() for t in (x, y, w))
        scale = np.abs(xs) @ np.abs(ys) + np.abs(xs) @ np.abs(ws)
        assert abs(got[0] - float(xs @ ys)) <= 1e-13 * scale + 1e-300
        assert abs(got[1] - float(xs @ ws)) <= 1e-13 * scale + 1e-300
    # n = 0 (the pointers must still be valid): both entry points give 0, 0
    v = torch.ones(4, dtype=torch.float64, device="cuda")
    outs = []
    for fn in (spk._lib.spk_vec_dot2, spk._lib.spk_vec_dot2_noalloc):
        r = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        spk._check(fn(0, v.data_ptr(), v.data_ptr(), v.data_ptr(), r.data_ptr(), None), "dot2 n = 0")
        torch.cuda.synchronize()
        outs.append(r.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], [0.0, 0.0])
    # two calls in a row on the same stream before one synchronisation
    rng = np.random.default_rng(7)
    a = [to_dev(rng.uniform(-1, 1, 1_000_000)) for _ in range(3)]
    b = [to_dev(rng.uniform(-1, 1, 4099)) for _ in range(3)]
    ra, rb = (torch.empty(2, dtype=torch.float64, device="cuda") for _ in range(2))
    ga, gb = (torch.empty(2, dtype=torch.float64, device="cuda") for _ in range(2))
    spk.vec_dot2_noalloc(*a, ga)
    spk.vec_dot2_noalloc(*b, gb)
    spk.vec_dot2(*a, ra)
    spk.vec_dot2(*b, rb)
    torch.cuda.synchronize()
    assert np.array_equal(ga.cpu().numpy(), ra.cpu().numpy())
    assert np.array_equal(gb.cpu().numpy(), rb.cpu().numpy())


def test_noalloc_dot2_rejects_bad_arguments():
    spk = need_gpu()
    import torch

    x = torch.ones(8, dtype=torch.float64, device="cuda")
    with pytest.raises(spk.SpkError) as e:
        spk._check(spk._lib.spk_vec_dot2_noalloc(-1, x.data_ptr(), x.data_ptr(), x.data_ptr(),
                                                  x.data_ptr(), None), "spk_vec_dot2_noalloc")
    assert e.value.status == spk.EINVAL
    with pytest.raises(spk.SpkError):
        spk._check(spk._lib.spk_vec_dot2_noalloc(8, x.data_ptr(), x.data_ptr(), None, x.data_ptr(), None),
                   "spk_vec_dot2_noalloc")
