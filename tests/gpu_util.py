"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""

import math

import numpy as np
import pytest

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_00715_amd import spk  # raises if the HIP library is missing

    return spk


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def mat_on_gpu(spk, A, flags=0):
    """spk_mat from a spkgen CSR, uploaded from device tensors."""
    return spk.mat_create_csr(to_dev(A.rowptr), to_dev(A.col), to_dev(A.val), flags=flags)


def spmv_bound_rows(A, kernel, lanes, u):
    """Per-row error bound factor (in units of sum_j |a_ij x_j|) of each
    kernel's summation order: stream sums the rounded products in sequence,
    vector sums ceil(len/L) FMA terms per lane then a log2(L) butterfly,
    merge walks <= 8 items per lane, an 8-level scan and a carry chain."""
    L = np.diff(A.rowptr).astype(np.float64)
    if kernel in ("stream", "sell", "sell_sigma"):  # sequential sum / FMA chain in column order
        f = L + 1
    elif kernel == "vector":
        f = np.ceil(L / lanes) + math.log2(lanes) + 2
    elif kernel == "sliced" and lanes == 2048:  # merge path over the slices, then 8 partials
        f = 8 + 8 + np.ceil(L / 2048) + 4 + 8
    elif kernel == "sliced":  # vector order within each of 8 column slices, then 8 partials in order
        f = np.ceil(L / lanes) + math.log2(lanes) + 8 + 2
    else:
        f = 8 + 8 + np.ceil(L / 2048) + 4
    return f * u


def check_spmv(y, y_ref, scale, tol_rows, what=""):
    err = np.abs(y - y_ref)
    bad = err > tol_rows * scale + 1e-300
    if bad.any():
        i = int(np.argmax(err / (scale + 1e-300)))
        raise AssertionError(f"{what}: {bad.sum()} rows exceed bound; worst row {i}: "
                             f"gpu {y[i]!r} ref {y_ref[i]!r} scale {scale[i]!r}")
