"""Helpers shared by the GPU tests: moving seeded inputs to the device, running
the oracle on the same arrays, and bit-level comparison."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle as O


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def bits(a) -> np.ndarray:
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def assert_bits_equal(got, want, what=""):
    """Bitwise equality, except that a NaN matches any NaN: the sign and
    payload of a NaN produced by arithmetic are not part of the result (x86
    returns the negative default NaN, gfx950 the positive one)."""
    gb, wb = bits(got), bits(want)
    assert gb.shape == wb.shape, (what, gb.shape, wb.shape)
    gn = np.isnan(gb.view(np.float64))
    wn = np.isnan(wb.view(np.float64))
    diff = (gb != wb) & ~(gn & wn)
    if diff.any():
        bad = np.nonzero(diff.reshape(-1))[0]
        gv = gb.view(np.float64)
        wv = wb.view(np.float64)
        i = bad[0]
        raise AssertionError(f"{what}: {bad.size} of {gb.size} values differ; first at {i}: "
                             f"got {gv.flat[i]!r} ({gb.flat[i]:#x}) want {wv.flat[i]!r} ({wb.flat[i]:#x})")


def oracle_pattern(A, k):
    return O.symbolic(A.n, A.rowptr, A.col, k)


def check_pattern(pat, rpF, ciF, lvF, A=None):
    ex = pat.export()
    assert np.array_equal(ex["rowptr"].cpu().numpy(), rpF), "rowptr of F differs"
    assert np.array_equal(ex["col"].cpu().numpy(), ciF), "columns of F differ"
    assert np.array_equal(ex["level"].cpu().numpy(), np.minimum(lvF, 255).astype(np.uint8)), "levels differ"
    rows = np.repeat(np.arange(rpF.size - 1), np.diff(rpF))
    diag = np.nonzero(ciF == rows)[0]
    assert np.array_equal(ex["diag"].cpu().numpy(), diag), "diag slots differ"
    if A is not None:
        a2f = ex["a2f"].cpu().numpy()
        assert np.array_equal(ciF[a2f], A.col), "a2f maps to wrong columns"
        assert np.array_equal(rows[a2f], np.repeat(np.arange(A.n), np.diff(A.rowptr))), "a2f maps to wrong rows"
    return ex
