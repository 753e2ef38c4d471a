"""Race check run against the jitter build (libtpilu_jitter.so: the same
kernels with a pseudo-random pause before every publishing store and after
every coherent load).  Run as ``TPILU_LIBRARY=jitter python -m
tests.jitter_check`` in a process of its own (test_gpu_jitter.py does that):
every hand-off then happens at times the normal timing never produces, and
every result must still equal the oracle's bits.

Cases: pattern (levels on the whole device and on one XCD); both
single-instance factorization kernels in both placements, with either
rounding of the update; every solve shape;
the incomplete inverses and their products; GMRES; a batch in a graph (short
rows in LDS, fused forward substitution) and a batch with global-memory
working rows, each also with the fused update; the reverse-mode sweeps of a batch.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import torch

import oracle as O
from paper_0803_0048_amd import binding as T
from paper_0803_0048_amd import inputs as I
from tests.gpu_util import assert_bits_equal, check_pattern, g, log


def loaded_jitter_build() -> bool:
    with open("/proc/self/maps") as fh:
        return "libtpilu_jitter.so" in fh.read()


def single(name, A, k, b):
    ctx = T.context(0)
    log(f"jitter: {name} n={A.n} k={k}")
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    x_ref, y_ref = O.apply(A.n, rpF, ciF, vF, b)
    vG = O.inverse(A.n, rpF, ciF, vF)
    for place in (ctx.PLACE_DEVICE, ctx.PLACE_XCD):
        ctx.set_placement(place)
        pat = T.symbolic(g(A.rowptr), g(A.col), k)
        check_pattern(pat, rpF, ciF, lvF, A)
        modes = [ctx.NUMERIC_PIVOT] + ([ctx.NUMERIC_FLOW] if pat.info["flow_ready"] else [])
        for mode in modes:
            ctx.set_numeric(mode)
            assert_bits_equal(T.numeric(pat, g(A.val)), vF, f"{name} F numeric {mode} placement {place}")
        ctx.set_numeric(0)
        # the fused update (one rounding of f - l u) in both kernels
        vFf, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF, fused=True)
        ctx.set_fused(True)
        try:
            for mode in modes:
                ctx.set_numeric(mode)
                assert_bits_equal(T.numeric(pat, g(A.val)), vFf, f"{name} fused F numeric {mode} placement {place}")
        finally:
            ctx.set_fused(False)
        ctx.set_numeric(0)
    ctx.set_placement(0)
    f = T.numeric(pat, g(A.val))
    for solver, place in ((ctx.SOLVER_DEVICE, ctx.PLACE_DEVICE), (ctx.SOLVER_DEVICE, ctx.PLACE_XCD),
                          (ctx.SOLVER_WORKGROUP, 0), (ctx.SOLVER_LANES, 0)):
        ctx.set_solver(solver)
        ctx.set_placement(place)
        y, x = T.apply(pat, f, g(b), return_x=True)
        assert_bits_equal(x, x_ref, f"{name} x solver {solver} placement {place}")
        assert_bits_equal(y, y_ref, f"{name} y solver {solver} placement {place}")
    ctx.set_solver(0)
    ctx.set_placement(0)
    gv = T.inverse(pat, f)
    assert_bits_equal(gv, vG, f"{name} incomplete inverses")
    _, y_inv = O.apply_inverse(A.n, rpF, ciF, vG, b)
    assert_bits_equal(T.apply_inverse(pat, gv, g(b)), y_inv, f"{name} inverse products")
    ref = O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, restart=30, rtol=1e-8)
    x, info = T.gmres(pat, g(A.val), f, g(b), restart=30, rtol=1e-8)
    assert info["iters"] == ref["iters"], (name, info["iters"], ref["iters"])
    assert_bits_equal(x, ref["x"], f"{name} GMRES x")


def batched(name, A, k, rhs):
    log(f"jitter: {name} n={A.n} k={k} B={A.batch}")
    B = A.batch
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    av, bv = g(A.val), g(rhs)
    f = T.numeric(pat, av)
    y = T.apply(pat, f, bv)
    graph = T.BatchedGraph(pat, av, bv)
    graph.launch()
    assert graph.check() == -1
    fh, yh = f.cpu().numpy(), y.cpu().numpy()
    gf, gy = graph.f_val.cpu().numpy(), graph.y.cpu().numpy()
    for i in range(B):
        vF, _ = O.numeric(A.n, A.rowptr, A.col, np.ascontiguousarray(A.val[:, i]), rpF, ciF)
        _, yr = O.apply(A.n, rpF, ciF, vF, np.ascontiguousarray(rhs[:, i]))
        for what, got, want in (("F", fh, vF), ("y", yh, yr), ("graph F", gf, vF), ("graph y", gy, yr)):
            assert_bits_equal(got[:, i], want, f"{name} {what} instance {i}")
    ctx = T.context(0)
    ctx.set_fused(True)
    try:
        ffh = T.numeric(pat, av).cpu().numpy()
    finally:
        ctx.set_fused(False)
    for i in range(0, B, 5):
        vFf, _ = O.numeric(A.n, A.rowptr, A.col, np.ascontiguousarray(A.val[:, i]), rpF, ciF, fused=True)
        assert_bits_equal(ffh[:, i], vFf, f"{name} fused F instance {i}")


def adjoint(name, A, k, B, seed):
    log(f"jitter: {name} reverse mode n={A.n} k={k} B={B}")
    rng = np.random.default_rng(seed)
    vals = rng.uniform(-1, 1, (A.nnz, B))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    rowsum = np.zeros((A.n, B))
    np.add.at(rowsum, rows, np.abs(vals))
    diag = A.col == rows
    vals[diag] = 1.1 * rowsum[rows[diag]] + 1.0
    rhs, tgt = rng.standard_normal((A.n, B)), rng.standard_normal((A.n, B))
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(vals))
    y, x = T.apply(pat, f, g(rhs), return_x=True)
    bbar, fbar = T.apply_adjoint(pat, f, x, y, 2.0 * (y - g(tgt)))
    abar, _ = T.numeric_adjoint(pat, f, fbar)
    for i in range(B):
        vF, _ = O.numeric(A.n, A.rowptr, A.col, np.ascontiguousarray(vals[:, i]), rpF, ciF)
        xr, yr = O.apply(A.n, rpF, ciF, vF, rhs[:, i])
        bb, Fb = O.apply_adjoint(A.n, rpF, ciF, vF, xr, yr, 2.0 * (yr - tgt[:, i]))
        ab, _ = O.numeric_adjoint(A.n, A.rowptr, A.col, rpF, ciF, vF, Fb)
        assert_bits_equal(bbar[:, i].contiguous(), bb, f"{name} bbar {i}")
        assert_bits_equal(abar[:, i].contiguous(), ab, f"{name} abar {i}")


def arrow(n):
    M = np.zeros((n, n), bool)
    M[np.arange(n), np.arange(n)] = True
    M[-1, :] = True
    M[:, -1] = True
    M[np.arange(1, n), np.arange(n - 1)] = True
    rows, cols = np.nonzero(M)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return I.CSR(n, np.cumsum(rp), cols.astype(np.int32), np.zeros(rows.size))


def main() -> int:
    assert os.environ.get("TPILU_LIBRARY") == "jitter", "run with TPILU_LIBRARY=jitter"
    torch.cuda.set_device(0)
    T.load_library()
    assert loaded_jitter_build(), "the jitter build is not the library in use"
    log(f"jitter: library {T.LIB_PATH}")
    c = I.conv_diff_2d_64x64_ilu1()
    single("conv_diff_2d 64^2 ILU(1)", c["A"], 1, c["b"])
    c = I.random_banded_ilu2(n=6000)
    single("random banded n=6000 ILU(2)", c["A"], 2, c["b"])
    c = I.conv_diff_3d_ilu(m=16, k=1)
    single("conv_diff_3d 16^3 ILU(1)", c["A"], 1, c["b"])
    c = I.batched_conv_diff_2d_ilu2(B=70, m=24)
    batched("batched conv_diff_2d 24^2 ILU(2)", c["A"], 2, c["b"])
    A = arrow(400)
    rng = np.random.default_rng(3)
    vals = rng.uniform(-1, 1, (A.nnz, 66))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    vals[A.col == rows] = 4.0 * A.n
    batched("batched arrow n=400 (global working rows)", I.CSR(A.n, A.rowptr, A.col, vals), 2,
            rng.standard_normal((A.n, 66)))
    adjoint("random pattern n=240", I.random_pattern(240, 0.02, seed=99), 2, 5, 12)
    log("jitter build: all cases bitwise")
    return 0


if __name__ == "__main__":
    sys.exit(main())
