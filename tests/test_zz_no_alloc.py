"""tpilu_apply_noalloc: the triangular solves with the library allocating
nothing (its intermediate vector in a fixed device scratch).  Checked through
the C ABI against tpilu_apply, bit for bit, on two calls in a row with the
second one smaller, under stream capture (where an allocation would fail),
and for its size limit."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from paper_0803_0048_amd import binding as T
from paper_0803_0048_amd import inputs as I
from tests.gpu_util import assert_bits_equal, g, log

pytestmark = pytest.mark.gpu

SCRATCH = 1 << 22  # doubles in the library's fixed scratch


@pytest.fixture(autouse=True)
def _gpu_guard(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log(f"[gpu] {request.node.nodeid}")
    ctx = T.context(0)
    for fn in (ctx.set_grid, ctx.set_solver, ctx.set_numeric, ctx.set_placement, ctx.set_group, ctx.set_tickets):
        fn(0)
    ctx.set_watchdog(0, -1)
    yield
    torch.cuda.synchronize()


def _case(cfg, k):
    A = cfg["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(A.val))
    return A, pat, f, g(cfg["b"])


def test_noalloc_matches_apply_two_calls():
    # first call: 16 instances of the 32^3 7-point stencil, ILU(1) (524,288 values)
    A1, p1, f1, b1 = _case(I.differentiated_conv_diff_3d_ilu1(), 1)
    log(f"  call 1: n={A1.n} batch={A1.batch}")
    y1 = torch.empty_like(b1)
    T.apply_noalloc(p1, f1, b1, y1)
    assert T.check(p1) == -1
    assert_bits_equal(y1, T.apply(p1, f1, b1), "noalloc vs apply (batch 16)")
    # second, smaller call: one 64 x 64 stencil, ILU(1); also against the oracle
    c2 = I.conv_diff_2d_64x64_ilu1()
    A2, p2, f2, b2 = _case(c2, 1)
    log(f"  call 2: n={A2.n} batch=1")
    y2 = torch.empty_like(b2)
    T.apply_noalloc(p2, f2, b2, y2)
    assert T.check(p2) == -1
    assert_bits_equal(y2, T.apply(p2, f2, b2), "noalloc vs apply (one instance)")
    rpF, ciF, _ = O.symbolic(A2.n, A2.rowptr, A2.col, 1)
    vF, _ = O.numeric(A2.n, A2.rowptr, A2.col, A2.val, rpF, ciF)
    assert_bits_equal(y2, O.apply(A2.n, rpF, ciF, vF, c2["b"])[1], "noalloc vs oracle")
    # and the first case once more: nothing left in the scratch leaks in
    y1b = torch.empty_like(b1)
    T.apply_noalloc(p1, f1, b1, y1b)
    assert_bits_equal(y1b, y1, "noalloc repeated")


def test_noalloc_rejects_oversize():
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 1)
    B = SCRATCH // A.n + 1
    log(f"  n={A.n} batch={B}: n*batch={A.n * B} > {SCRATCH}")
    f = torch.zeros(pat.nnz_f, B, dtype=torch.float64, device="cuda:0")
    b = torch.zeros(A.n, B, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(b)
    with pytest.raises(T.TpiluError) as e:
        T.apply_noalloc(pat, f, b, y)
    assert e.value.status == T.E_INVAL
    assert "scratch" in str(e.value)


def test_noalloc_under_stream_capture():
    """Captured in a graph (global capture mode: an allocation would fail the
    capture), replayed three times with eager work between replays; every
    replay equals the eager tpilu_apply."""
    c = I.conv_diff_2d_64x64_ilu1()
    A, pat, f, b = _case(c, 1)
    y_ref = T.apply(pat, f, b)
    y = torch.empty_like(b)
    T.apply_noalloc(pat, f, b, y)  # warm: binds the context outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            T.apply_noalloc(pat, f, b, y)
    torch.cuda.current_stream().wait_stream(s)
    T.context(0)  # re-bind the library to the current stream
    for rep in range(3):
        y.fill_(0.0)
        graph.replay()
        torch.cuda.synchronize()
        assert_bits_equal(y, y_ref, f"replay {rep}")
        _ = T.apply(pat, f, b)  # eager work between replays
        torch.cuda.synchronize()
    assert T.check(pat) == -1
