"""GPU tests of the failure paths of the Krylov drivers and of allocation,
through the C ABI, against the oracle where it defines the result:
GMRES and BiCGSTAB stopped by maxit (E_NOTCONV with the partial iterate),
a zero right-hand side, BiCGSTAB breakdowns (an inner product exactly zero),
E_NOMEM from a failing allocator callback, and the watchdog inside a
batched graph."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_0803_0048_amd import binding as T
from paper_0803_0048_amd import inputs as I
from tests.gpu_util import assert_bits_equal, g, log

pytestmark = pytest.mark.gpu


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


def _csr_from_dense(M):
    n = M.shape[0]
    mask = M != 0
    np.fill_diagonal(mask, True)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(mask.sum(axis=1))
    rows, cols = np.nonzero(mask)
    return I.CSR(n, rp, cols.astype(np.int32), M[rows, cols].astype(np.float64))


def _setup(A, k):
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, bad = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(A.val))
    assert_bits_equal(f, vF, "F")
    return pat, f, (rpF, ciF, vF)


def _same(info, ref, x, what):
    assert info["status"] == ref["status"], (what, info["status"], ref["status"])
    assert info["iters"] == ref["iters"], (what, info["iters"], ref["iters"])
    assert_bits_equal(np.array(info["hist"]), ref["hist"], f"{what}: history")
    assert_bits_equal(x, ref["x"], f"{what}: x")
    assert_bits_equal(np.array([info["relres"]]), np.array([ref["relres"]]), f"{what}: relres")


@pytest.mark.parametrize("restart,maxit", [(30, 3), (2, 5)])
def test_gmres_maxit_returns_partial_iterate(restart, maxit):
    c = I.conv_diff_2d_64x64_ilu1()
    A, b = c["A"], c["b"]
    pat, f, (rpF, ciF, vF) = _setup(A, 1)
    ref = O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, restart=restart, maxit=maxit, rtol=1e-14)
    assert ref["status"] == O.ENOTCONV
    x, info = T.gmres(pat, g(A.val), f, g(b), restart=restart, maxit=maxit, rtol=1e-14)
    assert info["status"] == T.E_NOTCONV
    _same(info, ref, x, f"GMRES({restart}) maxit {maxit}")
    with pytest.raises(T.TpiluError):
        T.gmres(pat, g(A.val), f, g(b), restart=restart, maxit=maxit, rtol=1e-14, raise_notconv=True)


def test_bicgstab_maxit_returns_partial_iterate():
    c = I.conv_diff_2d_64x64_ilu1()
    A, b = c["A"], c["b"]
    pat, f, (rpF, ciF, vF) = _setup(A, 1)
    ref = O.bicgstab(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, maxit=3, rtol=1e-14)
    assert ref["status"] == O.ENOTCONV and ref["iters"] == 3
    x, info = T.bicgstab(pat, g(A.val), f, g(b), maxit=3, rtol=1e-14)
    _same(info, ref, x, "BiCGSTAB maxit 3")


def test_zero_rhs():
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat, f, (rpF, ciF, vF) = _setup(A, 1)
    z = np.zeros(A.n)
    for name, run_g, run_o in (
            ("gmres", lambda: T.gmres(pat, g(A.val), f, g(z), x0=g(np.ones(A.n))),
             lambda: O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, z, x0=np.ones(A.n))),
            ("bicgstab", lambda: T.bicgstab(pat, g(A.val), f, g(z), x0=g(np.ones(A.n))),
             lambda: O.bicgstab(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, z, x0=np.ones(A.n)))):
        x, info = run_g()
        ref = run_o()
        assert info["status"] == T.OK, name
        assert not x.any(), f"{name}: a zero right-hand side gives x = 0"
        _same(info, ref, x, f"{name}, zero rhs")


# Two systems (small integers, exactly representable) on which BiCGSTAB with
# the ILU(0) preconditioner breaks down: an inner product it divides by is
# exactly zero.  The first breaks down before its first half step, the
# second after two.
BREAKDOWN = [
    ([[-1, 0, -1, -2], [0, 1, 0, -1], [2, 2, 4, 0], [0, -1, 0, 2]], [1, -1, -1, -1]),
    ([[-2, 0, -1, 0], [-2, 1, 0, 1], [0, 2, 2, 2], [1, 0, -2, -1]], [-1, 2, 2, 0]),
]


@pytest.mark.parametrize("case", range(len(BREAKDOWN)))
def test_bicgstab_breakdown(case):
    M, b = BREAKDOWN[case]
    A = _csr_from_dense(np.array(M, dtype=np.float64))
    b = np.array(b, dtype=np.float64)
    pat, f, (rpF, ciF, vF) = _setup(A, 0)
    ref = O.bicgstab(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, maxit=20, rtol=1e-12)
    assert ref["status"] == O.ENOTCONV and ref["iters"] < 20, ref
    x, info = T.bicgstab(pat, g(A.val), f, g(b), maxit=20, rtol=1e-12)
    _same(info, ref, x, f"breakdown case {case}")


# ---- allocation failure through the allocator callback ---------------------------
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class _Budget:
    """Device allocations through torch's caching allocator, refused once
    `left` reaches zero."""

    def __init__(self):
        self.left = 1 << 30
        self.live = set()
        self.refused = 0
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        if self.left <= 0:
            self.refused += 1
            return None
        self.left -= 1
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0)
        self.live.add(p)
        return p

    def _free(self, p, user):
        if p in self.live:
            self.live.discard(p)
            torch.cuda.caching_allocator_delete(p)


def test_enomem_from_allocator_callback():
    lib = T.load_library()
    bud = _Budget()
    h = C.c_void_p()
    stream = C.c_void_p(torch.cuda.current_stream(0).cuda_stream)
    assert lib.tpilu_ctx_create(0, stream, C.cast(bud.alloc, C.c_void_p), C.cast(bud.free, C.c_void_p), None,
                                C.byref(h)) == T.OK
    c = I.conv_diff_2d_64x64_ilu1()
    A, b = c["A"], c["b"]
    rp, ci, av, bv = g(A.rowptr), g(A.col), g(A.val), g(b)
    try:
        # no allocation allowed: symbolic fails cleanly
        bud.left = 0
        p = C.c_void_p()
        assert lib.tpilu_symbolic(h, A.n, A.nnz, C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()), 1,
                                  C.byref(p)) == T.E_NOMEM
        assert bud.refused >= 1 and not p
        # allocations allowed: symbolic and numeric succeed
        bud.left = 1 << 30
        assert lib.tpilu_symbolic(h, A.n, A.nnz, C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()), 1,
                                  C.byref(p)) == T.OK
        info = T.PatternInfo()
        lib.tpilu_pattern_info(p, C.byref(info))
        f = torch.empty(info.nnz_f, dtype=torch.float64, device="cuda:0")
        bad = C.c_int64(-1)
        assert lib.tpilu_numeric(h, p, C.c_void_p(av.data_ptr()), 1, C.c_void_p(f.data_ptr()), C.byref(bad)) == T.OK
        # GMRES needs its workspace: refused -> E_NOMEM, nothing written to x
        x = torch.full((A.n,), 7.0, dtype=torch.float64, device="cuda:0")
        it, rr = C.c_int32(0), C.c_double(0.0)
        bud.left = 0
        st = lib.tpilu_gmres(h, p, C.c_void_p(av.data_ptr()), C.c_void_p(f.data_ptr()), C.c_void_p(bv.data_ptr()),
                             C.c_void_p(x.data_ptr()), 30, 100, 1e-8, C.byref(it), C.byref(rr), None)
        assert st == T.E_NOMEM
        assert b"workspace" in lib.tpilu_last_error(h)
        assert torch.all(x == 7.0)
        # and the context recovers once memory is available
        bud.left = 1 << 30
        st = lib.tpilu_gmres(h, p, C.c_void_p(av.data_ptr()), C.c_void_p(f.data_ptr()), C.c_void_p(bv.data_ptr()),
                             C.c_void_p(x.data_ptr()), 30, 100, 1e-8, C.byref(it), C.byref(rr), None)
        assert st == T.OK and rr.value <= 1e-8
        torch.cuda.synchronize()
        lib.tpilu_pattern_destroy(p)
        assert not bud.live, "every allocation went back through the free callback"
    finally:
        torch.cuda.synchronize()
        lib.tpilu_ctx_destroy(h)


def test_batched_graph_watchdog_and_recovery():
    """A batched graph whose factorization never publishes one row (the
    library's test hook, forced from the host) ends with E_TIMEOUT: the rows
    waiting on it, the fused forward substitution and the backward sweep all
    give up at the watchdog and the kernels drain.  A graph captured after the
    hook is cleared gives the eager bits again."""
    c = I.batched_conv_diff_2d_ilu2(B=70, m=24)
    A, rhs = c["A"], c["b"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    av, bv = g(A.val), g(rhs)
    ctx = T.context(0)
    ctx.set_watchdog(timeout_us=20000, skip_publish_row=100)
    try:
        graph = T.BatchedGraph(pat, av, bv)
        graph.launch()
        with pytest.raises(T.TpiluError) as e:
            graph.check()
        assert e.value.status == T.E_TIMEOUT
    finally:
        ctx.set_watchdog(0, -1)
    del graph
    f = T.numeric(pat, av)
    y = T.apply(pat, f, bv)
    graph = T.BatchedGraph(pat, av, bv)
    graph.launch()
    assert graph.check() == -1
    assert torch.equal(graph.f_val.view(torch.int64), f.view(torch.int64))
    assert torch.equal(graph.y.view(torch.int64), y.view(torch.int64))
