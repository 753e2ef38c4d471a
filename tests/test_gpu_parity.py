"""GPU parity: the HIP path (through the C ABI) against the sequential oracle,
bit for bit, on the same seeded inputs.

Small cases span many rows and wavefronts; the named workloads run at their
full sizes with the launch configuration the benchmark uses.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from paper_0803_0048_amd import binding as T
from paper_0803_0048_amd import inputs as I
from tests.gpu_util import assert_bits_equal, bits, check_pattern, g, log

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu_guard(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log(f"[gpu] {request.node.nodeid}")
    ctx = T.context(0)
    ctx.set_grid(0)
    ctx.set_solver(0)
    ctx.set_numeric(0)
    ctx.set_fused(False)
    ctx.set_placement(0)
    ctx.set_group(0)
    ctx.set_tickets(0)
    ctx.set_watchdog(0, -1)
    yield
    torch.cuda.synchronize()


def _full(A, k, b=None, check_gmres=None):
    """symbolic + numeric + apply on GPU and oracle, compared bit for bit"""
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    check_pattern(pat, rpF, ciF, lvF, A)
    vF, bad = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    f = T.numeric(pat, g(A.val), check=False)
    bad_g = T.check(pat) if bad < 0 else None
    assert_bits_equal(f, vF, "F")
    # both single-instance kernels, whichever the automatic choice was
    ctx = T.context(0)
    modes = [ctx.NUMERIC_PIVOT] + ([ctx.NUMERIC_FLOW] if pat.info["flow_ready"] else [])
    try:
        for mode in modes:
            ctx.set_numeric(mode)
            assert_bits_equal(T.numeric(pat, g(A.val), check=False), vF, f"F (numeric kernel {mode})")
    finally:
        ctx.set_numeric(0)
    if b is not None:
        x_ref, y_ref = O.apply(A.n, rpF, ciF, vF, b)
        y, x = T.apply(pat, f, g(b), return_x=True)
        assert_bits_equal(x, x_ref, "x = L^-1 b")
        assert_bits_equal(y, y_ref, "y = U^-1 x")
    del bad_g
    return pat, f, (rpF, ciF, vF)


# ----------------------------------------------------------------------------------
# arithmetic probes through the product path
# ----------------------------------------------------------------------------------
def test_division_and_update_rounding_bits():
    """2 x 2 instances [[a, b], [c, d]]: f_10 = c / a and f_11 = d - f_10 * b
    for a million random (and special) operands, against IEEE host arithmetic."""
    rng = np.random.default_rng(0)
    B = 1 << 20
    a = rng.standard_normal(B) * np.exp2(rng.integers(-1060, 1000, B).astype(np.float64) / 1.0)
    c = rng.standard_normal(B) * np.exp2(rng.integers(-1060, 1000, B).astype(np.float64))
    bb = rng.standard_normal(B) * np.exp2(rng.integers(-500, 500, B).astype(np.float64))
    d = rng.standard_normal(B) * np.exp2(rng.integers(-500, 500, B).astype(np.float64))
    sp = np.array([5e-324, -5e-324, 2.2250738585072014e-308, 1.7976931348623157e308, 1.0, -0.0, 3.0])
    a[: sp.size] = sp
    c[sp.size: 2 * sp.size] = sp
    a[a == 0] = 1.0
    rp = np.array([0, 2, 4], np.int64)
    ci = np.array([0, 1, 0, 1], np.int32)
    vals = np.stack([a, bb, c, d], axis=0)  # [nnz=4, B]
    pat = T.symbolic(g(rp), g(ci), 1)
    f = T.numeric(pat, g(vals), check=False)
    fh = f.cpu().numpy()
    with np.errstate(all="ignore"):
        l10 = c / a
        u11 = d - l10 * bb
    assert_bits_equal(fh[2], l10, "c / a")
    fin = np.isfinite(u11)
    assert_bits_equal(fh[3][fin], u11[fin], "d - l b")


def test_givens_sqrt_and_division_bits():
    """The rotation step of GMRES, rho = sqrt(a*a + b*b), c = a / rho,
    s = b / rho, on 2^20 operand pairs spread over the whole binary64 range
    (subnormal to overflowing squares, zeros, infinities, NaNs), against IEEE
    host arithmetic (numpy's sqrt and division are correctly rounded)."""
    rng = np.random.default_rng(7)
    B = 1 << 20
    a = rng.standard_normal(B) * np.exp2(rng.integers(-1074, 1024, B).astype(np.float64))
    b = rng.standard_normal(B) * np.exp2(rng.integers(-1074, 1024, B).astype(np.float64))
    # a quarter with the two magnitudes close (cancellation-free but sqrt of a
    # sum of comparable squares), a quarter of raw random bit patterns
    q = B // 4
    b[:q] = a[:q] * rng.uniform(0.5, 2.0, q)
    a[q:2 * q] = rng.integers(0, 1 << 63, q, dtype=np.uint64).view(np.float64) * rng.choice([-1, 1], q)
    b[q:2 * q] = rng.integers(0, 1 << 63, q, dtype=np.uint64).view(np.float64)
    sp = np.array([0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, 1.4916681462400413e-154,
                   1.3407807929942596e154, 1.7976931348623157e308, np.inf, -np.inf, np.nan, 1.0, 3.0])
    k = sp.size
    a[2 * q:2 * q + k * k] = np.repeat(sp, k)
    b[2 * q:2 * q + k * k] = np.tile(sp, k)
    rho, c, s = T.givens(g(a), g(b))
    with np.errstate(all="ignore"):
        rho_r = np.sqrt(a * a + b * b)
        c_r = a / rho_r
        s_r = b / rho_r
    assert_bits_equal(rho, rho_r, "rho = sqrt(a*a + b*b)")
    assert_bits_equal(c, c_r, "c = a / rho")
    assert_bits_equal(s, s_r, "s = b / rho")
    # and the norms of the solvers: sqrt of a fixed-shape inner product
    for n in (1, 2, 16385):
        x = rng.standard_normal(n) * 10.0 ** rng.uniform(-150, 150)
        got = T.dot(g(x), g(x))
        assert bits(np.array([np.sqrt(got)]))[0] == bits(np.array([np.sqrt(O.dot(x, x))]))[0]


def test_critical_path_and_handoff_probe():
    """The hop-count mode of the elimination on matrices whose critical path
    is known: a tridiagonal matrix chains every row on the previous one
    (n - 1 hand-offs), a diagonal one has none; the hand-off probe returns a
    finite round trip on one XCD and across two."""
    n = 500
    rp = np.arange(0, 3 * n - 1, 3, dtype=np.int64)
    rows = [[j - 1, j, j + 1] for j in range(n)]
    rows[0] = [0, 1]
    rows[-1] = [n - 2, n - 1]
    col = np.concatenate([np.array(r, np.int32) for r in rows])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    ctx = T.context(0)
    ctx.set_numeric(ctx.NUMERIC_FLOW)
    try:
        for k in (0, 2):
            pat = T.symbolic(g(rp), g(col), k)
            assert T.numeric_critical_path(pat) == n - 1, k
            # one l per row on the chain: l_{j,j-1} waits for u_{j-1,j-1}
            assert T.numeric_critical_path(pat, 0.0, 1.0) == n - 1, k
            assert T.numeric_critical_path(pat, 2.0, 0.5) == 2.5 * (n - 1), k
        pat = T.symbolic(g(np.arange(n + 1, dtype=np.int64)), g(np.arange(n, dtype=np.int32)), 0)
        assert T.numeric_critical_path(pat) == 0
    finally:
        ctx.set_numeric(0)
    for same in (True, False):
        rt = T.handoff_probe(same, rounds=2000)
        log(f"  hand-off round trip ({'one XCD' if same else 'two XCDs'}): {rt:.1f} ns")
        assert 0.0 < rt < 1e5


def test_dot_bits_and_fixed_shape():
    rng = np.random.default_rng(2)
    for n in (0, 1, 63, 16384, 16385, 100_003, 1_000_000):
        x = rng.standard_normal(n)
        y = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
        got = T.dot(g(x), g(y))
        want = O.dot(x, y) if n else 0.0
        assert bits(np.array([got]))[0] == bits(np.array([want]))[0], (n, got, want)
    x = np.zeros(16384 * 3)
    x[[0, 1, 2, 3]] = [2.0**53, 1, 1, 1]
    assert T.dot(g(x), g(np.ones_like(x))) == 2.0**53 + 2.0


def test_spmv_bits():
    A = I.conv_diff_2d_64x64_ilu1()["A"]
    x = np.random.default_rng(1).standard_normal(A.n)
    pat = T.symbolic(g(A.rowptr), g(A.col), 0)
    assert_bits_equal(T.spmv(pat, g(A.val), g(x)), O.spmv(A.n, A.rowptr, A.col, A.val, x), "A x")


# ----------------------------------------------------------------------------------
# small random matrices: many shapes, all k, explicit zeros and signed zeros
# ----------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_small_random_sweep(seed):
    rng = np.random.default_rng(4000 + seed)
    for case in range(30):
        n = int(rng.integers(1, 400))
        dens = float(rng.choice([0.002, 0.01, 0.03, 0.08]))
        A = I.random_pattern(n, dens, seed=int(rng.integers(1 << 30)), diag_dominant=bool(rng.integers(2)),
                             explicit_zeros=float(rng.choice([0.0, 0.2])))
        if case % 5 == 0 and A.nnz > 3:
            A.val[1] = -0.0
            A.val[2] = 5e-324
        k = int(rng.choice([0, 1, 2, 3, 5, n]))
        b = rng.standard_normal(n)
        _full(A, k, b)


def test_overflow_rows_take_global_path():
    """An arrow matrix (dense last row and column) gives the last row a
    frontier of 2,999 pivots, more than the LDS lists of either LDS tier
    hold; the row is rebuilt in global memory."""
    n = 3000
    M = np.zeros((n, n), bool)
    M[np.arange(n), np.arange(n)] = True
    M[-1, :] = True
    M[:, -1] = True
    rng = np.random.default_rng(9)
    vals = np.where(M, rng.uniform(-1, 1, (n, n)), 0.0)
    vals[np.arange(n), np.arange(n)] = 2.0 * n
    rows, cols = np.nonzero(M)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    A = I.CSR(n, np.cumsum(rp), cols.astype(np.int32), vals[rows, cols])
    pat, _, _ = _full(A, 2, rng.standard_normal(n))
    assert pat.info["overflow_rows"] >= 1
    # a 3000-entry row does not fit the dataflow kernel's LDS staging
    assert pat.info["flow_ready"] == 0
    ctx = T.context(0)
    ctx.set_numeric(ctx.NUMERIC_FLOW)
    with pytest.raises(T.TpiluError) as e:
        T.numeric(pat, g(A.val))
    assert e.value.status == T.E_INVAL
    ctx.set_numeric(0)


def test_long_range_fill_k_infinity():
    A = I.random_pattern(300, 0.01, seed=77)
    _full(A, 2**31 - 1, np.random.default_rng(3).standard_normal(A.n))


def test_empty_and_single():
    A0 = I.CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    pat = T.symbolic(g(A0.rowptr), torch.zeros(0, dtype=torch.int32, device="cuda:0"), 1)
    assert pat.nnz_f == 0
    A1 = I.CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([3.0]))
    _full(A1, 1, np.array([2.0]))


# ----------------------------------------------------------------------------------
# the named workloads at full size
# ----------------------------------------------------------------------------------
def _gmres_parity(pat, f, A, b, restart, maxit, rtol):
    rpF, ciF, vF = f[1]
    ref = O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, restart=restart, maxit=maxit, rtol=rtol)
    x, info = T.gmres(pat, g(A.val), f[0], g(b), restart=restart, maxit=maxit, rtol=rtol)
    assert info["iters"] == ref["iters"], (info["iters"], ref["iters"])
    assert_bits_equal(np.array(info["hist"]), ref["hist"], "GMRES |g| history")
    assert_bits_equal(x, ref["x"], "GMRES x")
    assert bits(np.array([info["relres"]]))[0] == bits(np.array([ref["relres"]]))[0]
    return info


def test_config1_conv_diff_2d_ilu1():
    c = I.conv_diff_2d_64x64_ilu1()
    pat, f, ref = _full(c["A"], c["k"], c["b"])
    info = _gmres_parity(pat, (f, ref), c["A"], c["b"], 30, 1000, 1e-8)
    assert info["relres"] <= 1e-8


def test_config2_random_banded_ilu2():
    c = I.random_banded_ilu2()
    log("  oracle + gpu on n=160000, ILU(2)")
    pat, f, ref = _full(c["A"], c["k"], c["b"])
    log(f"  pattern info {pat.info}")
    info = _gmres_parity(pat, (f, ref), c["A"], c["b"], 30, 300, 1e-8)
    assert info["relres"] <= 1e-8


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_config3_conv_diff_3d(k):
    c = I.conv_diff_3d_ilu(k=k)
    _full(c["A"], k, c["b"])


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_config3_gmres_and_bicgstab(k):
    """Sec. 4.2's 3-D convection-dominated problem at 64^3: GMRES(50) and
    BiCGSTAB (the paper's solver) with ILU(k), iterates bit for bit."""
    c = I.conv_diff_3d_ilu(k=k)
    A, b = c["A"], c["b"]
    pat, f, ref = _full(A, k, b)
    info = _gmres_parity(pat, (f, ref), A, b, 50, 3000, 1e-8)
    assert info["relres"] <= 1e-8
    rpF, ciF, vF = ref
    r = O.bicgstab(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, maxit=3000, rtol=1e-8)
    x, binfo = T.bicgstab(pat, g(A.val), f, g(b), maxit=3000, rtol=1e-8)
    assert binfo["iters"] == r["iters"] and binfo["status"] == r["status"] == 0, (binfo["iters"], r["iters"])
    assert_bits_equal(np.array(binfo["hist"]), r["hist"], "BiCGSTAB residual history")
    assert_bits_equal(x, r["x"], "BiCGSTAB x")


def test_levels_on_one_xcd():
    """The dependency levels computed on one XCD per graph (placement 2)
    give the same pattern, schedules and factor bits as device-wide."""
    c = I.random_banded_ilu2(n=20_000)
    A = c["A"]
    ctx = T.context(0)
    ref = T.numeric(T.symbolic(g(A.rowptr), g(A.col), 2), g(A.val))
    ctx.set_placement(ctx.PLACE_XCD)
    try:
        pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    finally:
        ctx.set_placement(0)
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, 2)
    check_pattern(pat, rpF, ciF, lvF, A)
    assert_bits_equal(T.numeric(pat, g(A.val)), ref, "F with levels from one XCD")


def test_repeatable_across_launch_shapes():
    """Same bits for any number of wavefronts (race check by repetition)."""
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    av, bv = g(A.val), g(c["b"])
    ctx = T.context(0)
    ref_f = T.numeric(pat, av)
    ref_y = T.apply(pat, ref_f, bv)
    for solver, place in ((ctx.SOLVER_DEVICE, ctx.PLACE_DEVICE), (ctx.SOLVER_DEVICE, ctx.PLACE_XCD),
                          (ctx.SOLVER_WORKGROUP, 0), (ctx.SOLVER_LANES, 0)):
        ctx.set_solver(solver)
        ctx.set_placement(place)
        for waves, group, tickets in ((1, 1, 8), (2, 3, 8), (7, 0, 3), (64, 64, 1), (1000, 2, 5), (0, 0, 0),
                                      (40000, 5, 8)):
            ctx.set_grid(waves)
            ctx.set_group(group)
            ctx.set_tickets(tickets)
            for _ in range(3):
                f = T.numeric(pat, av)
                y = T.apply(pat, f, bv)
                key = (solver, place, waves, group, tickets)
                assert torch.equal(f.view(torch.int64), ref_f.view(torch.int64)), key
                assert torch.equal(y.view(torch.int64), ref_y.view(torch.int64)), key
    ctx.set_grid(0)
    ctx.set_group(0)
    ctx.set_tickets(0)
    ctx.set_solver(0)
    ctx.set_placement(0)


@pytest.mark.parametrize("cfg", ["cd3d_k1", "s27_k1"])
def test_row_groups_agree_full_size(cfg):
    """Rows per ticket and task counters of the row kernels (numeric,
    wavefront-per-row solves, inverses): the oracle's bits for every setting."""
    c = I.conv_diff_3d_ilu(k=1) if cfg == "cd3d_k1" else I.stencil27_ilu(m=50, k=1)
    A, b, k = c["A"], c["b"], 1
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    x_ref, y_ref = O.apply(A.n, rpF, ciF, vF, b)
    vG = O.inverse(A.n, rpF, ciF, vF)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    ctx = T.context(0)
    modes = [ctx.NUMERIC_PIVOT] + ([ctx.NUMERIC_FLOW] if pat.info["flow_ready"] else [])
    try:
        ctx.set_solver(ctx.SOLVER_DEVICE)
        for group, tickets, place in ((1, 1, 1), (1, 8, 2), (2, 3, 1), (5, 8, 2), (8, 2, 1), (64, 8, 2)):
            ctx.set_placement(place)
            ctx.set_group(group)
            ctx.set_tickets(tickets)
            for mode in modes:
                ctx.set_numeric(mode)
                f = T.numeric(pat, g(A.val))
                assert_bits_equal(f, vF, f"F group {group} kernel {mode}")
            y, x = T.apply(pat, f, g(b), return_x=True)
            assert_bits_equal(x, x_ref, f"x group {group}")
            assert_bits_equal(y, y_ref, f"y group {group}")
            assert_bits_equal(T.inverse(pat, f), vG, f"G group {group}")
    finally:
        ctx.set_group(0)
        ctx.set_tickets(0)
        ctx.set_numeric(0)
        ctx.set_solver(0)
        ctx.set_placement(0)


@pytest.mark.parametrize("cfg", ["banded", "cd3d_k1"])
def test_solver_shapes_agree_full_size(cfg):
    """Every solve launch shape: same bits as the oracle."""
    c = I.random_banded_ilu2() if cfg == "banded" else I.conv_diff_3d_ilu(k=1)
    A, b = c["A"], c["b"]
    pat = T.symbolic(g(A.rowptr), g(A.col), c["k"])
    f = T.numeric(pat, g(A.val))
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, c["k"])
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    x_ref, y_ref = O.apply(A.n, rpF, ciF, vF, b)
    ctx = T.context(0)
    for solver, place in ((ctx.SOLVER_DEVICE, ctx.PLACE_DEVICE), (ctx.SOLVER_DEVICE, ctx.PLACE_XCD),
                          (ctx.SOLVER_WORKGROUP, 0), (ctx.SOLVER_LANES, 0)):
        ctx.set_solver(solver)
        ctx.set_placement(place)
        y, x = T.apply(pat, f, g(b), return_x=True)
        assert_bits_equal(x, x_ref, f"x solver {solver} placement {place}")
        assert_bits_equal(y, y_ref, f"y solver {solver} placement {place}")
    ctx.set_solver(0)
    ctx.set_placement(0)


def test_repeatable_random_banded():
    c = I.random_banded_ilu2()
    A = c["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    av = g(A.val)
    ref = T.numeric(pat, av)
    for _ in range(5):
        assert torch.equal(T.numeric(pat, av).view(torch.int64), ref.view(torch.int64))


# ----------------------------------------------------------------------------------
# failure handling (forced from the host)
# ----------------------------------------------------------------------------------
def test_zero_pivot_reported():
    rp = np.array([0, 2, 4], np.int64)
    ci = np.array([0, 1, 0, 1], np.int32)
    pat = T.symbolic(g(rp), g(ci), 1)
    with pytest.raises(T.ZeroPivotError) as e:
        T.numeric(pat, g(np.array([1.0, 1.0, 1.0, 1.0])))
    assert e.value.bad_row == 1
    vals = np.ones((4, 70))
    vals[0, 5] = 0.0  # instance 5: zero first pivot
    with pytest.raises(T.ZeroPivotError) as e:
        T.numeric(pat, g(vals))
    assert e.value.bad_row == 0
    f = T.numeric(pat, g(np.array([2.0, 1.0, 1.0, 1.0])))
    assert f.cpu().numpy()[3] == 0.5


def test_watchdog_times_out_and_recovers():
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 1)
    ctx = T.context(0)
    ctx.set_watchdog(timeout_us=20000, skip_publish_row=100)
    with pytest.raises(T.TpiluError) as e:
        T.numeric(pat, g(A.val))
    assert e.value.status == T.E_TIMEOUT
    ctx.set_watchdog(0, -1)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, 1)
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    assert_bits_equal(T.numeric(pat, g(A.val)), vF, "F after recovery")


def test_context_settings_reject_out_of_range():
    """Launch-shape settings outside their documented ranges are refused with
    E_INVAL and leave the previous setting in force."""
    ctx = T.context(0)
    for call, bad in ((ctx.set_group, (-1, 65)), (ctx.set_tickets, (-1, 9)), (ctx.set_solver, (-1, 4)),
                      (ctx.set_numeric, (-1, 3)), (ctx.set_placement, (-1, 3)), (ctx.set_grid, (-1,))):
        for v in bad:
            with pytest.raises(T.TpiluError) as e:
                call(v)
            assert e.value.status == T.E_INVAL, (call.__name__, v)
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat = T.symbolic(g(A.rowptr), g(A.col), c["k"])
    f = T.numeric(pat, g(A.val))
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, c["k"])
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    assert_bits_equal(f, vF, "F after refused settings")


def test_invalid_csr_rejected():
    with pytest.raises(T.TpiluError) as e:
        T.symbolic(g(np.array([0, 1, 2], np.int64)), g(np.array([0, 0], np.int32)), 1)  # no diag in row 1
    assert e.value.status == T.E_INVAL
    with pytest.raises(T.TpiluError):
        T.symbolic(g(np.array([0, 2, 3], np.int64)), g(np.array([1, 0, 1], np.int32)), 1)  # unsorted
    with pytest.raises(T.TpiluError):
        T.symbolic(g(np.array([0, 1, 2], np.int64)), g(np.array([0, 5], np.int32)), 1)  # out of range


def test_reserved_nan_input_rejected():
    A = I.random_pattern(50, 0.05, seed=1)
    pat = T.symbolic(g(A.rowptr), g(A.col), 1)
    v = A.val.copy()
    v.view(np.uint64)[3] = 0x7FF4A5A5A5A5A5A5
    with pytest.raises(T.TpiluError) as e:
        T.numeric(pat, g(v))
    assert e.value.status == T.E_INVAL
    # and the next call is clean again
    T.numeric(pat, g(A.val))


# ----------------------------------------------------------------------------------
# batched factorization under one graph
# ----------------------------------------------------------------------------------
def test_config4_batched_graph():
    c = I.batched_conv_diff_2d_ilu2()
    A, rhs = c["A"], c["b"]
    B = A.batch
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, 2)
    check_pattern(pat, rpF, ciF, lvF, A)
    av, bv = g(A.val), g(rhs)
    f_eager = T.numeric(pat, av)
    y_eager = T.apply(pat, f_eager, bv)
    fh, yh = f_eager.cpu().numpy(), y_eager.cpu().numpy()
    for inst in range(B):
        Ai = A.instance(inst)
        vF, bad = O.numeric(A.n, A.rowptr, A.col, Ai.val, rpF, ciF)
        _, yr = O.apply(A.n, rpF, ciF, vF, rhs[:, inst])
        assert_bits_equal(fh[:, inst], vF, f"F instance {inst}")
        assert_bits_equal(yh[:, inst], yr, f"y instance {inst}")
    # single-instance GPU runs of a few instances agree too
    for inst in (0, 63, 64, 255):
        fs = T.numeric(pat, g(A.val[:, inst].copy()))
        assert_bits_equal(fs, fh[:, inst], f"single vs batched {inst}")
    graph = T.BatchedGraph(pat, av, bv)
    for rep in range(3):
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(graph.f_val.view(torch.int64), f_eager.view(torch.int64)), rep
        assert torch.equal(graph.y.view(torch.int64), y_eager.view(torch.int64)), rep
        _ = T.numeric(pat, av)  # eager work between replays
    av.mul_(1.5)
    graph.launch()
    torch.cuda.synchronize()
    f2 = T.numeric(pat, av)
    assert torch.equal(graph.f_val.view(torch.int64), f2.view(torch.int64))
    assert not torch.equal(f2.view(torch.int64), f_eager.view(torch.int64))
    assert graph.check() == -1
    assert T.check(pat) == -1


def test_graph_owns_its_workspace():
    """A graph captured at 16 instances keeps working after eager calls on the
    same pattern regrow the pattern's own workspace (64 instances) and reuse
    its control block: the graph has its own intermediate vector and control
    block.  Every instance is compared with the oracle."""
    c = I.batched_conv_diff_2d_ilu2(B=64, m=24)
    A, rhs = c["A"], c["b"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, 2)
    a16 = g(np.ascontiguousarray(A.val[:, :16]))
    b16 = g(np.ascontiguousarray(rhs[:, :16]))
    graph = T.BatchedGraph(pat, a16, b16)
    graph.launch()
    assert graph.check() == -1
    # eager work at a larger batch on the same pattern (regrows its workspace)
    f64 = T.numeric(pat, g(A.val))
    y64 = T.apply(pat, f64, g(rhs))
    graph.launch()
    y64b = T.apply(pat, f64, g(rhs))  # eager work queued behind the launch
    assert graph.check() == -1
    f = graph.f_val.cpu().numpy()
    y = graph.y.cpu().numpy()
    for inst in range(16):
        vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val[:, inst].copy(), rpF, ciF)
        _, yr = O.apply(A.n, rpF, ciF, vF, rhs[:, inst])
        assert_bits_equal(f[:, inst], vF, f"graph F {inst}")
        assert_bits_equal(y[:, inst], yr, f"graph y {inst}")
    assert torch.equal(y64.view(torch.int64), y64b.view(torch.int64))
    assert_bits_equal(y64[:, :16], y, "eager vs graph")


@pytest.mark.parametrize("k,B", [(2, 70), (3, 5)])
def test_batched_long_rows(k, B):
    """Batches whose rows are longer than the batched kernel's LDS working row
    (27-point 20^3: 115 entries at ILU(2), 183 at ILU(3)) run with the
    working rows in global memory: every instance's F and y equal the
    oracle's, eagerly and under a captured graph (which owns its own working
    rows), and an instance run alone agrees."""
    c = I.batched_stencil27_ilu(B=B, k=k)
    A, rhs = c["A"], c["b"]
    log(f"{c['name']}")
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, k)
    check_pattern(pat, rpF, ciF, lvF, A)
    assert pat.info["max_row"] > 80
    av, bv = g(A.val), g(rhs)
    f = T.numeric(pat, av)
    y = T.apply(pat, f, bv)
    assert T.check(pat) == -1
    graph = T.BatchedGraph(pat, av, bv)
    graph.launch()
    assert graph.check() == -1
    fh, yh = f.cpu().numpy(), y.cpu().numpy()
    for inst in range(B):
        vF, bad = O.numeric(A.n, A.rowptr, A.col, A.val[:, inst].copy(), rpF, ciF)
        assert bad == -1
        _, yr = O.apply(A.n, rpF, ciF, vF, rhs[:, inst])
        assert_bits_equal(fh[:, inst], vF, f"F instance {inst}")
        assert_bits_equal(yh[:, inst], yr, f"y instance {inst}")
    assert torch.equal(graph.f_val.view(torch.int64), f.view(torch.int64))
    assert torch.equal(graph.y.view(torch.int64), y.view(torch.int64))
    fs = T.numeric(pat, g(A.val[:, B - 1].copy()))
    assert_bits_equal(fs, fh[:, B - 1], "single vs batched")


def _dominant_batch(A, B, rng):
    vals = rng.uniform(-1, 1, (A.nnz, B))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    rowsum = np.zeros((A.n, B))
    np.add.at(rowsum, rows, np.abs(vals))
    diag = A.col == rows
    vals[diag] = 1.1 * rowsum[rows[diag]] + 1.0
    return vals


@pytest.mark.parametrize("case", ["arrow", "full_lu"])
def test_batched_global_rows(case):
    """Rows too long for an LDS working row (over 80 entries for 64 instances)
    are factored with the working rows in global memory: an arrow matrix
    (600-entry last row, 599 pivots with 2 pairs each, B=70: two instance
    groups, the second partial) and the complete LU of a random pattern
    (k = n: rows of up to 381 entries whose pivots have hundreds of pairs, more than the
    pair lists hold).  Every instance's F equals the oracle's, eagerly and
    under a graph."""
    rng = np.random.default_rng(21)
    if case == "arrow":
        A, B, k = _arrow(600, 5), 70, 2
    else:
        A, B, k = I.random_pattern(400, 0.05, seed=31), 3, 400
    vals = _dominant_batch(A, B, rng)
    rhs = rng.standard_normal((A.n, B))
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    check_pattern(pat, rpF, ciF, lvF, A)
    assert pat.info["max_row"] > 80
    av, bv = g(vals), g(rhs)
    f = T.numeric(pat, av)
    y = T.apply(pat, f, bv)
    assert T.check(pat) == -1
    graph = T.BatchedGraph(pat, av, bv)
    graph.launch()
    assert graph.check() == -1
    fh, yh = f.cpu().numpy(), y.cpu().numpy()
    for inst in range(B):
        vF, bad = O.numeric(A.n, A.rowptr, A.col, vals[:, inst].copy(), rpF, ciF)
        assert bad == -1
        _, yr = O.apply(A.n, rpF, ciF, vF, rhs[:, inst])
        assert_bits_equal(fh[:, inst], vF, f"F instance {inst}")
        assert_bits_equal(yh[:, inst], yr, f"y instance {inst}")
    assert torch.equal(graph.f_val.view(torch.int64), f.view(torch.int64))
    assert torch.equal(graph.y.view(torch.int64), y.view(torch.int64))


@pytest.mark.parametrize("case", ["conv_diff_2d_ilu1", "banded_n6000_ilu2", "banded_n160000_ilu2"])
def test_fused_update_single(case):
    """The fused update (one rounding of f - l u in Eq. 6b): both
    single-instance kernels, on the whole device and on one XCD, against the
    oracle's fused elimination; the default mode is unchanged afterwards and
    differs from the fused one."""
    A, k = {"conv_diff_2d_ilu1": lambda: (I.conv_diff_2d_64x64_ilu1()["A"], 1),
            "banded_n6000_ilu2": lambda: (I.random_banded_ilu2(n=6000)["A"], 2),
            "banded_n160000_ilu2": lambda: (I.random_banded_ilu2()["A"], 2)}[case]()
    ctx = T.context(0)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, bad = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF, fused=True)
    v0, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    assert bad == -1
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    modes = [ctx.NUMERIC_PIVOT] + ([ctx.NUMERIC_FLOW] if pat.info["flow_ready"] else [])
    try:
        ctx.set_fused(True)
        for place in (ctx.PLACE_DEVICE, ctx.PLACE_XCD):
            ctx.set_placement(place)
            for mode in modes:
                ctx.set_numeric(mode)
                assert_bits_equal(T.numeric(pat, g(A.val), check=False), vF, f"fused F kernel {mode} place {place}")
                assert T.check(pat) == -1
    finally:
        ctx.set_fused(False)
        ctx.set_numeric(0)
        ctx.set_placement(0)
    assert_bits_equal(T.numeric(pat, g(A.val), check=False), v0, "default F after the fused runs")
    assert not np.array_equal(bits(vF), bits(v0))


@pytest.mark.parametrize("case", ["lds_rows", "global_rows"])
def test_fused_update_batched(case):
    """The fused update in the batched kernels (working rows in LDS and in
    global memory), eagerly and in a graph created in fused mode (which
    keeps it for its launches): every instance against the oracle."""
    rng = np.random.default_rng(44)
    if case == "lds_rows":
        c = I.batched_conv_diff_2d_ilu2(B=70, m=24)
        A, k, vals, rhs = c["A"], 2, c["A"].val, c["b"]
        B = A.batch
    else:
        A, B, k = _arrow(600, 5), 66, 2
        vals = _dominant_batch(A, B, rng)
        rhs = rng.standard_normal((A.n, B))
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    av, bv = g(vals), g(rhs)
    ctx = T.context(0)
    try:
        ctx.set_fused(True)
        f = T.numeric(pat, av)
        y = T.apply(pat, f, bv)
        graph = T.BatchedGraph(pat, av, bv)
    finally:
        ctx.set_fused(False)
    graph.launch()
    torch.cuda.synchronize()
    assert graph.check() == -1
    fh, yh = f.cpu().numpy(), y.cpu().numpy()
    for inst in range(B):
        vF, bad = O.numeric(A.n, A.rowptr, A.col, np.ascontiguousarray(vals[:, inst]), rpF, ciF, fused=True)
        assert bad == -1
        _, yr = O.apply(A.n, rpF, ciF, vF, np.ascontiguousarray(rhs[:, inst]))
        assert_bits_equal(fh[:, inst], vF, f"fused F instance {inst}")
        assert_bits_equal(yh[:, inst], yr, f"fused y instance {inst}")
    assert torch.equal(graph.f_val.view(torch.int64), f.view(torch.int64))
    assert torch.equal(graph.y.view(torch.int64), y.view(torch.int64))
    f0 = T.numeric(pat, av)
    assert not torch.equal(f0.view(torch.int64), f.view(torch.int64))


def test_batched_partial_group():
    """A batch that is not a multiple of 64 instances."""
    c = I.batched_conv_diff_2d_ilu2(B=70, m=24)
    A, rhs = c["A"], c["b"]
    pat = T.symbolic(g(A.rowptr), g(A.col), 2)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, 2)
    f = T.numeric(pat, g(A.val)).cpu().numpy()
    y = T.apply(pat, g(f), g(rhs)).cpu().numpy()
    for inst in (0, 63, 64, 69):
        vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val[:, inst].copy(), rpF, ciF)
        assert_bits_equal(f[:, inst], vF, f"F {inst}")
        assert_bits_equal(y[:, inst], O.apply(A.n, rpF, ciF, vF, rhs[:, inst])[1], f"y {inst}")


# ----------------------------------------------------------------------------------
# reverse mode
# ----------------------------------------------------------------------------------
def _oracle_grads(A, rpF, ciF, vals, b, t):
    vF, _ = O.numeric(A.n, A.rowptr, A.col, vals, rpF, ciF)
    x, y = O.apply(A.n, rpF, ciF, vF, b)
    bbar, Fbar = O.apply_adjoint(A.n, rpF, ciF, vF, x, y, 2.0 * (y - t))
    abar, _ = O.numeric_adjoint(A.n, A.rowptr, A.col, rpF, ciF, vF, Fbar)
    return abar, bbar, Fbar


def test_adjoint_small_bits():
    rng = np.random.default_rng(11)
    for case in range(12):
        n = int(rng.integers(2, 300))
        A = I.random_pattern(n, float(rng.choice([0.01, 0.04])), seed=int(rng.integers(1 << 30)))
        k = int(rng.choice([0, 1, 2]))
        b, t = rng.standard_normal(n), rng.standard_normal(n)
        rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
        abar_r, bbar_r, Fbar_r = _oracle_grads(A, rpF, ciF, A.val, b, t)
        pat = T.symbolic(g(A.rowptr), g(A.col), k)
        f = T.numeric(pat, g(A.val))
        y, x = T.apply(pat, f, g(b), return_x=True)
        ctx = T.context(0)
        try:
            for place in (ctx.PLACE_AUTO, ctx.PLACE_DEVICE, ctx.PLACE_XCD):
                ctx.set_placement(place)
                bbar, fbar = T.apply_adjoint(pat, f, x, y, 2.0 * (y - g(t)))
                assert_bits_equal(bbar, bbar_r, f"bbar placement {place}")
                assert_bits_equal(fbar, Fbar_r, f"Fbar placement {place}")
        finally:
            ctx.set_placement(0)
        abar, _ = T.numeric_adjoint(pat, f, fbar)
        assert_bits_equal(abar, abar_r, "abar")


def test_adjoint_random_banded_bits():
    """Transposed solves of one instance at full size (narrow graph: one XCD
    by default) against the sequential adjoint, on both placements."""
    c = I.random_banded_ilu2()
    A, b = c["A"], c["b"]
    t = np.random.default_rng(21).standard_normal(A.n)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, c["k"])
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    x_r, y_r = O.apply(A.n, rpF, ciF, vF, b)
    bbar_r, Fbar_r = O.apply_adjoint(A.n, rpF, ciF, vF, x_r, y_r, 2.0 * (y_r - t))
    pat = T.symbolic(g(A.rowptr), g(A.col), c["k"])
    f = T.numeric(pat, g(A.val))
    y, x = T.apply(pat, f, g(b), return_x=True)
    ctx = T.context(0)
    try:
        for place in (ctx.PLACE_AUTO, ctx.PLACE_DEVICE, ctx.PLACE_XCD):
            ctx.set_placement(place)
            bbar, fbar = T.apply_adjoint(pat, f, x, y, 2.0 * (y - g(t)))
            assert_bits_equal(bbar, bbar_r, f"bbar placement {place}")
            assert_bits_equal(fbar, Fbar_r, f"Fbar placement {place}")
    finally:
        ctx.set_placement(0)


def _arrow(n, seed):
    M = np.zeros((n, n), bool)
    M[np.arange(n), np.arange(n)] = True
    M[-1, :] = True
    M[:, -1] = True
    M[np.arange(1, n), np.arange(n - 1)] = True
    rows, cols = np.nonzero(M)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return I.CSR(n, np.cumsum(rp), cols.astype(np.int32), np.zeros(rows.size))


@pytest.mark.parametrize("case", ["groups", "long_rows"])
def test_adjoint_batched_bits(case):
    """Reverse mode on batches: every instance equals its own sequential
    adjoint, with partial instance groups (B=70) and with rows too long for
    the lanes-as-instances reverse sweep (B=3, 150-entry row)."""
    rng = np.random.default_rng(12)
    if case == "groups":
        A = I.random_pattern(240, 0.02, seed=99)
        B, k = 70, 2
    else:
        A = _arrow(150, 5)
        B, k = 3, 1
    vals = rng.uniform(-1, 1, (A.nnz, B))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    diag = A.col == rows
    rowsum = np.zeros((A.n, B))
    np.add.at(rowsum, rows, np.abs(vals))
    vals[diag] = 1.1 * rowsum + 1.0  # diagonally dominant: no zero pivots
    rhs, tgt = rng.standard_normal((A.n, B)), rng.standard_normal((A.n, B))
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(vals))
    # the batched factors equal the single-instance ones
    for i in range(B):
        assert_bits_equal(f[:, i].contiguous(), T.numeric(pat, g(vals[:, i].copy())), f"instance {i}")
    y, x = T.apply(pat, f, g(rhs), return_x=True)
    bbar, fbar = T.apply_adjoint(pat, f, x, y, 2.0 * (y - g(tgt)))
    abar, _ = T.numeric_adjoint(pat, f, fbar.clone())
    for inst in sorted({0, 1, B // 2, B - 1}):
        abar_r, bbar_r, Fbar_r = _oracle_grads(A, rpF, ciF, vals[:, inst].copy(), rhs[:, inst], tgt[:, inst])
        assert_bits_equal(bbar[:, inst], bbar_r, f"bbar instance {inst}")
        assert_bits_equal(fbar[:, inst], Fbar_r, f"Fbar instance {inst}")
        assert_bits_equal(abar[:, inst], abar_r, f"abar instance {inst}")


def test_config5_autograd_against_oracle_and_fd():
    c = I.differentiated_conv_diff_3d_ilu1()
    A, rhs, tgt = c["A"], c["b"], c["t"]
    B = A.batch
    pat = T.symbolic(g(A.rowptr), g(A.col), 1)
    av = g(A.val).requires_grad_(True)
    bv = g(rhs).requires_grad_(True)
    y = T.ILUApply.apply(av, bv, pat)
    loss = ((y - g(tgt)) ** 2).sum()
    loss.backward()
    ga, gb = av.grad.cpu().numpy(), bv.grad.cpu().numpy()
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, 1)
    for inst in range(B):
        abar_r, bbar_r, _ = _oracle_grads(A, rpF, ciF, A.val[:, inst].copy(), rhs[:, inst], tgt[:, inst])
        assert_bits_equal(ga[:, inst], abar_r, f"d/dA instance {inst}")
        assert_bits_equal(gb[:, inst], bbar_r, f"d/db instance {inst}")
    # central finite differences on 64 sampled (instance, entry) pairs; the
    # loss difference is formed per element, (y+ - y-)(y+ + y- - 2t), so the
    # large loss itself never cancels
    rng = np.random.default_rng(5)
    eps = 1e-6

    def y_of(vals, inst):
        vF, _ = O.numeric(A.n, A.rowptr, A.col, vals, rpF, ciF)
        return O.apply(A.n, rpF, ciF, vF, rhs[:, inst])[1]

    scale = np.abs(ga).max()
    import math

    for _ in range(64):
        inst = int(rng.integers(B))
        p = int(rng.integers(A.nnz))
        vp = A.val[:, inst].copy()
        vm = vp.copy()
        vp[p] += eps
        vm[p] -= eps
        yp, ym = y_of(vp, inst), y_of(vm, inst)
        fd = math.fsum((yp - ym) * (yp + ym - 2.0 * tgt[:, inst])) / (vp[p] - vm[p])
        assert abs(fd - ga[p, inst]) <= 1e-5 * max(abs(fd), 1e-9 * scale) + 1e-9 * scale, (inst, p, fd, ga[p, inst])


# ----------------------------------------------------------------------------------
# level-based incomplete inverses (Sec. 3.5)
# ----------------------------------------------------------------------------------
def _inverse_parity(A, k, b, waves=0):
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    vG = O.inverse(A.n, rpF, ciF, vF)
    x_ref, y_ref = O.apply_inverse(A.n, rpF, ciF, vG, b)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(A.val), check=False)
    assert_bits_equal(f, vF, "F")
    ctx = T.context(0)
    ctx.set_grid(waves)
    try:
        G = T.inverse(pat, f)
    finally:
        ctx.set_grid(0)
    assert_bits_equal(G, vG, "G")
    # both shapes of the two products (wavefront per row, thread per row)
    for solver in (ctx.SOLVER_DEVICE, ctx.SOLVER_LANES, 0):
        ctx.set_solver(solver)
        try:
            y, x = T.apply_inverse(pat, G, g(b), return_x=True)
        finally:
            ctx.set_solver(0)
        assert_bits_equal(x, x_ref, "x = L~~^-1 b")
        assert_bits_equal(y, y_ref, "y = U~~^-1 x")
    return pat, f, G, (rpF, ciF, vF, vG)


def test_inverse_small_sweep():
    rng = np.random.default_rng(21)
    for case in range(40):
        n = int(rng.integers(1, 300))
        A = I.random_pattern(n, float(rng.choice([0.005, 0.02, 0.06])), seed=int(rng.integers(1 << 30)),
                             diag_dominant=bool(rng.integers(2)))
        if case % 7 == 0 and A.nnz > 3:
            A.val[1] = -0.0
        k = int(rng.choice([0, 1, 2, 3, n]))
        _inverse_parity(A, k, rng.standard_normal(n), waves=int(rng.choice([0, 1, 5, 64])))


@pytest.mark.parametrize("cfg", ["cd2d", "cd3d_k1", "cd3d_k2"])
def test_inverse_stencils(cfg):
    c = I.conv_diff_2d_64x64_ilu1() if cfg == "cd2d" else I.conv_diff_3d_ilu(k=int(cfg[-1]))
    _inverse_parity(c["A"], c["k"] if cfg == "cd2d" else int(cfg[-1]), c["b"])


def test_inverse_config2_full_size():
    c = I.random_banded_ilu2()
    _inverse_parity(c["A"], c["k"], c["b"])


def test_gmres_inverse_bits():
    c = I.conv_diff_2d_64x64_ilu1()
    A = c["A"]
    pat, f, G, (rpF, ciF, vF, vG) = _inverse_parity(A, 1, c["b"])
    ref = O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vG, c["b"], restart=30, maxit=400, rtol=1e-8,
                  inverse=True)
    x, info = T.gmres(pat, g(A.val), G, g(c["b"]), restart=30, maxit=400, rtol=1e-8, inverse=True)
    assert info["iters"] == ref["iters"]
    assert_bits_equal(np.array(info["hist"]), ref["hist"], "GMRES |g| history (inverse)")
    assert_bits_equal(x, ref["x"], "GMRES x (inverse)")


# ----------------------------------------------------------------------------------
# BiCGSTAB (Sec. 4's Krylov method)
# ----------------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["cd2d_ilu", "cd2d_inverse", "cd3dk1_ilu", "banded_ilu", "banded_inverse"])
def test_bicgstab_bits(case):
    name, prec = case.split("_")
    make = {"cd2d": I.conv_diff_2d_64x64_ilu1, "cd3dk1": lambda: I.conv_diff_3d_ilu(k=1),
            "banded": I.random_banded_ilu2}
    c = make[name]()
    A, k = c["A"], (1 if name != "banded" else c["k"])
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    pat = T.symbolic(g(A.rowptr), g(A.col), k)
    f = T.numeric(pat, g(A.val))
    inv = prec == "inverse"
    if inv:
        vM = O.inverse(A.n, rpF, ciF, vF)
        M = T.inverse(pat, f)
    else:
        vM, M = vF, f
    maxit = 200
    ref = O.bicgstab(A.n, A.rowptr, A.col, A.val, rpF, ciF, vM, c["b"], maxit=maxit, rtol=1e-8, inverse=inv)
    x, info = T.bicgstab(pat, g(A.val), M, g(c["b"]), maxit=maxit, rtol=1e-8, inverse=inv)
    assert info["iters"] == ref["iters"], (info["iters"], ref["iters"])
    assert info["status"] == ref["status"]
    assert_bits_equal(np.array(info["hist"]), ref["hist"], "BiCGSTAB residual history")
    assert_bits_equal(x, ref["x"], "BiCGSTAB x")
    assert bits(np.array([info["relres"]]))[0] == bits(np.array([ref["relres"]]))[0]


# ----------------------------------------------------------------------------------
# 27-point 3-D stencil (Sec. 4.2's problem), k = 0..3
# ----------------------------------------------------------------------------------
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_stencil27_small(k):
    c = I.stencil27_ilu(m=12, k=k)
    pat, f, ref = _full(c["A"], k, c["b"])
    if k == 1:
        _gmres_parity(pat, (f, ref), c["A"], c["b"], 50, 200, 1e-8)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_stencil27_50cubed(k):
    """At the paper's smallest size (50^3 = 125,000 rows): pattern, factor and
    both solves bit for bit."""
    c = I.stencil27_ilu(m=50, k=k)
    _full(c["A"], k, c["b"])


def test_stencil27_90cubed_ilu1():
    """The largest 27-point size the benchmark runs (90^3 = 729,000 rows,
    4.4 x 10^7 entries of F, lane-per-row solves): pattern, factor and both
    solves bit for bit."""
    c = I.stencil27_ilu(m=90, k=1)
    _full(c["A"], 1, c["b"])


# ----------------------------------------------------------------------------------
# Paper-scale ILU(1) (Table 3's general sparse matrices, about 1,250 entries per row
# of F): long rows through the larger symbolic maps and the pivot-serial kernel
# ----------------------------------------------------------------------------------
PAPER_ROW = 9_832_794 / 160_000  # entries per row of A in Table 3's 160K matrix


def test_paper_scale_rows_small_bits():
    """Rows of the paper's length (~1,000 entries of F, up to ~1,550) on a
    3,000-row matrix: pattern, factor and both solves bit for bit."""
    c = I.paper_scale_random_ilu1(n=3000, per_row=PAPER_ROW)
    pat, _, _ = _full(c["A"], 1, c["b"])
    assert pat.info["long_rows"] > 0


def test_paper_scale_160k_all_rows():
    """Table 3's 160K size at full scale (about 2 x 10^8 entries of F): every
    row's pattern, levels and factor values and both solves, against the
    digests the oracle wrote (tests/golden/paper_scale_ilu1_digests.py), per
    block of 1,000 rows."""
    from tests.golden.paper_scale_ilu1_digests import block_digests, read_digests

    meta, want = read_digests()
    c = I.paper_scale_random_ilu1()
    A = c["A"]
    assert int(meta["n"]) == A.n and int(meta["nnz_a"]) == A.nnz
    pat = T.symbolic(g(A.rowptr), g(A.col), 1)
    info = pat.info
    log(f"[gpu] paper-scale 160K: nnz_f {info['nnz_f']} long rows {info['long_rows']} "
        f"overflow {info['overflow_rows']} depth {info['depth_l']}")
    assert info["nnz_f"] == int(meta["nnz_f"])
    f = T.numeric(pat, g(A.val))
    y, x = T.apply(pat, f, g(c["b"]), return_x=True)
    ex = pat.export()
    got = block_digests(ex["rowptr"].cpu().numpy(), ex["col"].cpu().numpy(), ex["level"].cpu().numpy(),
                        f.cpu().numpy(), x.cpu().numpy(), y.cpu().numpy())
    assert len(got) == len(want)
    what = ("pattern", "factor", "x", "y")
    bad = [(w[0], what[q]) for w, h in zip(want, got) for q in range(4) if w[2 + q] != h[2 + q]]
    assert not bad, f"{len(bad)} mismatching (first row of block, part): {bad[:10]}"
