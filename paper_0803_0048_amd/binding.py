"""Python binding of the gfx950 ILU(k) library (``libtpilu.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/tpilu.h``.  PyTorch provides
device memory and the current HIP stream.  There is no CPU fallback: if the
library is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# TPILU_LIBRARY=jitter selects the race check build (libtpilu_jitter.so, same
# kernels with random pauses at every hand-off), which only a test uses
LIB_PATH = os.path.join(HERE, "libtpilu_jitter.so" if os.environ.get("TPILU_LIBRARY") == "jitter" else "libtpilu.so")

OK, E_INVAL, E_NOMEM, E_ZEROPIVOT, E_DEVICE, E_NOTCONV, E_TIMEOUT = range(7)

EXPORTED = [
    "tpilu_ctx_create", "tpilu_ctx_set_stream", "tpilu_ctx_destroy", "tpilu_status_string",
    "tpilu_last_error", "tpilu_ctx_set_watchdog", "tpilu_ctx_set_grid", "tpilu_ctx_set_solver", "tpilu_ctx_set_numeric", "tpilu_ctx_set_fused", "tpilu_ctx_set_placement", "tpilu_ctx_set_group", "tpilu_ctx_set_tickets", "tpilu_inverse", "tpilu_apply_inverse", "tpilu_gmres_inverse", "tpilu_bicgstab", "tpilu_ctx_set_trace", "tpilu_ctx_set_timing", "tpilu_ctx_read_timing", "tpilu_symbolic", "tpilu_pattern_info",
    "tpilu_pattern_export", "tpilu_pattern_destroy", "tpilu_numeric", "tpilu_pattern_check",
    "tpilu_apply", "tpilu_gmres", "tpilu_spmv", "tpilu_dot", "tpilu_apply_adjoint",
    "tpilu_numeric_adjoint", "tpilu_batched_graph_create", "tpilu_batched_graph_launch",
    "tpilu_batched_graph_check", "tpilu_batched_graph_destroy", "tpilu_apply_noalloc", "tpilu_givens",
    "tpilu_numeric_critical_path", "tpilu_handoff_probe",
]


class TpiluError(RuntimeError):
    def __init__(self, status: int, message: str, bad_row: int = -1):
        super().__init__(f"[status {status}] {message}")
        self.status = status
        self.bad_row = bad_row


class ZeroPivotError(TpiluError):
    pass


class PatternInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_f", C.c_int64), ("nnz_l", C.c_int64),
                ("nnz_u", C.c_int64), ("n_updates", C.c_int64), ("k", C.c_int32),
                ("max_row", C.c_int32), ("max_lrow", C.c_int32), ("depth_l", C.c_int32),
                ("depth_u", C.c_int32), ("overflow_rows", C.c_int32), ("flow_ready", C.c_int32),
                ("long_rows", C.c_int32)]


_lib = None
_lock = threading.Lock()


def load_library():
    """Load libtpilu.so (after torch, so that it binds to torch's HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_0803_0048_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        st = C.c_int
        sig = {
            "tpilu_ctx_create": ([C.c_int, P, P, P, P, C.POINTER(P)], st),
            "tpilu_ctx_set_stream": ([P, P], st),
            "tpilu_ctx_destroy": ([P], None),
            "tpilu_status_string": ([st], C.c_char_p),
            "tpilu_last_error": ([P], C.c_char_p),
            "tpilu_ctx_set_watchdog": ([P, u32, i64], st),
            "tpilu_ctx_set_grid": ([P, i32], st),
            "tpilu_ctx_set_solver": ([P, C.c_int], st),
            "tpilu_ctx_set_numeric": ([P, C.c_int], st),
            "tpilu_ctx_set_fused": ([P, C.c_int], st),
            "tpilu_ctx_set_placement": ([P, C.c_int], st),
            "tpilu_ctx_set_group": ([P, C.c_int32], st),
            "tpilu_ctx_set_tickets": ([P, C.c_int32], st),
            "tpilu_ctx_set_trace": ([P, P], st),
            "tpilu_ctx_set_timing": ([P, C.c_int], st),
            "tpilu_ctx_read_timing": ([P, C.c_int, C.POINTER(dbl), C.POINTER(i64)], st),
            "tpilu_symbolic": ([P, i64, i64, P, P, i32, C.POINTER(P)], st),
            "tpilu_pattern_info": ([P, C.POINTER(PatternInfo)], st),
            "tpilu_pattern_export": ([P, P, P, P, P, P, P], st),
            "tpilu_pattern_destroy": ([P], None),
            "tpilu_numeric": ([P, P, P, i32, P, C.POINTER(i64)], st),
            "tpilu_pattern_check": ([P, P, C.POINTER(i64)], st),
            "tpilu_apply": ([P, P, P, i32, P, P, P], st),
            "tpilu_apply_noalloc": ([P, P, P, i32, P, P], st),
            "tpilu_gmres": ([P, P, P, P, P, P, i32, i32, dbl, C.POINTER(i32), C.POINTER(dbl), P], st),
            "tpilu_gmres_inverse": ([P, P, P, P, P, P, i32, i32, dbl, C.POINTER(i32), C.POINTER(dbl), P], st),
            "tpilu_inverse": ([P, P, P, i32, P], st),
            "tpilu_bicgstab": ([P, P, P, P, i32, P, P, i32, dbl, C.POINTER(i32), C.POINTER(dbl), P], st),
            "tpilu_apply_inverse": ([P, P, P, i32, P, P, P], st),
            "tpilu_spmv": ([P, P, P, P, P], st),
            "tpilu_dot": ([P, i64, P, P, C.POINTER(dbl)], st),
            "tpilu_givens": ([P, i64, P, P, P, P, P], st),
            "tpilu_numeric_critical_path": ([P, P, dbl, dbl, C.POINTER(dbl)], st),
            "tpilu_handoff_probe": ([P, i32, i32, C.POINTER(dbl)], st),
            "tpilu_apply_adjoint": ([P, P, P, i32, P, P, P, P, P], st),
            "tpilu_numeric_adjoint": ([P, P, P, i32, P, P], st),
            "tpilu_batched_graph_create": ([P, P, P, i32, P, P, P, C.POINTER(P)], st),
            "tpilu_batched_graph_launch": ([P, P], st),
            "tpilu_batched_graph_check": ([P, P, C.POINTER(i64)], st),
            "tpilu_batched_graph_destroy": ([P], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
        return L


# ----------------------------------------------------------------------------------
# context per device
# ----------------------------------------------------------------------------------
_ctxs: dict[int, "Context"] = {}


class Context:
    def __init__(self, device: int):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the ILU(k) library runs on the GPU only")
        self.device = device
        h = C.c_void_p()
        st = lib.tpilu_ctx_create(device, None, None, None, None, C.byref(h))
        if st != OK:
            raise TpiluError(st, "tpilu_ctx_create failed")
        self.h = h

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        load_library().tpilu_ctx_set_stream(self.h, C.c_void_p(s))

    def check(self, st: int, what: str, bad_row: int = -1):
        if st == OK:
            return
        msg = load_library().tpilu_last_error(self.h).decode(errors="replace")
        if st == E_ZEROPIVOT:
            raise ZeroPivotError(st, f"{what}: {msg}", bad_row)
        raise TpiluError(st, f"{what}: {msg}", bad_row)

    KERNEL_NUMERIC, KERNEL_FORWARD, KERNEL_BACKWARD = 0, 1, 2

    def set_timing(self, on: bool):
        self.check(load_library().tpilu_ctx_set_timing(self.h, 1 if on else 0), "set_timing")

    def read_timing(self, kernel: int):
        """(total ms, launches) of one kernel kind since the last read."""
        ms = C.c_double(0.0)
        cnt = C.c_int64(0)
        self.check(load_library().tpilu_ctx_read_timing(self.h, kernel, C.byref(ms), C.byref(cnt)), "read_timing")
        return ms.value, cnt.value

    SOLVER_AUTO, SOLVER_DEVICE, SOLVER_WORKGROUP, SOLVER_LANES = 0, 1, 2, 3

    def set_solver(self, mode: int = 0):
        self.check(load_library().tpilu_ctx_set_solver(self.h, mode), "set_solver")

    NUMERIC_AUTO, NUMERIC_FLOW, NUMERIC_PIVOT = 0, 1, 2

    def set_numeric(self, mode: int = 0):
        """Kernel of the single-instance numeric factorization (same bits in
        every mode): 0 automatic, 1 dataflow, 2 pivot-serial."""
        self.check(load_library().tpilu_ctx_set_numeric(self.h, mode), "set_numeric")

    def set_fused(self, on: bool = False):
        """Update of the numeric factorization (Eq. 6b): False rounds the
        product and the difference on their own, True rounds the exact
        f - l * u once (fused multiply-add)."""
        self.check(load_library().tpilu_ctx_set_fused(self.h, int(bool(on))), "set_fused")

    PLACE_AUTO, PLACE_DEVICE, PLACE_XCD = 0, 1, 2

    def set_placement(self, where: int = 0):
        """Where the single-instance numeric kernels, wavefront-per-row
        solves and single-instance transposed solves run (same bits
        everywhere): 0 automatic, 1 whole device, 2 one XCD."""
        self.check(load_library().tpilu_ctx_set_placement(self.h, where), "set_placement")

    def set_group(self, rows: int = 0):
        """Level-order rows per ticket of the wavefront-per-row kernels
        (0 automatic, else 1..64); same bits for every value."""
        self.check(load_library().tpilu_ctx_set_group(self.h, rows), "set_group")

    def set_tickets(self, counters: int = 0):
        """Task counters of the wavefront-per-row kernels (0 automatic, else
        1..8); same bits for every value."""
        self.check(load_library().tpilu_ctx_set_tickets(self.h, counters), "set_tickets")

    def set_trace(self, buf=None):
        """Per-row timeline: a uint64/int64 device tensor of 4n entries, or None."""
        self.check(load_library().tpilu_ctx_set_trace(self.h, _ptr(buf)), "set_trace")

    def set_grid(self, waves: int = 0):
        self.check(load_library().tpilu_ctx_set_grid(self.h, waves), "set_grid")

    def set_watchdog(self, timeout_us: int = 0, skip_publish_row: int = -1):
        self.check(load_library().tpilu_ctx_set_watchdog(self.h, timeout_us, skip_publish_row),
                   "set_watchdog")


def context(device=None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    c = _ctxs.get(device)
    if c is None:
        c = Context(device)
        _ctxs[device] = c
    c.bind_stream()
    return c


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _need_size(t, dtype, name, device, lead, batch=1):
    """_need plus the shape the kernels will index: [lead] for one instance,
    [lead, batch] for a batch (entry-major, instance-minor)."""
    _need(t, dtype, name, device)
    want = (lead,) if batch == 1 and t.dim() == 1 else (lead, batch)
    if tuple(t.shape) != want:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
    return t


# ----------------------------------------------------------------------------------
# pattern (Phase I)
# ----------------------------------------------------------------------------------
class Pattern:
    """Level-of-fill pattern of F for one CSR structure and level k."""

    def __init__(self, handle, ctx: Context, device: torch.device):
        self.h = handle
        self.ctx = ctx
        self.device = device
        info = PatternInfo()
        load_library().tpilu_pattern_info(self.h, C.byref(info))
        self.info = {f: getattr(info, f) for f, _ in PatternInfo._fields_}
        self.n = info.n
        self.nnz_a = info.nnz_a
        self.nnz_f = info.nnz_f

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            _lib.tpilu_pattern_destroy(h)
            self.h = None

    def export(self):
        """Pattern arrays as device tensors: rowptr, col, diag, level, a2f."""
        ctx = context(self.device)
        d = self.device
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=d)
        ci = torch.empty(max(self.nnz_f, 1), dtype=torch.int32, device=d)
        dg = torch.empty(max(self.n, 1), dtype=torch.int32, device=d)
        lv = torch.empty(max(self.nnz_f, 1), dtype=torch.uint8, device=d)
        a2f = torch.empty(max(self.nnz_a, 1), dtype=torch.int32, device=d)
        st = load_library().tpilu_pattern_export(ctx.h, self.h, _ptr(rp), _ptr(ci), _ptr(dg), _ptr(lv), _ptr(a2f))
        ctx.check(st, "pattern_export")
        return {"rowptr": rp, "col": ci[: self.nnz_f], "diag": dg[: self.n], "level": lv[: self.nnz_f],
                "a2f": a2f[: self.nnz_a]}


def symbolic(rowptr: torch.Tensor, col: torch.Tensor, k: int, n: int | None = None) -> Pattern:
    """Phase I (Algorithm 1): pattern of every entry of level <= k."""
    d = rowptr.device
    _need(rowptr, torch.int64, "rowptr", None)
    _need(col, torch.int32, "col", d)
    n = rowptr.numel() - 1 if n is None else n
    ctx = context(d)
    h = C.c_void_p()
    st = load_library().tpilu_symbolic(ctx.h, n, col.numel(), _ptr(rowptr), _ptr(col), int(min(k, 2**31 - 1)),
                                       C.byref(h))
    ctx.check(st, "symbolic")
    return Pattern(h, ctx, d)


def _batch_of(t: torch.Tensor, lead: int, name: str) -> int:
    if t.dim() == 1:
        if t.shape[0] != lead:
            raise ValueError(f"{name} has {t.shape[0]} entries, expected {lead}")
        return 1
    if t.dim() == 2 and t.shape[0] == lead:
        return t.shape[1]
    raise ValueError(f"{name} must have shape [{lead}] or [{lead}, batch]")


def numeric(pat: Pattern, a_val: torch.Tensor, out: torch.Tensor | None = None, check: bool = True):
    """Phase II (Eqs. 6a/6b): F values, shape [nnz_f] or [nnz_f, batch]."""
    _need(a_val, torch.float64, "a_val", pat.device)
    B = _batch_of(a_val, pat.nnz_a, "a_val")
    shape = (pat.nnz_f,) if a_val.dim() == 1 else (pat.nnz_f, B)
    if out is None:
        f = torch.empty(shape, dtype=torch.float64, device=pat.device)
    else:
        f = _need(out, torch.float64, "out", pat.device)
        if tuple(f.shape) != shape:
            raise ValueError(f"out has shape {tuple(f.shape)}, expected {shape}")
    ctx = context(pat.device)
    bad = C.c_int64(-1)
    st = load_library().tpilu_numeric(ctx.h, pat.h, _ptr(a_val), B, _ptr(f), C.byref(bad) if check else None)
    ctx.check(st, "numeric", bad.value)
    return f


def check(pat: Pattern) -> int:
    """Wait and report the sticky device status of the last calls; returns bad_row or -1."""
    ctx = context(pat.device)
    bad = C.c_int64(-1)
    st = load_library().tpilu_pattern_check(ctx.h, pat.h, C.byref(bad))
    ctx.check(st, "check", bad.value)
    return bad.value


def apply(pat: Pattern, f_val: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
          return_x: bool = False):
    """y = U~^-1 L~^-1 b (Eq. 1)."""
    _need(f_val, torch.float64, "f_val", pat.device)
    _need(b, torch.float64, "b", pat.device)
    B = _batch_of(b, pat.n, "b")
    if _batch_of(f_val, pat.nnz_f, "f_val") != B or f_val.dim() != b.dim():
        raise ValueError("f_val and b batch sizes differ")
    y = torch.empty_like(b) if out is None else _need_size(out, torch.float64, "out", pat.device, pat.n, B)
    if out is not None and (out.dim() != b.dim() or out.data_ptr() == b.data_ptr()):
        raise ValueError("out must be shaped like b and must not be b")
    x = torch.empty_like(b) if return_x else None
    ctx = context(pat.device)
    st = load_library().tpilu_apply(ctx.h, pat.h, _ptr(f_val), B, _ptr(b), _ptr(y), _ptr(x))
    ctx.check(st, "apply")
    return (y, x) if return_x else y


def apply_noalloc(pat: Pattern, f_val: torch.Tensor, b: torch.Tensor, y: torch.Tensor):
    """y = U~^-1 L~^-1 b into the caller's y, with the library allocating
    nothing (its intermediate vector lives in a fixed 32 MiB device scratch;
    n * batch must be at most 4,194,304).  Calls on one device must not
    overlap."""
    _need(f_val, torch.float64, "f_val", pat.device)
    _need(b, torch.float64, "b", pat.device)
    B = _batch_of(b, pat.n, "b")
    if _batch_of(f_val, pat.nnz_f, "f_val") != B or f_val.dim() != b.dim():
        raise ValueError("f_val and b batch sizes differ")
    _need_size(y, torch.float64, "y", pat.device, pat.n, B)
    if y.dim() != b.dim() or y.data_ptr() == b.data_ptr():
        raise ValueError("y must be shaped like b and must not be b")
    ctx = context(pat.device)
    st = load_library().tpilu_apply_noalloc(ctx.h, pat.h, _ptr(f_val), B, _ptr(b), _ptr(y))
    ctx.check(st, "apply_noalloc")
    return y


def inverse(pat: Pattern, f_val: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Level-based incomplete inverses of L~ and U~ (Sec. 3.5), shaped like F."""
    _need(f_val, torch.float64, "f_val", pat.device)
    if _batch_of(f_val, pat.nnz_f, "f_val") != 1:
        raise ValueError("incomplete inverses: one instance only")
    g = torch.empty_like(f_val) if out is None else _need_size(out, torch.float64, "out", pat.device, pat.nnz_f)
    if g.data_ptr() == f_val.data_ptr():
        raise ValueError("out must not be f_val")
    ctx = context(pat.device)
    ctx.check(load_library().tpilu_inverse(ctx.h, pat.h, _ptr(f_val), 1, _ptr(g)), "inverse")
    return g


def apply_inverse(pat: Pattern, g_val: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
                  return_x: bool = False):
    """y = U~~^-1 L~~^-1 b with the incomplete inverses (two products, Eq. 3a)."""
    _need(g_val, torch.float64, "g_val", pat.device)
    _need(b, torch.float64, "b", pat.device)
    if _batch_of(b, pat.n, "b") != 1 or _batch_of(g_val, pat.nnz_f, "g_val") != 1:
        raise ValueError("incomplete inverses: one instance only")
    y = torch.empty_like(b) if out is None else _need_size(out, torch.float64, "out", pat.device, pat.n)
    if y.data_ptr() == b.data_ptr():
        raise ValueError("out must not be b")
    x = torch.empty_like(b) if return_x else None
    ctx = context(pat.device)
    st = load_library().tpilu_apply_inverse(ctx.h, pat.h, _ptr(g_val), 1, _ptr(b), _ptr(y), _ptr(x))
    ctx.check(st, "apply_inverse")
    return (y, x) if return_x else y


def spmv(pat: Pattern, a_val: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    _need_size(a_val, torch.float64, "a_val", pat.device, pat.nnz_a)
    _need_size(x, torch.float64, "x", pat.device, pat.n)
    y = torch.empty(pat.n, dtype=torch.float64, device=pat.device)
    ctx = context(pat.device)
    ctx.check(load_library().tpilu_spmv(ctx.h, pat.h, _ptr(a_val), _ptr(x), _ptr(y)), "spmv")
    return y


def dot(x: torch.Tensor, y: torch.Tensor) -> float:
    """Fixed-shape inner product (16384 strided partial sums, then a pairwise tree)."""
    _need(x, torch.float64, "x", None)
    _need(y, torch.float64, "y", x.device)
    if y.numel() != x.numel():
        raise ValueError(f"x has {x.numel()} entries, y {y.numel()}")
    ctx = context(x.device)
    r = C.c_double(0.0)
    ctx.check(load_library().tpilu_dot(ctx.h, x.numel(), _ptr(x), _ptr(y), C.byref(r)), "dot")
    return r.value


def givens(a: torch.Tensor, b: torch.Tensor):
    """(rho, c, s) of the rotation of every pair (a_i, b_i), computed by the
    device code of the GMRES rotation step."""
    _need(a, torch.float64, "a", None)
    _need(b, torch.float64, "b", a.device)
    if a.shape != b.shape:
        raise ValueError("a and b differ in shape")
    rho, c, s = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    ctx = context(a.device)
    ctx.check(load_library().tpilu_givens(ctx.h, a.numel(), _ptr(a), _ptr(b), _ptr(rho), _ptr(c), _ptr(s)),
              "givens")
    return rho, c, s


def numeric_critical_path(pat: Pattern, w_hop: float = 1.0, w_step: float = 0.0) -> float:
    """Longest dependency chain of the numeric factorization, a row-to-row
    hand-off weighing w_hop and an l of a row weighing w_step (the dataflow
    kernel run in critical-path mode); the defaults count hand-offs."""
    ctx = context(pat.device)
    h = C.c_double(0.0)
    ctx.check(load_library().tpilu_numeric_critical_path(ctx.h, pat.h, float(w_hop), float(w_step), C.byref(h)),
              "numeric_critical_path")
    return h.value


def handoff_probe(same_xcd: bool, rounds: int = 2000, device=None) -> float:
    """Mean round trip (ns) of a value passed between two wavefronts through
    device memory, on one XCD or across two."""
    ctx = context(device)
    ns = C.c_double(0.0)
    ctx.check(load_library().tpilu_handoff_probe(ctx.h, 1 if same_xcd else 0, rounds, C.byref(ns)),
              "handoff_probe")
    return ns.value


def gmres(pat: Pattern, a_val: torch.Tensor, f_val: torch.Tensor, b: torch.Tensor, x0: torch.Tensor | None = None,
          restart: int = 30, maxit: int | None = None, rtol: float = 1e-8, raise_notconv: bool = False,
          inverse: bool = False):
    """Right-preconditioned restarted GMRES.  Returns (x, info).  inverse=True:
    f_val holds the incomplete inverses (from inverse()) and M^-1 is applied by
    two products."""
    _need_size(a_val, torch.float64, "a_val", pat.device, pat.nnz_a)
    _need_size(f_val, torch.float64, "f_val", pat.device, pat.nnz_f)
    _need_size(b, torch.float64, "b", pat.device, pat.n)
    x = torch.zeros_like(b) if x0 is None else _need_size(x0, torch.float64, "x0", pat.device, pat.n).clone()
    if maxit is None:
        maxit = min(10 * pat.n, 100000)
    hist = (C.c_double * max(maxit, 1))()
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    ctx = context(pat.device)
    fn = load_library().tpilu_gmres_inverse if inverse else load_library().tpilu_gmres
    st = fn(ctx.h, pat.h, _ptr(a_val), _ptr(f_val), _ptr(b), _ptr(x), restart, maxit, rtol, C.byref(it),
            C.byref(rr), hist)
    if st != E_NOTCONV or raise_notconv:
        ctx.check(st, "gmres")
    info = {"iters": it.value, "relres": rr.value, "status": st, "hist": list(hist[: it.value])}
    return x, info


def bicgstab(pat: Pattern, a_val: torch.Tensor, m_val: torch.Tensor, b: torch.Tensor,
             x0: torch.Tensor | None = None, maxit: int | None = None, rtol: float = 1e-8,
             inverse: bool = False, raise_notconv: bool = False):
    """Right-preconditioned BiCGSTAB (Sec. 4's solver).  m_val: the factor, or
    the incomplete inverses with inverse=True.  maxit / iters count half steps.
    Returns (x, info)."""
    _need_size(a_val, torch.float64, "a_val", pat.device, pat.nnz_a)
    _need_size(m_val, torch.float64, "m_val", pat.device, pat.nnz_f)
    _need_size(b, torch.float64, "b", pat.device, pat.n)
    x = torch.zeros_like(b) if x0 is None else _need_size(x0, torch.float64, "x0", pat.device, pat.n).clone()
    if maxit is None:
        maxit = min(10 * pat.n, 100000)
    hist = (C.c_double * max(maxit, 1))()
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    ctx = context(pat.device)
    st = load_library().tpilu_bicgstab(ctx.h, pat.h, _ptr(a_val), _ptr(m_val), 1 if inverse else 0, _ptr(b),
                                       _ptr(x), maxit, rtol, C.byref(it), C.byref(rr), hist)
    if st != E_NOTCONV or raise_notconv:
        ctx.check(st, "bicgstab")
    info = {"iters": it.value, "relres": rr.value, "status": st, "hist": list(hist[: it.value])}
    return x, info


def apply_adjoint(pat: Pattern, f_val, x, y, ybar):
    """Reverse mode of y = U~^-1 L~^-1 b.  Returns (bbar, fbar)."""
    for t, nm in ((f_val, "f_val"), (x, "x"), (y, "y"), (ybar, "ybar")):
        _need(t, torch.float64, nm, pat.device)
    B = _batch_of(ybar, pat.n, "ybar")
    _need_size(f_val, torch.float64, "f_val", pat.device, pat.nnz_f, B)
    for t, nm in ((x, "x"), (y, "y")):
        if tuple(t.shape) != tuple(ybar.shape):
            raise ValueError(f"{nm} has shape {tuple(t.shape)}, expected {tuple(ybar.shape)}")
    bbar = torch.empty_like(ybar)
    fbar = torch.empty_like(f_val)
    ctx = context(pat.device)
    st = load_library().tpilu_apply_adjoint(ctx.h, pat.h, _ptr(f_val), B, _ptr(x), _ptr(y), _ptr(ybar),
                                            _ptr(bbar), _ptr(fbar))
    ctx.check(st, "apply_adjoint")
    return bbar, fbar


def numeric_adjoint(pat: Pattern, f_val, fbar):
    """Reverse sweep of the elimination.  Returns (abar, fbar after the sweep)."""
    _need(f_val, torch.float64, "f_val", pat.device)
    B = _batch_of(f_val, pat.nnz_f, "f_val")
    if tuple(fbar.shape) != tuple(f_val.shape):
        raise ValueError(f"fbar has shape {tuple(fbar.shape)}, expected {tuple(f_val.shape)}")
    fb = _need(fbar, torch.float64, "fbar", pat.device).clone()
    shape = (pat.nnz_a,) if f_val.dim() == 1 else (pat.nnz_a, B)
    abar = torch.empty(shape, dtype=torch.float64, device=pat.device)
    ctx = context(pat.device)
    st = load_library().tpilu_numeric_adjoint(ctx.h, pat.h, _ptr(f_val), B, _ptr(fb), _ptr(abar))
    ctx.check(st, "numeric_adjoint")
    return abar, fb


class BatchedGraph:
    """All numeric factorizations plus all solves of a batch in one HIP graph.

    The tensors given here are baked into the graph; every launch() recomputes
    f_val and y from the current contents of a_val and b.
    """

    def __init__(self, pat: Pattern, a_val, b, f_val=None, y=None):
        _need(a_val, torch.float64, "a_val", pat.device)
        _need(b, torch.float64, "b", pat.device)
        B = _batch_of(a_val, pat.nnz_a, "a_val")
        if _batch_of(b, pat.n, "b") != B:
            raise ValueError("a_val and b batch sizes differ")
        if a_val.dim() != b.dim():
            raise ValueError("a_val and b must both be 1-D or both 2-D")
        self.pat, self.a_val, self.b = pat, a_val, b
        self.f_val = torch.empty((pat.nnz_f, B) if a_val.dim() == 2 else (pat.nnz_f,), dtype=torch.float64,
                                 device=pat.device) if f_val is None else f_val
        self.y = torch.empty_like(b) if y is None else y
        _need_size(self.f_val, torch.float64, "f_val", pat.device, pat.nnz_f, B)
        _need_size(self.y, torch.float64, "y", pat.device, pat.n, B)
        if self.f_val.dim() != a_val.dim() or self.y.dim() != b.dim() or self.y.data_ptr() == b.data_ptr():
            raise ValueError("f_val and y must be shaped like the factor and b, and y must not be b")
        ctx = context(pat.device)
        h = C.c_void_p()
        st = load_library().tpilu_batched_graph_create(ctx.h, pat.h, _ptr(a_val), B, _ptr(self.f_val), _ptr(b),
                                                       _ptr(self.y), C.byref(h))
        ctx.check(st, "batched_graph_create")
        self.h = h

    def launch(self):
        s = torch.cuda.current_stream(self.pat.device).cuda_stream
        st = load_library().tpilu_batched_graph_launch(self.h, C.c_void_p(s))
        if st != OK:
            raise TpiluError(st, "batched_graph_launch failed")

    def check(self) -> int:
        """Wait for the current stream and report the status of the last
        launch on it; returns bad_row or -1, raises on a zero pivot or timeout."""
        s = torch.cuda.current_stream(self.pat.device).cuda_stream
        bad = C.c_int64(-1)
        st = load_library().tpilu_batched_graph_check(self.h, C.c_void_p(s), C.byref(bad))
        if st == E_ZEROPIVOT:
            raise ZeroPivotError(st, f"batched graph: zero pivot in row {bad.value}", bad.value)
        if st != OK:
            raise TpiluError(st, "batched graph: device status", bad.value)
        return bad.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            try:
                torch.cuda.synchronize(self.pat.device)
            except Exception:
                pass
            _lib.tpilu_batched_graph_destroy(h)
            self.h = None


class ILUApply(torch.autograd.Function):
    """y = M^-1 b with M = L~ U~ = ILU(k) of A (values a_val on pattern pat).

    Forward: numeric factorization + triangular solves.  Backward: transposed
    solves and the reverse sweep of the elimination, giving d/d a_val and
    d/d b.  Shapes [nnz_a] / [n] or batched [nnz_a, B] / [n, B].
    """

    @staticmethod
    def forward(ctx, a_val, b, pat):
        f = numeric(pat, a_val.detach().contiguous())
        y, x = apply(pat, f, b.detach().contiguous(), return_x=True)
        ctx.pat = pat
        ctx.save_for_backward(f, x, y)
        return y

    @staticmethod
    def backward(ctx, ybar):
        f, x, y = ctx.saved_tensors
        bbar, fbar = apply_adjoint(ctx.pat, f, x, y, ybar.contiguous())
        abar, _ = numeric_adjoint(ctx.pat, f, fbar)
        return abar, bbar, None
