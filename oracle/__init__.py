"""Sequential CPU oracle for ILU(k) -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never loads it.

The arithmetic lives in ``ilu_oracle.c`` (plain sequential C, compiled with
``-O2 -ffp-contract=off``); this module only builds that file and marshals
numpy arrays in and out of it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ilu_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EZEROPIVOT, ENOTCONV = 0, 1, 2, 3, 5


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Pattern(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("lev", C.POINTER(C.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        L.orc_validate.argtypes = [i64, P, P]
        L.orc_symbolic.argtypes = [i64, P, P, i32, C.POINTER(_Pattern)]
        L.orc_pattern_free.argtypes = [C.POINTER(_Pattern)]
        L.orc_numeric.argtypes = [i64, P, P, P, P, P, P, C.POINTER(i64)]
        L.orc_numeric_fused.argtypes = [i64, P, P, P, P, P, P, C.POINTER(i64)]
        L.orc_numeric_rows.argtypes = [i64, P, P, P, P, P, P, i64, P, P]
        L.orc_apply.argtypes = [i64, P, P, P, P, P, P]
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_spmv.restype = None
        L.orc_dot.argtypes = [i64, P, P]
        L.orc_dot.restype = dbl
        L.orc_nrm2.argtypes = [i64, P]
        L.orc_nrm2.restype = dbl
        L.orc_gmres.argtypes = [i64, P, P, P, P, P, P, P, P, i32, i32, dbl,
                                C.POINTER(i32), C.POINTER(dbl), P]
        L.orc_gmres_inverse.argtypes = [i64, P, P, P, P, P, P, P, P, i32, i32, dbl,
                                        C.POINTER(i32), C.POINTER(dbl), P]
        L.orc_inverse.argtypes = [i64, P, P, P, P]
        L.orc_bicgstab.argtypes = [i64, P, P, P, P, P, P, i32, P, P, i32, dbl,
                                   C.POINTER(i32), C.POINTER(dbl), P]
        L.orc_apply_inverse.argtypes = [i64, P, P, P, P, P, P]
        L.orc_apply_adjoint.argtypes = [i64, P, P, P, P, P, P, P, P]
        L.orc_numeric_adjoint.argtypes = [i64, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"oracle status {status} {msg}")
        self.status = status


def validate(n, rowptr, col) -> int:
    rp, ci = _c(rowptr, np.int64), _c(col, np.int32)
    return lib().orc_validate(n, _p(rp), _p(ci))


def symbolic(n, rowptr, col, k):
    """Algorithm 1.  Returns (rowptrF int64, colF int32, levF int32)."""
    rp, ci = _c(rowptr, np.int64), _c(col, np.int32)
    pat = _Pattern()
    st = lib().orc_symbolic(n, _p(rp), _p(ci), int(min(k, 2**31 - 1)), C.byref(pat))
    if st:
        raise OracleError(st, "symbolic")
    nnz = pat.nnz
    try:
        rpF = np.ctypeslib.as_array(pat.rowptr, shape=(n + 1,)).copy()
        if nnz > 0:
            ciF = np.ctypeslib.as_array(pat.col, shape=(nnz,)).copy()
            lvF = np.ctypeslib.as_array(pat.lev, shape=(nnz,)).copy()
        else:
            ciF = np.zeros(0, np.int32)
            lvF = np.zeros(0, np.int32)
    finally:
        lib().orc_pattern_free(C.byref(pat))
    return rpF, ciF, lvF


def numeric(n, rowptr, col, val, rowptrF, colF, fused=False):
    """Row-wise IKJ elimination on the pattern.  Returns (F values, bad_row).
    ``fused``: every update f - l * u rounded once (fused multiply-add)
    instead of product and difference rounded on their own."""
    rp, ci, v = _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64)
    rpF, ciF = _c(rowptrF, np.int64), _c(colF, np.int32)
    vF = np.empty(ciF.shape[0], dtype=np.float64)
    bad = C.c_int64(-1)
    fn = lib().orc_numeric_fused if fused else lib().orc_numeric
    st = fn(n, _p(rp), _p(ci), _p(v), _p(rpF), _p(ciF), _p(vF), C.byref(bad))
    if st not in (OK, EZEROPIVOT):
        raise OracleError(st, "numeric")
    return vF, int(bad.value)


def numeric_rows(n, rowptr, col, val, rowptrF, colF, valF, rows):
    """The listed rows alone, each eliminated exactly as in ``numeric`` but
    against the pivot rows given in ``valF`` (e.g. a factor computed
    elsewhere).  Returns one array per row, in the order of ``rows``."""
    rp, ci, v = _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64)
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    rr = _c(rows, np.int64)
    lens = rpF[rr + 1] - rpF[rr]
    out = np.empty(int(lens.sum()), dtype=np.float64)
    st = lib().orc_numeric_rows(n, _p(rp), _p(ci), _p(v), _p(rpF), _p(ciF), _p(vF), rr.shape[0], _p(rr), _p(out))
    if st:
        raise OracleError(st, "numeric_rows")
    return np.split(out, np.cumsum(lens)[:-1])


def apply(n, rowptrF, colF, valF, p):
    """y = U~^-1 L~^-1 p.  Returns (x = L~^-1 p, y)."""
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    pp = _c(p, np.float64)
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    st = lib().orc_apply(n, _p(rpF), _p(ciF), _p(vF), _p(pp), _p(x), _p(y))
    if st:
        raise OracleError(st, "apply")
    return x, y


def spmv(n, rowptr, col, val, x):
    rp, ci, v, xx = _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    y = np.empty(n, dtype=np.float64)
    lib().orc_spmv(n, _p(rp), _p(ci), _p(v), _p(xx), _p(y))
    return y


def dot(x, y) -> float:
    xx, yy = _c(x, np.float64), _c(y, np.float64)
    return lib().orc_dot(xx.shape[0], _p(xx), _p(yy))


def inverse(n, rowptrF, colF, valF):
    """Level-based incomplete inverses of L~ and U~ on F's pattern (Sec. 3.5).
    Returns G: inverse of L~ in the strict lower slots, of U~ in the upper ones."""
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    vG = np.empty(ciF.shape[0], dtype=np.float64)
    st = lib().orc_inverse(n, _p(rpF), _p(ciF), _p(vF), _p(vG))
    if st:
        raise OracleError(st, "inverse")
    return vG


def apply_inverse(n, rowptrF, colF, valG, p):
    """y = U~~^-1 L~~^-1 p by two products.  Returns (x = L~~^-1 p, y)."""
    rpF, ciF, vG = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valG, np.float64)
    pp = _c(p, np.float64)
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    st = lib().orc_apply_inverse(n, _p(rpF), _p(ciF), _p(vG), _p(pp), _p(x), _p(y))
    if st:
        raise OracleError(st, "apply_inverse")
    return x, y


def gmres(n, rowptr, col, val, rowptrF, colF, valF, b, x0=None, restart=30, maxit=None, rtol=1e-8,
          inverse=False):
    """Right-preconditioned restarted GMRES.  Returns dict(x, iters, relres, status, hist).
    inverse=True: valF holds the incomplete inverses G and M^-1 is applied by products."""
    rp, ci, v = _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64)
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if maxit is None:
        maxit = min(10 * n, 100000)
    hist = np.zeros(max(maxit, 1), dtype=np.float64)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    fn = lib().orc_gmres_inverse if inverse else lib().orc_gmres
    st = fn(n, _p(rp), _p(ci), _p(v), _p(rpF), _p(ciF), _p(vF), _p(bb), _p(x),
            int(restart), int(maxit), float(rtol), C.byref(it), C.byref(rr), _p(hist))
    if st not in (OK, ENOTCONV):
        raise OracleError(st, "gmres")
    return {"x": x, "iters": int(it.value), "relres": float(rr.value), "status": st,
            "hist": hist[: it.value].copy()}


def bicgstab(n, rowptr, col, val, rowptrF, colF, valM, b, x0=None, maxit=None, rtol=1e-8, inverse=False):
    """Right-preconditioned BiCGSTAB.  maxit and iters count half steps (one
    per preconditioner application).  Returns dict(x, iters, relres, status, hist)."""
    rp, ci, v = _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64)
    rpF, ciF, vM = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valM, np.float64)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if maxit is None:
        maxit = min(10 * n, 100000)
    hist = np.zeros(max(maxit, 1), dtype=np.float64)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    st = lib().orc_bicgstab(n, _p(rp), _p(ci), _p(v), _p(rpF), _p(ciF), _p(vM), int(bool(inverse)), _p(bb),
                            _p(x), int(maxit), float(rtol), C.byref(it), C.byref(rr), _p(hist))
    if st not in (OK, ENOTCONV):
        raise OracleError(st, "bicgstab")
    return {"x": x, "iters": int(it.value), "relres": float(rr.value), "status": st,
            "hist": hist[: it.value].copy()}


def apply_adjoint(n, rowptrF, colF, valF, x, y, ybar):
    """Adjoint of y = U~^-1 L~^-1 b.  Returns (bbar, Fbar)."""
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    xx, yy, yb = _c(x, np.float64), _c(y, np.float64), _c(ybar, np.float64)
    bbar = np.empty(n, dtype=np.float64)
    Fbar = np.empty(ciF.shape[0], dtype=np.float64)
    st = lib().orc_apply_adjoint(n, _p(rpF), _p(ciF), _p(vF), _p(xx), _p(yy), _p(yb), _p(bbar), _p(Fbar))
    if st:
        raise OracleError(st, "apply_adjoint")
    return bbar, Fbar


def numeric_adjoint(n, rowptr, col, rowptrF, colF, valF, Fbar):
    """Reverse sweep of the elimination.  Returns (abar, Fbar after the sweep)."""
    rp, ci = _c(rowptr, np.int64), _c(col, np.int32)
    rpF, ciF, vF = _c(rowptrF, np.int64), _c(colF, np.int32), _c(valF, np.float64)
    Fb = np.array(Fbar, dtype=np.float64, copy=True)
    abar = np.empty(ci.shape[0], dtype=np.float64)
    st = lib().orc_numeric_adjoint(n, _p(rp), _p(ci), _p(rpF), _p(ciF), _p(vF), _p(Fb), _p(abar))
    if st:
        raise OracleError(st, "numeric_adjoint")
    return abar, Fb


def ilu(A, k):
    """Convenience: symbolic + numeric for a single-instance inputs.CSR."""
    rpF, ciF, lvF = symbolic(A.n, A.rowptr, A.col, k)
    vF, bad = numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    return rpF, ciF, lvF, vF, bad
