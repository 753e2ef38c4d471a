"""MI355X (gfx950) level-of-fill ILU(k) preconditioning, bit-compatible with
the sequential algorithm (Dong & Cooperman, TPILU(k)).

Entry points (GPU only; they raise if the HIP library is missing):

    pat = symbolic(rowptr, col, k)          # Phase I, Algorithm 1
    f   = numeric(pat, a_val)               # Phase II, Eqs. 6a/6b
    y   = apply(pat, f, b)                  # y = U~^-1 L~^-1 b, Eq. 1
    x, info = gmres(pat, a_val, f, b)       # right-preconditioned GMRES(m)
    g   = inverse(pat, f)                   # level-based incomplete inverses, Sec. 3.5
    y   = apply_inverse(pat, g, b)          # M^-1 b by two products, Eq. 3a
    x, info = bicgstab(pat, a_val, f, b)    # right-preconditioned BiCGSTAB (Sec. 4)
    ILUApply.apply(a_val, b, pat)           # autograd: d/d a_val, d/d b
    BatchedGraph(pat, a_vals, bs).launch()  # batch in one HIP graph

``inputs`` builds the seeded synthetic workloads.
"""

_BINDING_NAMES = {
    "symbolic", "numeric", "apply", "gmres", "spmv", "dot", "apply_adjoint", "numeric_adjoint",
    "inverse", "apply_inverse", "bicgstab",
    "check", "BatchedGraph", "ILUApply", "Pattern", "TpiluError", "ZeroPivotError", "context",
    "load_library", "LIB_PATH",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding

        return getattr(binding, name)
    raise AttributeError(name)
