"""Independent reference computations used to pin the oracle.

None of these share code with ``oracle/`` or with the GPU library.  Each one
is a different route to a quantity the paper or textbook mathematics fixes:

* ``levels_dp``     -- Def. 2.3 evaluated literally on a dense level table,
                       pairs taken by increasing min(i, j) (every term of the
                       recurrence has a smaller min, so it is already known).
* ``levels_paths``  -- the fill-path characterisation of the same levels:
                       level(i,j) + 1 is the number of edges of the shortest
                       path i -> j in the graph of A whose interior vertices
                       are all smaller than min(i, j).
* ``full_fill``     -- symbolic Gaussian elimination without dropping (the
                       k = infinity case, Sec. 2).
* ``dense_masked_lu`` -- dense Gaussian elimination in KIJ order (pivot loop
                       outermost) restricted to a 0/1 mask; per entry the
                       updates still arrive in ascending pivot order, so its
                       bits must equal the row-wise IKJ result.
"""
from __future__ import annotations

from collections import deque

from fractions import Fraction

import numpy as np

INF = 1 << 40


def dense_pattern(n, rowptr, col):
    M = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    M[rows, col] = True
    return M


def levels_dp(M: np.ndarray) -> np.ndarray:
    n = M.shape[0]
    lev = np.full((n, n), INF, dtype=np.int64)
    lev[M] = 0
    for m in range(n):
        if m == 0:
            continue
        # row m, columns j > m : min over h < m of lev[m,h] + lev[h,j] + 1
        cand = (lev[m, :m][:, None] + lev[:m, m:]).min(axis=0) + 1
        row = lev[m, m:]
        lev[m, m:] = np.where(M[m, m:], 0, np.minimum(INF, cand))
        del row
        # column m, rows i > m : min over h < m of lev[i,h] + lev[h,m] + 1
        cand = (lev[m + 1:, :m] + lev[:m, m][None, :]).min(axis=1) + 1
        lev[m + 1:, m] = np.where(M[m + 1:, m], 0, np.minimum(INF, cand))
    return lev


def levels_paths(M: np.ndarray) -> np.ndarray:
    n = M.shape[0]
    adj = [np.nonzero(M[v])[0] for v in range(n)]
    lev = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            if M[i, j]:
                lev[i, j] = 0
                continue
            lim = min(i, j)
            dist = {i: 0}
            dq = deque([i])
            found = INF
            while dq:
                v = dq.popleft()
                for w in adj[v]:
                    if w == j:
                        found = min(found, dist[v] + 1)
                    elif w < lim and w not in dist:
                        dist[w] = dist[v] + 1
                        dq.append(w)
            lev[i, j] = found - 1 if found < INF else INF
    return lev


def full_fill(M: np.ndarray) -> np.ndarray:
    G = M.copy()
    n = G.shape[0]
    for h in range(n):
        rows = np.nonzero(G[h + 1:, h])[0] + h + 1
        if rows.size:
            G[np.ix_(rows, np.arange(h + 1, n))] |= G[h, h + 1:][None, :]
    return G


def dense_masked_lu(Ad: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """KIJ elimination on the mask: for each pivot h, every later row i with
    (i,h) in the mask is scaled and then updated on columns j > h where both
    (h,j) and (i,j) are in the mask.  Products and differences are rounded
    separately (numpy elementwise ops)."""
    F = np.where(mask, Ad, 0.0).astype(np.float64)
    n = F.shape[0]
    for h in range(n):
        rows = np.nonzero(mask[h + 1:, h])[0] + h + 1
        if rows.size == 0:
            continue
        F[rows, h] = F[rows, h] / F[h, h]
        cols = np.nonzero(mask[h, h + 1:])[0] + h + 1
        if cols.size == 0:
            continue
        sub = mask[np.ix_(rows, cols)]
        prod = np.multiply(F[rows, h][:, None], F[h, cols][None, :])
        upd = np.subtract(F[np.ix_(rows, cols)], prod)
        blk = F[np.ix_(rows, cols)]
        F[np.ix_(rows, cols)] = np.where(sub, upd, blk)
    return np.where(mask, F, 0.0)


def fused_update(f: float, l: float, u: float) -> float:
    """f - l * u rounded once to the nearest double (ties to even), from exact
    rational arithmetic: what a fused multiply-add must return.  An exact
    zero takes the sign IEEE-754 gives the float expression, which is then
    exact as well."""
    ex = Fraction(f) - Fraction(l) * Fraction(u)
    if ex == 0:
        return f - l * u
    return ex.numerator / ex.denominator  # int / int is correctly rounded


def dense_masked_lu_fused(Ad: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """The elimination of dense_masked_lu (KIJ on the mask), every update
    f_ij - l_ih f_hj rounded once (fused_update); divisions as usual."""
    n = Ad.shape[0]
    F = [[float(Ad[i, j]) if mask[i, j] else 0.0 for j in range(n)] for i in range(n)]
    for h in range(n):
        for i in range(h + 1, n):
            if not mask[i, h]:
                continue
            F[i][h] = F[i][h] / F[h][h]
            for j in range(h + 1, n):
                if mask[h, j] and mask[i, j]:
                    F[i][j] = fused_update(F[i][j], F[i][h], F[h][j])
    return np.where(mask, np.array(F, dtype=np.float64).reshape(n, n), 0.0)


def to_dense_vals(n, rowptr, col, val):
    D = np.zeros((n, n), dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    D[rows, col] = val
    return D


def csr_from_dense_mask(M: np.ndarray, vals: np.ndarray | None = None):
    n = M.shape[0]
    rows, cols = np.nonzero(M)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    v = None if vals is None else vals[rows, cols].astype(np.float64)
    return rowptr, cols.astype(np.int32), v


def bits(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)
