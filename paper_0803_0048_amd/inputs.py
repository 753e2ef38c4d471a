"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds matrices and vectors; it holds none of the ILU(k)
arithmetic.  Both the GPU path and the sequential oracle consume the arrays it
returns, so that the two sides see identical inputs.

All matrices are returned as CSR with 0-based indices, columns sorted
ascending inside every row, the diagonal always stored:

    rowptr  int64[n+1]
    col     int32[nnz]
    val     float64[nnz]            (single instance)
    val     float64[nnz, B]         (batch of B instances sharing one pattern,
                                     entry-major / instance-minor, the layout
                                     the batched entry points take)

Workloads (the paper's own matrices are not available; these stand in for
them):

* ``conv_diff_2d`` / ``conv_diff_3d``: -eps*Laplace(u) + b.grad(u) on the unit
  square / cube, central differences on an m^d interior grid, h = 1/(m+1),
  Dirichlet boundary, natural (lexicographic) row order, every coefficient
  multiplied by h^2.  With cell Peclet number |b_c| h / (2 eps) > 1 the matrix
  is not diagonally dominant (stand-in for the paper's driven-cavity and 3-D
  stencil problems, Sec. 4.1-4.2).
* ``stencil27_3d``: the 27-point 3-D stencil (diffusion on all 26 neighbours,
  convection on the 6 face neighbours), stand-in for the 27-point central
  differencing problem of Sec. 4.2.
* ``random_uniform``: general sparse non-symmetric matrix with a given entry
  count, columns uniform over the whole row (stand-in for the generated
  matrices of the paper's Table 3, whose counts it matches).
* ``random_banded``: general sparse non-symmetric matrix, a fixed number of
  off-diagonal columns per row drawn uniformly inside a band plus a few drawn
  anywhere, values U(-1, 1), diagonal 1.1 x the row's absolute sum, so the
  matrix is strictly diagonally dominant (stand-in for the diagonally dominant
  general sparse matrices of dimension up to 160,000 in Sec. 4.4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CSR",
    "conv_diff_2d",
    "conv_diff_3d",
    "random_banded",
    "random_pattern",
    "stencil27_3d",
    "stencil27_ilu",
    "conv_diff_2d_64x64_ilu1",
    "random_banded_ilu2",
    "conv_diff_3d_ilu",
    "batched_conv_diff_2d_ilu2",
    "batched_stencil27_ilu",
    "differentiated_conv_diff_3d_ilu1",
    "random_uniform",
    "paper_scale_random_ilu1",
]


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz] or float64[nnz, B]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def batch(self) -> int:
        return 1 if self.val.ndim == 1 else int(self.val.shape[1])

    def instance(self, b: int) -> "CSR":
        """Instance ``b`` of a batch as a single-instance CSR (values copied)."""
        v = self.val if self.val.ndim == 1 else np.ascontiguousarray(self.val[:, b])
        return CSR(self.n, self.rowptr, self.col, v, dict(self.meta))

    def to_dense(self, b: int | None = None) -> np.ndarray:
        v = self.val if self.val.ndim == 1 else self.val[:, 0 if b is None else b]
        d = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.col] = v
        return d


def _stencil_pattern(shape):
    """Rows/cols/offset-id arrays of a (2*dim+1)-point stencil in natural order.

    Returns (rowptr, col, kind, sign) where ``kind[e]`` is the axis (0..dim-1)
    of a neighbour entry or -1 for the diagonal, and ``sign[e]`` is +1 for the
    forward neighbour, -1 for the backward one, 0 for the diagonal.
    """
    dim = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n)
    coords = np.unravel_index(idx, shape[::-1])[::-1]  # coords[0] = fastest axis
    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * shape[a - 1])
    # offsets in increasing column order: -stride[dim-1] .. -1, 0, +1 .. +stride[dim-1]
    offs = []
    for a in reversed(range(dim)):
        offs.append((a, -1))
    offs.append((-1, 0))
    for a in range(dim):
        offs.append((a, +1))
    cols = np.empty((n, len(offs)), dtype=np.int64)
    valid = np.empty((n, len(offs)), dtype=bool)
    kind = np.empty((n, len(offs)), dtype=np.int64)
    sign = np.empty((n, len(offs)), dtype=np.int64)
    for k, (a, s) in enumerate(offs):
        if a < 0:
            cols[:, k] = idx
            valid[:, k] = True
        else:
            cols[:, k] = idx + s * strides[a]
            c = coords[a]
            valid[:, k] = (c > 0) if s < 0 else (c < shape[a] - 1)
        kind[:, k] = a
        sign[:, k] = s
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols[valid].astype(np.int32), kind[valid], sign[valid]


def _stencil_values(kind, sign, eps, bvec, h, dim):
    """Coefficients of -eps*Laplace + b.grad, central differences, times h^2."""
    eps = np.asarray(eps, dtype=np.float64)
    bvec = np.asarray(bvec, dtype=np.float64)
    batched = eps.ndim == 1
    if not batched:
        eps = eps[None]
        bvec = bvec[None, :]
    B = eps.shape[0]
    val = np.empty((kind.shape[0], B), dtype=np.float64)
    diag = kind < 0
    val[diag, :] = (2.0 * dim) * eps[None, :]
    for a in range(dim):
        m = kind == a
        half = bvec[:, a] * (h / 2.0)  # [B]
        val[m, :] = -eps[None, :] + sign[m][:, None] * half[None, :]
    return val if batched else val[:, 0].copy()


def conv_diff_2d(m: int, eps, bx, by) -> CSR:
    """2-D 5-point convection-diffusion on an m x m grid (see module doc)."""
    h = 1.0 / (m + 1)
    rowptr, col, kind, sign = _stencil_pattern((m, m))
    eps_a = np.asarray(eps, dtype=np.float64)
    bvec = np.stack([np.asarray(bx, dtype=np.float64), np.asarray(by, dtype=np.float64)], axis=-1)
    val = _stencil_values(kind, sign, eps_a, bvec, h, 2)
    return CSR(m * m, rowptr, col, val, {"kind": "conv_diff_2d", "m": m, "h": h})


def conv_diff_3d(m: int, eps, bvec) -> CSR:
    """3-D 7-point convection-diffusion on an m^3 grid (see module doc)."""
    h = 1.0 / (m + 1)
    rowptr, col, kind, sign = _stencil_pattern((m, m, m))
    val = _stencil_values(kind, sign, np.asarray(eps, dtype=np.float64), np.asarray(bvec, dtype=np.float64), h, 3)
    return CSR(m**3, rowptr, col, val, {"kind": "conv_diff_3d", "m": m, "h": h})


def stencil27_3d(m: int, eps: float, bvec) -> CSR:
    """3-D 27-point stencil on an m^3 grid, natural order: the diffusion part of
    the 27-point central-difference Laplacian (every one of the 26 neighbours
    -eps, the diagonal 26 eps) plus central-difference convection b.grad on
    the six face neighbours (+-b_a h / 2), all times h^2 like the 7-point
    stencils.  Stand-in for the 27-point central differencing problem of
    Sec. 4.2 (50^3 to 90^3)."""
    h = 1.0 / (m + 1)
    n = m**3
    idx = np.arange(n, dtype=np.int64)
    x = idx % m
    y = (idx // m) % m
    z = idx // (m * m)
    bvec = np.asarray(bvec, dtype=np.float64)
    cols, vals, valid = [], [], []
    for dz in (-1, 0, 1):  # lexicographic (dz, dy, dx) = ascending column order
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = (x + dx >= 0) & (x + dx < m) & (y + dy >= 0) & (y + dy < m) & (z + dz >= 0) & (z + dz < m)
                c = idx + dz * m * m + dy * m + dx
                if dx == dy == dz == 0:
                    v = np.full(n, 26.0 * eps)
                else:
                    v = np.full(n, -eps)
                    if abs(dx) + abs(dy) + abs(dz) == 1:  # face neighbour: convection
                        a = 0 if dx else (1 if dy else 2)
                        v = v + (dx + dy + dz) * bvec[a] * (h / 2.0)
                cols.append(c)
                vals.append(v)
                valid.append(ok)
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    M = np.stack(valid, axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(M.sum(axis=1))
    col = C[M].astype(np.int32)
    val = V[M] * (h * h)
    return CSR(n, rowptr, col, val, {"kind": "stencil27_3d", "m": m, "h": h})


def stencil27_ilu(m: int = 50, k: int = 1, seed: int = 1006):
    """3-D 27-point stencil (next-step workload, Sec. 4.2's 50^3 to 90^3),
    eps = 1, b ~ U[-10, 10]^3 (convection mild enough to keep the diagonal
    dominant), rhs ~ N(0, 1); ILU(k) for k = 0..3."""
    rng = np.random.default_rng(seed)
    bvec = rng.uniform(-10.0, 10.0, size=3)
    A = stencil27_3d(m, 1.0, bvec)
    b = rng.standard_normal(A.n)
    return {"name": f"stencil27_3d_{m}cubed_ilu{k}", "A": A, "b": b, "k": k, "restart": 50, "rtol": 1e-8}


def _first_distinct(cand: np.ndarray, forbid: np.ndarray, need: int) -> tuple[np.ndarray, np.ndarray]:
    """For every row take the first ``need`` candidates that are distinct from
    each other and from the row's forbidden values.  Returns (chosen, ok)."""
    n, K = cand.shape
    dup = np.zeros((n, K), dtype=bool)
    for f in range(forbid.shape[1]):
        dup |= cand == forbid[:, f : f + 1]
    for a in range(1, K):
        dup[:, a] |= (cand[:, :a] == cand[:, a : a + 1]).any(axis=1)
    good = ~dup
    rank = np.cumsum(good, axis=1)
    ok = rank[:, -1] >= need
    chosen = np.zeros((n, need), dtype=np.int64)
    for r in range(need):
        pos = np.argmax(good & (rank == r + 1), axis=1)
        chosen[:, r] = cand[np.arange(n), pos]
    return chosen, ok


def random_banded(n: int, seed: int, band: int = 2000, n_band: int = 8, n_any: int = 2,
                  dominance: float = 1.1) -> CSR:
    """General sparse non-symmetric, strictly diagonally dominant matrix.

    Row i holds its diagonal, ``n_band`` distinct columns drawn uniformly from
    [max(0, i-band), min(n-1, i+band)] minus {i}, and ``n_any`` further
    distinct columns drawn uniformly from [0, n) minus the ones already taken.
    Off-diagonal values are U(-1, 1); a_ii = dominance * sum_j |a_ij|.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - band)
    hi = np.minimum(n - 1, i + band)
    K1 = n_band * 3
    cand = rng.integers(lo[:, None], hi[:, None] + 1, size=(n, K1))
    bcols, ok = _first_distinct(cand, i[:, None], n_band)
    for r in np.nonzero(~ok)[0]:  # rare: not enough distinct draws; redraw that row
        while True:
            c = rng.integers(lo[r], hi[r] + 1, size=4 * n_band)
            ch, okr = _first_distinct(c[None, :], np.array([[r]]), n_band)
            if okr[0]:
                bcols[r] = ch[0]
                break
    K2 = n_any * 4
    cand2 = rng.integers(0, n, size=(n, K2))
    acols, ok2 = _first_distinct(cand2, np.concatenate([i[:, None], bcols], axis=1), n_any)
    for r in np.nonzero(~ok2)[0]:
        while True:
            c = rng.integers(0, n, size=8 * n_any)
            ch, okr = _first_distinct(c[None, :], np.concatenate([[r], bcols[r]])[None, :], n_any)
            if okr[0]:
                acols[r] = ch[0]
                break
    off = np.concatenate([bcols, acols], axis=1)
    offv = rng.uniform(-1.0, 1.0, size=off.shape)
    diagv = dominance * np.abs(offv).sum(axis=1)
    cols = np.concatenate([off, i[:, None]], axis=1)
    vals = np.concatenate([offv, diagv[:, None]], axis=1)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    per = cols.shape[1]
    rowptr = np.arange(n + 1, dtype=np.int64) * per
    return CSR(n, rowptr, cols.reshape(-1).astype(np.int32), vals.reshape(-1).copy(),
               {"kind": "random_banded", "band": band, "n_band": n_band, "n_any": n_any})


def random_uniform(n: int, nnz: int, seed: int, dominance: float = 1.1) -> CSR:
    """General sparse non-symmetric, strictly diagonally dominant matrix with
    exactly ``nnz`` stored entries, columns uniform over the whole row.

    Row i holds its diagonal and c_i - 1 distinct off-diagonal columns drawn
    uniformly from [0, n) minus {i}, c_i = nnz // n, plus one for the first
    nnz % n rows.  Off-diagonal values are U(-1, 1); a_ii = dominance x the
    row's absolute sum.  With d entries per row, ILU(1) keeps about d^2 / 3
    per row (a pivot h < j contributes its upper part, d (1 - h/n) entries on
    average, and column h is stored in d (1 - h/n) of the later rows).
    """
    rng = np.random.default_rng(seed)
    base, extra = divmod(int(nnz), int(n))
    cnt = np.full(n, base, dtype=np.int64)
    cnt[:extra] += 1
    if (cnt < 1).any() or (cnt > n).any():
        raise ValueError("nnz must give every row 1..n entries")
    off = cnt - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), off)
    cols = rng.integers(0, n - 1, size=rows.size)
    cols += cols >= rows  # skip the diagonal
    # redraw repeated columns inside a row until every row's are distinct
    while True:
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.size, dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            break
        c = rng.integers(0, n - 1, size=nd)
        cols[dup] = c + (c >= rows[dup])
    offv = rng.uniform(-1.0, 1.0, size=rows.size)
    absum = np.zeros(n)
    np.add.at(absum, rows, np.abs(offv))
    allr = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    allc = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    allv = np.concatenate([offv, dominance * absum])
    order = np.lexsort((allc, allr))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(cnt)
    return CSR(n, rowptr, allc[order].astype(np.int32), allv[order].copy(), {"kind": "random_uniform", "nnz": int(nnz)})


def random_pattern(n: int, density: float, seed: int, *, diag_dominant: bool = True,
                   batch: int | None = None, explicit_zeros: float = 0.0) -> CSR:
    """Small random non-symmetric matrix for sweeps and edge cases.

    Every diagonal entry is stored.  Off-diagonal entries are kept with
    probability ``density``; values U(-1, 1); with ``diag_dominant`` the
    diagonal is 1 + sum |a_ij| of its row, else U(-1, 1) shifted away from 0.
    ``explicit_zeros`` is the probability that a stored off-diagonal value is
    set to exactly 0.0 (the entry stays in the pattern).
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    np.fill_diagonal(mask, True)
    rows, cols = np.nonzero(mask)
    nnz = rows.size
    B = 1 if batch is None else batch
    vals = rng.uniform(-1.0, 1.0, size=(nnz, B))
    if explicit_zeros > 0:
        z = rng.random(nnz) < explicit_zeros
        z &= rows != cols
        vals[z, :] = 0.0
    isdiag = rows == cols
    if diag_dominant:
        absum = np.zeros((n, B))
        np.add.at(absum, rows[~isdiag], np.abs(vals[~isdiag]))
        vals[isdiag, :] = 1.0 + absum[rows[isdiag]]
    else:
        d = vals[isdiag, :]
        vals[isdiag, :] = np.where(d >= 0, d + 0.5, d - 0.5)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    v = vals[:, 0].copy() if batch is None else np.ascontiguousarray(vals)
    return CSR(n, rowptr, cols.astype(np.int32), v, {"kind": "random_pattern", "density": density})


# ----------------------------------------------------------------------------
# The named workloads.  Seeds 1001-1007; batched instance i draws from
# SeedSequence(seed).spawn(B)[i].
# ----------------------------------------------------------------------------

def conv_diff_2d_64x64_ilu1(seed: int = 1001):
    """2-D 5-point, 64 x 64, eps = 1, (bx, by) ~ U[-20, 20]^2; ILU(1)."""
    rng = np.random.default_rng(seed)
    bx, by = rng.uniform(-20.0, 20.0, size=2)
    A = conv_diff_2d(64, 1.0, bx, by)
    b = rng.standard_normal(A.n)
    return {"name": "conv_diff_2d_64x64_ilu1", "A": A, "b": b, "k": 1, "restart": 30, "rtol": 1e-8}


def random_banded_ilu2(seed: int = 1002, n: int = 160_000):
    """Random banded n = 160,000, 8 band + 2 anywhere columns; ILU(2), GMRES(30)."""
    A = random_banded(n, seed)
    rng = np.random.default_rng(seed + 7919)
    b = rng.standard_normal(n)
    return {"name": f"random_banded_n{n}_ilu2", "A": A, "b": b, "k": 2, "restart": 30, "rtol": 1e-8}


# Table 3 of the paper (ILU(1) on its generated general sparse matrices):
# n -> (initial entries, final entries)
PAPER_K1_COUNTS = {40_000: (5_120_950, 196_223_519), 80_000: (6_960_983, 195_202_037),
                   160_000: (9_832_794, 198_969_083), 320_000: (14_090_553, 206_489_590)}


def paper_scale_random_ilu1(n: int = 160_000, seed: int = 1007, per_row: float | None = None):
    """Paper-scale ILU(1): a uniform random sparse matrix with Table 3's entry
    count for this n (the generator behind the table is not available, so the
    count is matched, not the matrix).  ``per_row`` overrides the entries per
    row (smaller n at the same row length, for parity tests)."""
    if per_row is None:
        nnz = PAPER_K1_COUNTS[n][0]
    else:
        nnz = int(round(per_row * n))
    A = random_uniform(n, nnz, seed)
    rng = np.random.default_rng(seed + 7919)
    b = rng.standard_normal(n)
    return {"name": f"paper_scale_random_n{n}_ilu1", "A": A, "b": b, "k": 1,
            "paper_final_entries": PAPER_K1_COUNTS.get(n, (None, None))[1]}


def conv_diff_3d_ilu(seed: int = 1003, m: int = 64, k: int = 2):
    """3-D 7-point, 64^3, eps = 1, b ~ U[-200, 200]^3 with max |b_c| > 2/h
    (cell Peclet > 1, not diagonally dominant); ILU(k) for k = 0..3, GMRES(50)."""
    h = 1.0 / (m + 1)
    s = seed
    while True:
        rng = np.random.default_rng(s)
        bvec = rng.uniform(-200.0, 200.0, size=3)
        if np.max(np.abs(bvec)) > 2.0 / h:
            break
        s += 1
    A = conv_diff_3d(m, 1.0, bvec)
    b = rng.standard_normal(A.n)
    return {"name": f"conv_diff_3d_{m}cubed_ilu{k}", "A": A, "b": b, "k": k, "restart": 50, "rtol": 1e-8}


def batched_conv_diff_2d_ilu2(seed: int = 1004, B: int = 256, m: int = 128):
    """B instances of a 2-D 5-point 128 x 128 stencil sharing one pattern,
    eps ~ U[0.5, 2], (bx, by) ~ U[-50, 50]^2 per instance; ILU(2)."""
    kids = np.random.SeedSequence(seed).spawn(B)
    eps = np.empty(B)
    bxy = np.empty((B, 2))
    rhs = np.empty((m * m, B))
    for i, ss in enumerate(kids):
        rng = np.random.default_rng(ss)
        eps[i] = rng.uniform(0.5, 2.0)
        bxy[i] = rng.uniform(-50.0, 50.0, size=2)
        rhs[:, i] = rng.standard_normal(m * m)
    A = conv_diff_2d(m, eps, bxy[:, 0], bxy[:, 1])
    return {"name": f"batched_conv_diff_2d_{m}x{m}_x{B}_ilu2", "A": A, "b": rhs, "k": 2}


def batched_stencil27_ilu(seed: int = 1008, B: int = 70, m: int = 20, k: int = 2):
    """B instances of the 27-point stencil on an m^3 grid sharing one pattern,
    eps ~ U[0.5, 2], b ~ U[-10, 10]^3 per instance, rhs ~ N(0, 1).  At
    ILU(2) and ILU(3) its rows reach 115 and 183 entries: the batched
    factorization's long-row case."""
    kids = np.random.SeedSequence(seed).spawn(B)
    base = None
    vals = []
    rhs = np.empty((m**3, B))
    for i, ss in enumerate(kids):
        rng = np.random.default_rng(ss)
        eps = rng.uniform(0.5, 2.0)
        bvec = rng.uniform(-10.0, 10.0, size=3)
        rhs[:, i] = rng.standard_normal(m**3)
        Ai = stencil27_3d(m, eps, bvec)
        base = base or Ai
        vals.append(Ai.val)
    A = CSR(base.n, base.rowptr, base.col, np.ascontiguousarray(np.stack(vals, axis=1)),
            {"kind": "stencil27_3d", "m": m, "h": base.meta["h"]})
    return {"name": f"batched_stencil27_3d_{m}cubed_x{B}_ilu{k}", "A": A, "b": rhs, "k": k}


def differentiated_conv_diff_3d_ilu1(seed: int = 1005, B: int = 16, m: int = 32):
    """B instances of a 3-D 7-point 32^3 stencil, eps ~ U[0.5, 2],
    b ~ U[-50, 50]^3 per instance, rhs and target t ~ N(0, 1); ILU(1)."""
    kids = np.random.SeedSequence(seed).spawn(B)
    n = m**3
    eps = np.empty(B)
    bv = np.empty((B, 3))
    rhs = np.empty((n, B))
    tgt = np.empty((n, B))
    for i, ss in enumerate(kids):
        rng = np.random.default_rng(ss)
        eps[i] = rng.uniform(0.5, 2.0)
        bv[i] = rng.uniform(-50.0, 50.0, size=3)
        rhs[:, i] = rng.standard_normal(n)
        tgt[:, i] = rng.standard_normal(n)
    A = conv_diff_3d(m, eps, bv)
    return {"name": f"diff_conv_diff_3d_{m}cubed_x{B}_ilu1", "A": A, "b": rhs, "t": tgt, "k": 1}
