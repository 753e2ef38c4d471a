"""Write the stored digests of the paper-scale ILU(1) factor (Table 3's 160K
size: n = 160,000 and 9,832,794 entries of A; the seeded synthetic matrix
that stands in for the paper's generated one).

Only the oracle computes anything here: its symbolic pass (Def. 2.3), its
numeric factorization (Eq. 2 / Eqs. 6a-6b) and its two substitutions (Eq. 1,
Eq. 3b).  The full factor (about 2 x 10^8 entries) is too large to store, so
what is stored is a SHA-256 digest per block of 1,000 rows: one over the
block's pattern (row lengths as int64, columns as int32, levels as uint8)
and one over its factor values (IEEE-754 binary64 bits), plus digests of the
solve results x = L~^-1 b and y = U~^-1 x per block.  A GPU test recomputes
the same digests from the GPU's pattern, factor and solves and compares all
160 blocks.

Run from the repository root:  python tests/golden/paper_scale_ilu1_digests.py
(a few minutes and about 6 GB of host memory).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_scale_ilu1_n160000.digests.txt")
BLOCK = 1000


def block_digests(rowptr, col, lev, val, x, y, block=BLOCK):
    """(pattern, values, x, y) SHA-256 hex digests of every block of rows.
    The same function runs on the oracle's arrays here and on the GPU's
    arrays in the test."""
    n = rowptr.size - 1
    out = []
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        a, b = int(rowptr[r0]), int(rowptr[r1])
        hp = hashlib.sha256()
        hp.update(np.ascontiguousarray(np.diff(rowptr[r0:r1 + 1]).astype(np.int64)).tobytes())
        hp.update(np.ascontiguousarray(col[a:b].astype(np.int32)).tobytes())
        hp.update(np.ascontiguousarray(np.minimum(lev[a:b], 255).astype(np.uint8)).tobytes())
        hv = hashlib.sha256(np.ascontiguousarray(val[a:b], dtype=np.float64).view(np.uint64).tobytes())
        hx = hashlib.sha256(np.ascontiguousarray(x[r0:r1], dtype=np.float64).view(np.uint64).tobytes())
        hy = hashlib.sha256(np.ascontiguousarray(y[r0:r1], dtype=np.float64).view(np.uint64).tobytes())
        out.append((r0, r1, hp.hexdigest(), hv.hexdigest(), hx.hexdigest(), hy.hexdigest()))
    return out


def read_digests(path=OUT):
    meta, rows = {}, []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("meta "):
                k, v = line[5:].split("=", 1)
                meta[k] = v
                continue
            r0, r1, hp, hv, hx, hy = line.split()
            rows.append((int(r0), int(r1), hp, hv, hx, hy))
    return meta, rows


def main():
    import oracle as O
    from paper_0803_0048_amd import inputs as I

    c = I.paper_scale_random_ilu1()
    A, b = c["A"], c["b"]
    t0 = time.time()
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, 1)
    t1 = time.time()
    print(f"symbolic: nnz(F) = {rpF[-1]} in {t1 - t0:.1f} s", flush=True)
    vF, bad = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
    t2 = time.time()
    print(f"numeric: bad_row {bad} in {t2 - t1:.1f} s", flush=True)
    assert bad < 0 and not np.isnan(vF).any()
    x, y = O.apply(A.n, rpF, ciF, vF, b)
    print(f"apply: {time.time() - t2:.1f} s", flush=True)
    dig = block_digests(rpF, ciF, lvF, vF, x, y)
    with open(OUT, "w") as fh:
        fh.write("# Paper-scale ILU(1) (Table 3, 160K): per block of rows r0 r1, SHA-256 of the\n")
        fh.write("# pattern (row lengths int64, columns int32, levels uint8), of the factor values\n")
        fh.write("# (binary64 bits), of x = L~^-1 b and of y = U~^-1 x.  Written by\n")
        fh.write("# tests/golden/paper_scale_ilu1_digests.py from the oracle alone.\n")
        fh.write(f"meta n={A.n}\nmeta nnz_a={A.nnz}\nmeta nnz_f={int(rpF[-1])}\nmeta seed=1007\n")
        for r in dig:
            fh.write(" ".join(str(v) for v in r) + "\n")
    print(f"wrote {OUT}: {len(dig)} blocks", flush=True)


if __name__ == "__main__":
    main()
