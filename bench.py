#!/usr/bin/env python
"""Benchmark of the gfx950 ILU(k) path on one GPU.

Workload: the random banded, diagonally dominant matrix of dimension 160,000
(8 band + 2 anywhere off-diagonals per row), ILU(2), right-preconditioned
GMRES(30) to rtol 1e-8, synthetic inputs from a fixed seed, already resident
in device memory when the timed region starts.

A step is one pass of the whole path: validation + symbolic pattern (Phase I)
+ numeric factorization (Phase II) + GMRES(30) with the triangular solves.
`value` is the headline: the numeric factorization time (median over repeated
launches, pattern precomputed, measured with HIP events around the kernel on
the stream it runs on).  Side figures: the batched graph (256 matrices of one
128 x 128 stencil pattern) and the reverse-mode pass (16 matrices of a 32^3
stencil), each next to the plain single-matrix path on the same GPU.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ILU(k) numeric factor ms & HBM GB/s frac at n=160k k=2; batched/bwd vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "random_banded_n160000_ilu2_hbm_counters.md")


def library_source_digest():
    """sha256 over the library's HIP sources and its header: what the HBM
    counters in the committed summary were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0803_0048_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "tpilu.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` ("numeric", "forward", "backward") from
    the committed FETCH_SIZE / WRITE_SIZE summary (calibrated against a plain
    copy), or None when the library has changed since those counters were taken."""
    try:
        with open(COUNTER_SUMMARY) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec.get("source_sha256") != library_source_digest():
                return None
            k = rec.get("kernels", {}).get(kernel)
            return None if k is None else int(k["bytes_per_launch"])
    return None


def model_bytes(n, nnz_a, nnz_f, nnz_l, B=1):
    """Compulsory HBM bytes (each array touched once; fills avoided).
    numeric: A's columns and values, F's columns, rowptr, diag, F written, U read once.
    forward/backward: their half of F (columns + values), rowptr, diag, vectors."""
    nnz_u = nnz_f - nnz_l
    fac = 4 * nnz_a + 4 * nnz_f + 8 * (n + 1) + 4 * n + B * (8 * nnz_a + 8 * nnz_f + 8 * nnz_u)
    fwd = 4 * nnz_l + 8 * (n + 1) + 4 * n + B * (8 * nnz_l + 16 * n)
    bwd = 4 * nnz_u + 8 * (n + 1) + 4 * n + B * (8 * nnz_u + 16 * n)
    return {"numeric": fac, "forward": fwd, "backward": bwd}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--numeric-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--extra", choices=["batched", "reverse", "stencil27", "paper_scale"],
                    help="run only this extra workload and print its figures (no bench step)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU layout is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0803_0048_amd import binding as T
    from paper_0803_0048_amd import inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies done")
        del src, dst
    if args.extra:
        ctx = T.context(0)
        if args.extra == "stencil27":
            res = stencil27_extra(T, I, torch, dev, ctx)
        elif args.extra == "paper_scale":
            res = paper_scale_extra(T, I, torch, dev, ctx)
        else:
            res = extras(T, I, torch, np, dev, ctx, only=args.extra)
        print(json.dumps({"extra": args.extra, "result": res}), flush=True)
        return
    log("building the n=160000 workload")
    cfg = I.random_banded_ilu2()
    A, k, restart, rtol = cfg["A"], cfg["k"], cfg["restart"], cfg["rtol"]
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    av = torch.from_numpy(A.val).to(dev)
    bv = torch.from_numpy(cfg["b"]).to(dev)
    ctx = T.context(0)
    maxit = 300

    def step():
        pat = T.symbolic(rp, ci, k)
        f = T.numeric(pat, av, check=False)
        x, info = T.gmres(pat, av, f, bv, restart=restart, maxit=maxit, rtol=rtol)
        return pat, f, x, info

    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for kk in range(3):
        ctx.read_timing(kk)
    log(f"timed steps x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        pat, f, x, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    ktime = {name: ctx.read_timing(kind) for kind, name in enumerate(("numeric", "forward", "backward"))}
    pinfo = pat.info
    n, nnz_a, nnz_f, nnz_l = pinfo["n"], pinfo["nnz_a"], pinfo["nnz_f"], pinfo["nnz_l"]

    # phase split of one step (symbolic and GMRES host-timed, after a sync)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    pat = T.symbolic(rp, ci, k)
    torch.cuda.synchronize()
    sym_ms = (time.perf_counter() - ts) * 1e3
    f = T.numeric(pat, av, check=False)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    _, ginfo = T.gmres(pat, av, f, bv, restart=restart, maxit=maxit, rtol=rtol)
    torch.cuda.synchronize()
    gmres_ms = (time.perf_counter() - tg) * 1e3
    for kk in range(3):
        ctx.read_timing(kk)

    # headline: numeric factorization with the pattern precomputed
    log(f"numeric factorization x{args.numeric_reps}")
    fout = torch.empty(nnz_f, dtype=torch.float64, device=dev)
    per = []
    for _ in range(args.numeric_reps):
        T.numeric(pat, av, out=fout, check=False)
        ms, cnt = ctx.read_timing(ctx.KERNEL_NUMERIC)
        per.append(ms / max(cnt, 1))
    T.check(pat)
    numeric_ms = statistics.median(per)
    # one apply, for its own kernel times
    for _ in range(5):
        T.apply(pat, fout, bv)
    fwd_ms, fwd_n = ctx.read_timing(ctx.KERNEL_FORWARD)
    bwd_ms, bwd_n = ctx.read_timing(ctx.KERNEL_BACKWARD)
    ctx.set_timing(False)

    mb = model_bytes(n, nnz_a, nnz_f, nnz_l)
    # dominant kernel over the timed steps
    tot = {name: v[0] for name, v in ktime.items()}
    dom = max(tot, key=tot.get)
    avg = {"numeric": numeric_ms, "forward": fwd_ms / max(fwd_n, 1), "backward": bwd_ms / max(bwd_n, 1)}
    achieved = mb[dom] / (avg[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(dom), "kernel": dom,
                "algorithmic_bytes_per_launch": mb[dom], "avg_launch_ms": avg[dom]}
    numeric_gbs = mb["numeric"] / (numeric_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(numeric_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random_banded_n160000_ilu2_gmres30", "n": n, "k": k, "nnz_a": nnz_a,
                   "nnz_f": nnz_f, "restart": restart, "rtol": rtol, "seed": 1002},
        "roofline": roofline,
        "numeric": {"ms": numeric_ms, "min_ms": min(per), "model_bytes": mb["numeric"],
                    "model_gbs": numeric_gbs, "frac": numeric_gbs / HBM_PEAK_GBS,
                    "updates": pinfo["n_updates"], "depth_l": pinfo["depth_l"], "depth_u": pinfo["depth_u"],
                    "n_over_depth": n / max(pinfo["depth_l"], 1)},
        "phases_ms": {"symbolic": sym_ms, "numeric": numeric_ms, "gmres": gmres_ms,
                      "gmres_iters": ginfo["iters"], "gmres_relres": ginfo["relres"],
                      "forward_kernel": avg["forward"], "backward_kernel": avg["backward"],
                      "kernel_totals_per_step": {kk: v / args.steps for kk, v in tot.items()}},
    }

    if not args.no_extras:
        out["extras"] = extras(T, I, torch, np, dev, ctx)
        out["extras"]["incomplete_inverse"] = inverse_extra(T, torch, pat, av, fout, bv, restart, rtol, maxit,
                                                            gmres_ms, ginfo, n, nnz_f, nnz_l)
        out["extras"]["stencil27"] = stencil27_extra(T, I, torch, dev, ctx)
        out["extras"]["paper_scale_ilu1"] = paper_scale_extra(T, I, torch, dev, ctx)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, k, np)
    # the paper's headline speedups, with their hardware: context for the
    # figures above (other machines, other matrices, parallel vs sequential CPU)
    out["paper_context"] = {
        "solver_speedup": {"value": 9.0, "hardware": "16 cores, 4x Intel Xeon E5520",
                           "what": "enhanced TPILU(k) (incomplete inverses) preconditioner + solve vs sequential"},
        "distributed_speedup": {"value": 50.0, "hardware": "80 cluster nodes",
                                "what": "general sparse matrix, n = 160,000, vs sequential"},
    }
    if "cpu_baseline" in out:
        out["paper_context"]["this_gpu_numeric_vs_oracle_one_core"] = out["cpu_baseline"]["value"] / numeric_ms

    print(json.dumps(out), flush=True)


def extras(T, I, torch, np, dev, ctx, only=None):
    """Batched graph and reverse mode next to the plain single-matrix path
    (``only``: "batched" or "reverse" for one of the two)."""
    res = {}
    if only not in (None, "batched"):
        return res | reverse_extra(T, I, torch, dev)
    log("batched: 256 x 128^2 ILU(2) in one graph")
    c4 = I.batched_conv_diff_2d_ilu2()
    A4 = c4["A"]
    rp4 = torch.from_numpy(A4.rowptr).to(dev)
    ci4 = torch.from_numpy(A4.col).to(dev)
    av4 = torch.from_numpy(A4.val).to(dev)
    bv4 = torch.from_numpy(c4["b"]).to(dev)
    pat4 = T.symbolic(rp4, ci4, 2)
    graph = T.BatchedGraph(pat4, av4, bv4)
    for _ in range(2):
        graph.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        graph.launch()
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / reps
    T.check(pat4)
    # plain: one instance, numeric + apply, eager
    a1 = av4[:, 0].contiguous()
    b1 = bv4[:, 0].contiguous()
    for _ in range(2):
        T.apply(pat4, T.numeric(pat4, a1, check=False), b1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        T.apply(pat4, T.numeric(pat4, a1, check=False), b1)
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / reps
    B = A4.batch
    res["batched"] = {"instances": B, "n": A4.n, "graph_ms": gms, "per_instance_ms": gms / B,
                      "plain_single_instance_ms": pms, "speedup_per_instance_vs_plain": pms / (gms / B)}
    if only == "batched":
        return res
    return res | reverse_extra(T, I, torch, dev)


def reverse_extra(T, I, torch, dev):
    """Reverse mode of 16 x 32^3 ILU(1): forward pass next to backward pass."""
    res = {}
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log("reverse mode: 16 x 32^3 ILU(1)")
    c5 = I.differentiated_conv_diff_3d_ilu1()
    A5 = c5["A"]
    pat5 = T.symbolic(torch.from_numpy(A5.rowptr).to(dev), torch.from_numpy(A5.col).to(dev), 1)
    av5 = torch.from_numpy(A5.val).to(dev)
    bv5 = torch.from_numpy(c5["b"]).to(dev)
    tv5 = torch.from_numpy(c5["t"]).to(dev)

    def fwd():
        f = T.numeric(pat5, av5, check=False)
        y, x = T.apply(pat5, f, bv5, return_x=True)
        return f, x, y

    def bwd(f, x, y):
        bbar, fbar = T.apply_adjoint(pat5, f, x, y, 2.0 * (y - tv5))
        abar, _ = T.numeric_adjoint(pat5, f, fbar)
        return abar, bbar

    f, x, y = fwd()
    bwd(f, x, y)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        f, x, y = fwd()
    e1.record()
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        bwd(f, x, y)
    e1.record()
    torch.cuda.synchronize()
    bms = e0.elapsed_time(e1) / reps
    T.check(pat5)
    res["reverse_mode"] = {"instances": A5.batch, "n": A5.n, "forward_ms": fms, "backward_ms": bms,
                           "backward_over_forward": bms / fms}
    return res


def paper_scale_extra(T, I, torch, dev, ctx):
    """ILU(1) at the size of the paper's Table 3 (n = 160,000, 9,832,794
    entries, uniform random columns; the paper's factor has 198,969,083
    entries): symbolic (host clock), numeric and the two solves (HIP events,
    median of 3).  The paper's figures for its own matrix (Tables 3 and 4,
    2008-era CPUs) are context, not a baseline."""
    log("paper-scale ILU(1), n = 160,000")
    c = I.paper_scale_random_ilu1()
    A = c["A"]
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    av = torch.from_numpy(A.val).to(dev)
    bv = torch.from_numpy(c["b"]).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pat = T.symbolic(rp, ci, 1)
    torch.cuda.synchronize()
    sym_ms = (time.perf_counter() - t0) * 1e3
    f = T.numeric(pat, av)
    y = torch.empty_like(bv)
    T.apply(pat, f, bv, out=y)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for kk in range(3):
        ctx.read_timing(kk)
    num, fwd, bwd = [], [], []
    for _ in range(3):
        T.numeric(pat, av, out=f, check=False)
        T.apply(pat, f, bv, out=y)
        num.append(ctx.read_timing(ctx.KERNEL_NUMERIC)[0])
        fwd.append(ctx.read_timing(ctx.KERNEL_FORWARD)[0])
        bwd.append(ctx.read_timing(ctx.KERNEL_BACKWARD)[0])
    ctx.set_timing(False)
    T.check(pat)
    info = pat.info
    res = {"n": info["n"], "nnz_a": info["nnz_a"], "nnz_f": info["nnz_f"],
           "paper_nnz_f": c["paper_final_entries"], "updates": info["n_updates"], "max_row": info["max_row"],
           "depth_l": info["depth_l"], "symbolic_ms": sym_ms, "numeric_ms": statistics.median(num),
           "forward_ms": statistics.median(fwd), "backward_ms": statistics.median(bwd),
           "paper_context_s": {"sequential_symbolic": 140.2, "sequential_numeric": 2112.7,
                               "tpilu_60_cores_symbolic": 2.5, "tpilu_60_cores_numeric": 64.4}}
    del pat, f, y, av, bv, rp, ci
    return res


def stencil27_extra(T, I, torch, dev, ctx):
    """The 27-point 3-D stencil of Sec. 4.2 at 50^3 (k = 0..3) and 90^3 (k = 1):
    symbolic (host clock), numeric and the two solves (HIP events around each
    kernel, median of 3)."""
    out = []
    for m, k in ((50, 0), (50, 1), (50, 2), (50, 3), (90, 1)):
        log(f"27-point stencil {m}^3 ILU({k})")
        c = I.stencil27_ilu(m=m, k=k)
        A = c["A"]
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.col).to(dev)
        av = torch.from_numpy(A.val).to(dev)
        bv = torch.from_numpy(c["b"]).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pat = T.symbolic(rp, ci, k)
        torch.cuda.synchronize()
        sym_ms = (time.perf_counter() - t0) * 1e3
        f = T.numeric(pat, av)
        y = torch.empty_like(bv)
        T.apply(pat, f, bv, out=y)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for kk in range(3):
            ctx.read_timing(kk)
        num, fwd, bwd = [], [], []
        for _ in range(3):
            T.numeric(pat, av, out=f, check=False)
            T.apply(pat, f, bv, out=y)
            num.append(ctx.read_timing(ctx.KERNEL_NUMERIC)[0])
            fwd.append(ctx.read_timing(ctx.KERNEL_FORWARD)[0])
            bwd.append(ctx.read_timing(ctx.KERNEL_BACKWARD)[0])
        ctx.set_timing(False)
        T.check(pat)
        info = pat.info
        out.append({"m": m, "k": k, "n": info["n"], "nnz_a": info["nnz_a"], "nnz_f": info["nnz_f"],
                    "depth_l": info["depth_l"], "symbolic_ms": sym_ms, "numeric_ms": statistics.median(num),
                    "forward_ms": statistics.median(fwd), "backward_ms": statistics.median(bwd)})
        del pat, f, y, av, bv, rp, ci
    return out


def inverse_extra(T, torch, pat, av, f, bv, restart, rtol, maxit, gmres_ms, ginfo, n, nnz_f, nnz_l):
    """The optional level-based incomplete inverses (Sec. 3.5) on the same
    n=160000 ILU(2) factor: building them, applying M^-1 by two products next
    to the two substitutions, GMRES(30) with them next to GMRES(30) with the
    substitutions, and BiCGSTAB (the paper's solver) with either.  The
    products are bandwidth-bound: their roofline."""
    log("incomplete inverses on the n=160000 factor")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    G = T.inverse(pat, f)
    per = []
    for _ in range(5):
        e0.record()
        T.inverse(pat, f, out=G)
        e1.record()
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1))
    y = torch.empty_like(bv)
    x = torch.empty_like(bv)
    reps = 50
    T.apply_inverse(pat, G, bv, out=y)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        T.apply_inverse(pat, G, bv, out=y)
    e1.record()
    torch.cuda.synchronize()
    app_ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(5):
        T.apply(pat, f, bv, out=x)
    e1.record()
    torch.cuda.synchronize()
    tri_ms = e0.elapsed_time(e1) / 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = T.gmres(pat, av, G, bv, restart=restart, maxit=maxit, rtol=rtol, inverse=True)
    torch.cuda.synchronize()
    gi_ms = (time.perf_counter() - t0) * 1e3
    # compulsory bytes of the two products: G and its columns once, row
    # pointers and diagonal slots, b read twice (gathered and added), x
    # written then gathered, y written
    app_bytes = 12 * nnz_f + 8 * (n + 1) + 4 * n + 5 * 8 * n
    gbs = app_bytes / (app_ms * 1e-3) / 1e9
    # BiCGSTAB (the paper's solver) with either preconditioner
    bi = {}
    for name, mval, inv in (("substitutions", f, False), ("incomplete_inverse", G, True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, binfo = T.bicgstab(pat, av, mval, bv, maxit=2 * maxit, rtol=rtol, inverse=inv)
        torch.cuda.synchronize()
        bi[name] = {"half_steps": binfo["iters"], "relres": binfo["relres"],
                    "ms": (time.perf_counter() - t0) * 1e3}
    return {"bicgstab": bi,
            "inverse_ms": statistics.median(per), "apply_ms": app_ms, "triangular_apply_ms": tri_ms,
            "apply_speedup": tri_ms / app_ms,
            "apply_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": app_bytes},
            "gmres_iters": info["iters"], "gmres_relres": info["relres"], "gmres_ms": gi_ms,
            "gmres_with_substitutions": {"iters": ginfo["iters"], "ms": gmres_ms}}


def cpu_baseline(A, k, np):
    """The oracle (sequential, one host core) on the headline: the numeric
    factorization of the same n=160000 ILU(2) workload, pattern precomputed;
    median of 3 runs."""
    import oracle as O

    log("cpu baseline: oracle numeric factorization x3")
    O.build(force=False)
    rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, k)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
        times.append((time.perf_counter() - t0) * 1e3)
    return {"value": statistics.median(times), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": "full numeric factorization of the n=160000 ILU(2) workload, median of 3"}


if __name__ == "__main__":
    main()
