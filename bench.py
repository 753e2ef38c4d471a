#!/usr/bin/env python
"""Benchmark of the gfx950 ILU(k) path on one GPU.

Headline workload: the random banded, diagonally dominant matrix of dimension
160,000 (8 band + 2 anywhere off-diagonals per row), ILU(2), right-
preconditioned GMRES(30) to rtol 1e-8, synthetic inputs from a fixed seed,
already resident in device memory when the timed region starts.

A step is one pass of the whole path on that workload: validation + symbolic
pattern (Phase I) + numeric factorization (Phase II) + GMRES(30) with the
triangular solves.  `value` is the headline: the numeric factorization time
(median over repeated calls, pattern precomputed, HIP events on the stream it
runs on around the pending-marker fill of F and the elimination kernel).

Also reported, each next to its algorithmic-bytes roofline and, where the
paper's method defines it, the oracle on the host's cores with a bitwise
comparison of the results:
  * every phase (symbolic, numeric, forward / backward solve, apply, GMRES)
    of the other single-matrix workloads: the 64 x 64 2-D stencil ILU(1) and
    the 64^3 3-D convection-dominated stencil ILU(0..3);
  * the batched graph (256 matrices of one 128 x 128 pattern) and the
    reverse-mode pass (16 matrices of a 32^3 stencil), next to the plain
    single-matrix path;
  * the 27-point stencil, the paper-scale ILU(1) matrix of Table 3's size and
    the incomplete-inverse variant (extras);
  * latency floors: the dependency critical path (row-to-row hand-offs) times
    the hand-off time measured by a probe in the same run.

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
    """sha256 over the library's HIP sources (kernels and runtime): what the
    HBM counters in the committed summary were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0803_0048_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (calibrated against a plain copy), or None when the
    library has changed since those counters were taken."""
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
    """Algorithmic (compulsory) HBM bytes, each array touched once:
    numeric  4 nnzA + 4 nnzF + 8(n+1) + 4n + B(8 nnzA + 8 nnzF + 8 nnzU)
             (A's columns and values, F's columns, rowptr, diagonal slots, F
             written, U~ read once as pivot rows);
    forward  4 nnzL + 8(n+1) + 4n + B(8 nnzL + 16n)   (L~ half, b read, x written);
    backward 4 nnzU + 8(n+1) + 4n + B(8 nnzU + 16n)   (U~ half, x read, y written);
    apply    4 nnzF + 8(n+1) + 4n + B(8 nnzF + 32n)   (both, structure read once)."""
    nnz_u = nnz_f - nnz_l
    fac = 4 * nnz_a + 4 * nnz_f + 8 * (n + 1) + 4 * n + B * (8 * nnz_a + 8 * nnz_f + 8 * nnz_u)
    fwd = 4 * nnz_l + 8 * (n + 1) + 4 * n + B * (8 * nnz_l + 16 * n)
    bwd = 4 * nnz_u + 8 * (n + 1) + 4 * n + B * (8 * nnz_u + 16 * n)
    app = 4 * nnz_f + 8 * (n + 1) + 4 * n + B * (8 * nnz_f + 32 * n)
    return {"numeric": fac, "forward": fwd, "backward": bwd, "apply": app}


def roof(nbytes, ms, kernel=None):
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    r = {"bound": "hbm", "achieved": round(gbs, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": int(nbytes), "ms": ms}
    if kernel:
        r["kernel"] = kernel
    return r


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def oracle_threads():
    """Threads for the oracle runs that spread whole instances over the host
    (at most 16: the host share of one GPU)."""
    return max(1, min(16, host_info()["usable_cores"]))


def bits_equal(np, got, want):
    """Bitwise equality, a NaN matching any NaN (its sign and payload are not
    part of the result)."""
    g = np.ascontiguousarray(got, dtype=np.float64)
    w = np.ascontiguousarray(want, dtype=np.float64)
    if g.shape != w.shape:
        return False
    same = g.view(np.uint64) == w.view(np.uint64)
    return bool(np.all(same | (np.isnan(g) & np.isnan(w))))


# ----------------------------------------------------------------------------------
# one single-matrix workload on the GPU, phase by phase
# ----------------------------------------------------------------------------------
def gpu_phases(T, torch, ctx, A, b, k, restart, rtol, maxit, reps=5, sym_reps=3):
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    av = torch.from_numpy(A.val).to(dev)
    bv = torch.from_numpy(b).to(dev)
    sym = []
    pat = None
    for _ in range(sym_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pat = T.symbolic(rp, ci, k)
        torch.cuda.synchronize()
        sym.append((time.perf_counter() - t0) * 1e3)
    info = pat.info
    f = T.numeric(pat, av)
    y = torch.empty_like(bv)
    T.apply(pat, f, bv, out=y)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for kk in range(3):
        ctx.read_timing(kk)
    num, fwd, bwd, app = [], [], [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        T.numeric(pat, av, out=f, check=False)
        num.append(ctx.read_timing(ctx.KERNEL_NUMERIC)[0])
        e0.record()
        T.apply(pat, f, bv, out=y)
        e1.record()
        torch.cuda.synchronize()
        app.append(e0.elapsed_time(e1))
        fwd.append(ctx.read_timing(ctx.KERNEL_FORWARD)[0])
        bwd.append(ctx.read_timing(ctx.KERNEL_BACKWARD)[0])
    ctx.set_timing(False)
    T.check(pat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, ginfo = T.gmres(pat, av, f, bv, restart=restart, maxit=maxit, rtol=rtol)
    torch.cuda.synchronize()
    gm_ms = (time.perf_counter() - t0) * 1e3
    mb = model_bytes(info["n"], info["nnz_a"], info["nnz_f"], info["nnz_l"])
    med = {"numeric": statistics.median(num), "forward": statistics.median(fwd),
           "backward": statistics.median(bwd), "apply": statistics.median(app)}
    res = {"n": info["n"], "k": k, "nnz_a": info["nnz_a"], "nnz_f": info["nnz_f"], "updates": info["n_updates"],
           "depth_l": info["depth_l"], "depth_u": info["depth_u"],
           "symbolic_ms": statistics.median(sym), "numeric_ms": med["numeric"], "forward_ms": med["forward"],
           "backward_ms": med["backward"], "apply_ms": med["apply"], "gmres_ms": gm_ms,
           "gmres_restart": restart, "gmres_iters": ginfo["iters"], "gmres_relres": ginfo["relres"],
           "roofline": {ph: roof(mb[ph], med[ph]) for ph in ("numeric", "forward", "backward", "apply")}}
    return res, {"pat": pat, "f": f, "y": y, "x": x, "ginfo": ginfo, "av": av, "bv": bv}


def oracle_phases(O, np, A, b, k, restart, rtol, maxit, numeric_reps=1):
    """The oracle, one host core, the same phases."""
    t0 = time.perf_counter()
    rpF, ciF, lvF = O.symbolic(A.n, A.rowptr, A.col, k)
    t1 = time.perf_counter()
    num = []
    vF = None
    for _ in range(numeric_reps):
        ta = time.perf_counter()
        vF, _ = O.numeric(A.n, A.rowptr, A.col, A.val, rpF, ciF)
        num.append((time.perf_counter() - ta) * 1e3)
    t2 = time.perf_counter()
    x, y = O.apply(A.n, rpF, ciF, vF, b)
    t3 = time.perf_counter()
    r = O.gmres(A.n, A.rowptr, A.col, A.val, rpF, ciF, vF, b, restart=restart, maxit=maxit, rtol=rtol)
    t4 = time.perf_counter()
    times = {"symbolic_ms": (t1 - t0) * 1e3, "numeric_ms": statistics.median(num), "apply_ms": (t3 - t2) * 1e3,
             "gmres_ms": (t4 - t3) * 1e3, "cores": 1}
    return times, {"rpF": rpF, "ciF": ciF, "vF": vF, "y": y, "gmres": r}


def bitwise(np, g, ref):
    ex = g["pat"].export()
    return {
        "pattern": bool(np.array_equal(ex["rowptr"].cpu().numpy(), ref["rpF"])
                        and np.array_equal(ex["col"].cpu().numpy(), ref["ciF"])),
        "factor": bits_equal(np, g["f"].cpu().numpy(), ref["vF"]),
        "solve": bits_equal(np, g["y"].cpu().numpy(), ref["y"]),
        "gmres": (g["ginfo"]["iters"] == ref["gmres"]["iters"]
                  and bits_equal(np, g["x"].cpu().numpy(), ref["gmres"]["x"])),
    }


# ----------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--numeric-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--step-only", action="store_true",
                    help="only the timed step and the numeric / apply timings (for profiling one workload): "
                         "no latency floors, no other workloads, no extras")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--extra", choices=["batched", "reverse", "stencil27", "paper_scale", "conv_diff_3d",
                                        "conv_diff_2d", "probe"],
                    help="run only this workload and print its figures (no bench step)")
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
    ctx = T.context(0)
    if args.extra:
        res = run_extra(args.extra, T, I, torch, np, dev, ctx, oracle=not args.no_cpu_baseline)
        print(json.dumps({"extra": args.extra, "result": res}), flush=True)
        return

    log("building the n=160000 workload")
    cfg = I.random_banded_ilu2()
    A, k, restart, rtol = cfg["A"], cfg["k"], cfg["restart"], cfg["rtol"]
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    av = torch.from_numpy(A.val).to(dev)
    bv = torch.from_numpy(cfg["b"]).to(dev)
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
    for _ in range(args.steps):
        pat, f, x, info = step()
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
    xg, ginfo = T.gmres(pat, av, f, bv, restart=restart, maxit=maxit, rtol=rtol)
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
    # the same factorization with the update of Eq. 6b as one fused
    # multiply-add (the optional rounding; compared with the oracle's below)
    ffused, fused_ms = None, None
    if not args.step_only:
        log(f"numeric factorization, fused update, x{args.numeric_reps}")
        ffused = torch.empty_like(fout)
        perf = []
        ctx.set_fused(True)
        try:
            for _ in range(args.numeric_reps):
                T.numeric(pat, av, out=ffused, check=False)
                ms, cnt = ctx.read_timing(ctx.KERNEL_NUMERIC)
                perf.append(ms / max(cnt, 1))
            T.check(pat)
        finally:
            ctx.set_fused(False)
        fused_ms = statistics.median(perf)
    # applies, for their own kernel times
    yout = torch.empty_like(bv)
    xout = torch.empty_like(bv)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    app = []
    for _ in range(5):
        e0.record()
        T.apply(pat, fout, bv, out=yout)
        e1.record()
        torch.cuda.synchronize()
        app.append(e0.elapsed_time(e1))
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

    # latency floors: dependency critical path x measured hand-off time
    log("latency floors: hand-off probes and the elimination's critical path")
    floors = None if args.step_only else latency_floors(T, ctx, pat, pinfo, avg, n)

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
                    "timed_region": "pending-marker fill of F + elimination kernel",
                    "fused_update_ms": fused_ms,
                    "updates": pinfo["n_updates"], "depth_l": pinfo["depth_l"], "depth_u": pinfo["depth_u"],
                    "n_over_depth": n / max(pinfo["depth_l"], 1)},
        "phases_ms": {"symbolic": sym_ms, "numeric": numeric_ms, "gmres": gmres_ms,
                      "gmres_iters": ginfo["iters"], "gmres_relres": ginfo["relres"],
                      "forward_kernel": avg["forward"], "backward_kernel": avg["backward"],
                      "apply": statistics.median(app),
                      "kernel_totals_per_step": {kk: v / args.steps for kk, v in tot.items()}},
        "phase_rooflines": {ph: roof(mb[ph], v) for ph, v in
                            (("numeric", numeric_ms), ("forward", avg["forward"]), ("backward", avg["backward"]),
                             ("apply", statistics.median(app)))},
        "latency_floor": floors,
        "host": host_info(),
    }

    # the other single-matrix workloads, every phase, GPU next to the oracle
    out["workloads"] = {}
    for name, c in () if args.step_only else (
            ("conv_diff_2d_64x64_ilu1", I.conv_diff_2d_64x64_ilu1()),
            *((f"conv_diff_3d_64cubed_ilu{kk}", I.conv_diff_3d_ilu(k=kk)) for kk in (0, 1, 2, 3))):
        log(f"workload {name}")
        out["workloads"][name] = single_workload(T, I, torch, np, ctx, c, oracle=not args.no_cpu_baseline)

    if not args.no_extras and not args.step_only:
        out["extras"] = {}
        out["extras"]["batched"] = batched_extra(T, I, torch, np, dev, ctx, oracle=not args.no_cpu_baseline)
        out["extras"]["reverse_mode"] = reverse_extra(T, I, torch, np, dev, oracle=not args.no_cpu_baseline)
        out["extras"]["incomplete_inverse"] = inverse_extra(T, torch, pat, av, fout, bv, restart, rtol, maxit,
                                                            gmres_ms, ginfo, n, nnz_f, nnz_l)
        out["extras"]["stencil27"] = stencil27_extra(T, I, torch, dev, ctx)
        out["extras"]["paper_scale_ilu1"] = paper_scale_extra(T, I, torch, dev, ctx)

    if not args.no_cpu_baseline:
        cb, match = cpu_baseline(np, A, k, cfg["b"], restart, rtol, maxit, pat, fout, yout, xg, ginfo, bv, T,
                                 ffused)
        out["cpu_baseline"] = cb
        out["bitwise_match"] = match
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


def latency_floors(T, ctx, pat, pinfo, avg, n):
    """Critical path x hand-off time.  Numeric: the elimination's critical
    path in row-to-row hand-offs (the dataflow kernel in hop-count mode) x one
    device-wide hand-off (agent-scope store, agent-scope poll; the numeric
    kernels run on every XCD).  Solves: the row-level dependency depth minus
    one x one hand-off on one XCD (where the narrow solves run)."""
    rt_dev = T.handoff_probe(False, rounds=4000)
    rt_xcd = T.handoff_probe(True, rounds=4000)
    hop_dev, hop_xcd = rt_dev / 2.0, rt_xcd / 2.0
    res = {"handoff_round_trip_ns": {"two_xcds": rt_dev, "one_xcd": rt_xcd},
           "hop_ns": {"two_xcds": hop_dev, "one_xcd": hop_xcd}}
    try:
        hops = int(round(T.numeric_critical_path(pat, 1.0, 0.0)))
        steps = int(round(T.numeric_critical_path(pat, 0.0, 1.0)))
    except T.TpiluError:
        hops = steps = None
    if hops is not None:
        res["numeric_longest_l_chain"] = steps
        fl = hops * hop_dev * 1e-6
        res["numeric"] = {"critical_path_hops": hops, "floor_ms": fl, "achieved_ms": avg["numeric"],
                          "achieved_over_floor": avg["numeric"] / fl if fl > 0 else None,
                          "achieved_ns_per_hop": avg["numeric"] * 1e6 / max(hops, 1)}
    for ph, depth in (("forward", pinfo["depth_l"]), ("backward", pinfo["depth_u"])):
        hops_s = max(depth - 1, 0)
        fl = hops_s * hop_xcd * 1e-6
        res[ph] = {"critical_path_hops": hops_s, "floor_ms": fl, "achieved_ms": avg[ph],
                   "achieved_over_floor": avg[ph] / fl if fl > 0 else None,
                   "achieved_ns_per_hop": avg[ph] * 1e6 / max(hops_s, 1)}
    return res


def single_workload(T, I, torch, np, ctx, c, oracle=True):
    A, b, k = c["A"], c["b"], c["k"]
    restart = c.get("restart", 30)
    rtol = c.get("rtol", 1e-8)
    res, g = gpu_phases(T, torch, ctx, A, b, k, restart, rtol, 3000)
    if oracle:
        import oracle as O
        ot, ref = oracle_phases(O, np, A, b, k, restart, rtol, 3000)
        res["oracle"] = ot
        res["bitwise_match"] = bitwise(np, g, ref)
    del g
    return res


def run_extra(name, T, I, torch, np, dev, ctx, oracle=True):
    if name == "stencil27":
        return stencil27_extra(T, I, torch, dev, ctx)
    if name == "paper_scale":
        return paper_scale_extra(T, I, torch, dev, ctx)
    if name == "batched":
        return batched_extra(T, I, torch, np, dev, ctx, oracle=oracle)
    if name == "reverse":
        return reverse_extra(T, I, torch, np, dev, oracle=oracle)
    if name == "probe":
        return {"round_trip_ns": {"two_xcds": T.handoff_probe(False, rounds=4000),
                                  "one_xcd": T.handoff_probe(True, rounds=4000)}}
    if name == "conv_diff_2d":
        return single_workload(T, I, torch, np, ctx, I.conv_diff_2d_64x64_ilu1(), oracle=oracle)
    return {f"k{kk}": single_workload(T, I, torch, np, ctx, I.conv_diff_3d_ilu(k=kk), oracle=oracle)
            for kk in (0, 1, 2, 3)}


def _threads_map(fn, items):
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=oracle_threads()) as ex:
        return list(ex.map(fn, items))


def batched_extra(T, I, torch, np, dev, ctx, oracle=True):
    """256 x 128^2 ILU(2): all numeric factorizations + all solves in one
    captured graph, next to one instance on its own; roofline of the graph
    from the batched algorithmic bytes (B = 256); the oracle over every host
    core (instances spread over threads, each sequential) with every instance
    compared bit for bit."""
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
    graph.check()
    # the two halves of the graph, eagerly, for their own rooflines
    ctx.set_timing(True)
    for kk in range(3):
        ctx.read_timing(kk)
    fb = torch.empty_like(graph.f_val)
    yb = torch.empty_like(bv4)
    num, fw, bw = [], [], []
    for _ in range(5):
        T.numeric(pat4, av4, out=fb, check=False)
        T.apply(pat4, fb, bv4, out=yb)
        num.append(ctx.read_timing(ctx.KERNEL_NUMERIC)[0])
        fw.append(ctx.read_timing(ctx.KERNEL_FORWARD)[0])
        bw.append(ctx.read_timing(ctx.KERNEL_BACKWARD)[0])
    ctx.set_timing(False)
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
    info = pat4.info
    mb = model_bytes(info["n"], info["nnz_a"], info["nnz_f"], info["nnz_l"], B=B)
    gbytes = mb["numeric"] + mb["apply"]
    res = {"instances": B, "n": A4.n, "nnz_f": info["nnz_f"], "graph_ms": gms, "per_instance_ms": gms / B,
           "plain_single_instance_ms": pms, "speedup_per_instance_vs_plain": pms / (gms / B),
           "roofline": roof(gbytes, gms, "graph: numeric + apply, 256 instances"),
           "numeric_roofline": roof(mb["numeric"], statistics.median(num), "numeric (batched)"),
           "forward_roofline": roof(mb["forward"], statistics.median(fw), "forward (batched)"),
           "backward_roofline": roof(mb["backward"], statistics.median(bw), "backward (batched)"),
           "graph_kernels": "fill the U slots of F, fill x, factorization with the forward substitution fused in, fill y, "
                            "backward substitution",
           "depth_l": info["depth_l"]}
    res["long_rows"] = batched_long_rows(T, I, torch, np, dev, oracle=oracle)
    if oracle:
        import oracle as O

        log(f"batched: oracle on {oracle_threads()} threads")
        rpF, ciF, _ = O.symbolic(A4.n, A4.rowptr, A4.col, 2)

        def one(i):
            vF, _ = O.numeric(A4.n, A4.rowptr, A4.col, np.ascontiguousarray(A4.val[:, i]), rpF, ciF)
            _, y = O.apply(A4.n, rpF, ciF, vF, np.ascontiguousarray(c4["b"][:, i]))
            return vF, y

        t0 = time.perf_counter()
        outs = _threads_map(one, range(B))
        oms = (time.perf_counter() - t0) * 1e3
        fh = graph.f_val.cpu().numpy()
        yh = graph.y.cpu().numpy()
        ok = all(bits_equal(np, fh[:, i], outs[i][0]) and bits_equal(np, yh[:, i], outs[i][1]) for i in range(B))
        res["oracle"] = {"ms": oms, "cores": oracle_threads(), "what": "256 x (numeric + apply), one instance "
                         "per thread at a time, each sequential"}
        res["bitwise_match_all_instances"] = ok
    return res


def batched_long_rows(T, I, torch, np, dev, oracle=True):
    """70 x 27-point 20^3 ILU(2) (rows of up to 115 entries: the working rows
    live in global memory) in one graph; roofline from the batched
    algorithmic bytes; every instance against the oracle."""
    log("batched: 70 x 27-point 20^3 ILU(2) in one graph (long rows)")
    c = I.batched_stencil27_ilu(B=70, k=2)
    A = c["A"]
    pat = T.symbolic(torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.col).to(dev), 2)
    av = torch.from_numpy(A.val).to(dev)
    bv = torch.from_numpy(c["b"]).to(dev)
    graph = T.BatchedGraph(pat, av, bv)
    graph.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        graph.launch()
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / reps
    graph.check()
    info = pat.info
    B = A.batch
    mb = model_bytes(info["n"], info["nnz_a"], info["nnz_f"], info["nnz_l"], B=B)
    res = {"instances": B, "n": A.n, "nnz_f": info["nnz_f"], "max_row": info["max_row"], "graph_ms": gms,
           "roofline": roof(mb["numeric"] + mb["apply"], gms, "graph: numeric + apply, 70 instances"),
           "depth_l": info["depth_l"]}
    if oracle:
        import oracle as O

        rpF, ciF, _ = O.symbolic(A.n, A.rowptr, A.col, 2)
        fh, yh = graph.f_val.cpu().numpy(), graph.y.cpu().numpy()
        ok = True
        for i in range(B):
            vF, _ = O.numeric(A.n, A.rowptr, A.col, np.ascontiguousarray(A.val[:, i]), rpF, ciF)
            _, y = O.apply(A.n, rpF, ciF, vF, np.ascontiguousarray(c["b"][:, i]))
            ok = ok and bits_equal(np, fh[:, i], vF) and bits_equal(np, yh[:, i], y)
        res["bitwise_match_all_instances"] = ok
    return res


def reverse_extra(T, I, torch, np, dev, oracle=True):
    """Reverse mode of 16 x 32^3 ILU(1): forward pass next to backward pass,
    each with its algorithmic-bytes roofline; the oracle over every host core
    with every instance's gradients compared bit for bit."""
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
        abar, bbar = bwd(f, x, y)
    e1.record()
    torch.cuda.synchronize()
    bms = e0.elapsed_time(e1) / reps
    T.check(pat5)
    info = pat5.info
    B, n, nf, na = A5.batch, info["n"], info["nnz_f"], info["nnz_a"]
    mb = model_bytes(n, na, nf, info["nnz_l"], B=B)
    # backward algorithmic bytes: F read by the transposed solves and by the
    # reverse sweep, Fbar written, read and rewritten, abar written, the
    # vectors x, y, ybar read and bbar written (plus z), structure once each
    bwd_bytes = B * (5 * 8 * nf + 8 * na + 40 * n) + 2 * 4 * nf + 2 * (8 * (n + 1) + 4 * n)
    res = {"instances": B, "n": A5.n, "forward_ms": fms, "backward_ms": bms, "backward_over_forward": bms / fms,
           "forward_roofline": roof(mb["numeric"] + mb["apply"], fms, "numeric + apply (16 instances)"),
           "backward_roofline": roof(bwd_bytes, bms, "apply_adjoint + numeric_adjoint (16 instances)")}
    if oracle:
        import oracle as O

        log(f"reverse mode: oracle on {oracle_threads()} threads")
        rpF, ciF, _ = O.symbolic(A5.n, A5.rowptr, A5.col, 1)

        def one(i):
            vals = np.ascontiguousarray(A5.val[:, i])
            vF, _ = O.numeric(A5.n, A5.rowptr, A5.col, vals, rpF, ciF)
            xo, yo = O.apply(A5.n, rpF, ciF, vF, np.ascontiguousarray(c5["b"][:, i]))
            bb, Fb = O.apply_adjoint(A5.n, rpF, ciF, vF, xo, yo, 2.0 * (yo - c5["t"][:, i]))
            ab, _ = O.numeric_adjoint(A5.n, A5.rowptr, A5.col, rpF, ciF, vF, Fb)
            return ab, bb

        t0 = time.perf_counter()
        outs = _threads_map(one, range(B))
        oms = (time.perf_counter() - t0) * 1e3
        ah, bh = abar.cpu().numpy(), bbar.cpu().numpy()
        ok = all(bits_equal(np, ah[:, i], outs[i][0]) and bits_equal(np, bh[:, i], outs[i][1]) for i in range(B))
        res["oracle"] = {"ms": oms, "cores": oracle_threads(),
                         "what": "16 x (numeric + apply + both adjoints), one instance per thread at a time"}
        res["bitwise_match_all_instances"] = ok
    return res


def paper_scale_extra(T, I, torch, dev, ctx):
    """ILU(1) at the size of the paper's Table 3 (n = 160,000, 9,832,794
    entries, uniform random columns; the paper's factor has 198,969,083
    entries): symbolic (host clock), numeric and the two solves (HIP events,
    median of 3), with rooflines.  The paper's figures for its own matrix
    (Tables 3 and 4, 2008-era CPUs) are context, not a baseline."""
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
    mb = model_bytes(info["n"], info["nnz_a"], info["nnz_f"], info["nnz_l"])
    med = {"numeric": statistics.median(num), "forward": statistics.median(fwd), "backward": statistics.median(bwd)}
    res = {"n": info["n"], "nnz_a": info["nnz_a"], "nnz_f": info["nnz_f"],
           "paper_nnz_f": c["paper_final_entries"], "updates": info["n_updates"], "max_row": info["max_row"],
           "depth_l": info["depth_l"], "symbolic_ms": sym_ms, "numeric_ms": med["numeric"],
           "forward_ms": med["forward"], "backward_ms": med["backward"],
           "roofline": {ph: roof(mb[ph], med[ph]) for ph in med},
           "paper_context_s": {"sequential_symbolic": 140.2, "sequential_numeric": 2112.7,
                               "tpilu_60_cores_symbolic": 2.5, "tpilu_60_cores_numeric": 64.4}}
    del pat, f, y, av, bv, rp, ci
    return res


def stencil27_extra(T, I, torch, dev, ctx):
    """The 27-point 3-D stencil of Sec. 4.2 at 50^3 (k = 0..3) and 90^3 (k = 1):
    symbolic (host clock), numeric and the two solves (HIP events around each
    kernel, median of 3), with rooflines."""
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
        mb = model_bytes(info["n"], info["nnz_a"], info["nnz_f"], info["nnz_l"])
        med = {"numeric": statistics.median(num), "forward": statistics.median(fwd),
               "backward": statistics.median(bwd)}
        out.append({"m": m, "k": k, "n": info["n"], "nnz_a": info["nnz_a"], "nnz_f": info["nnz_f"],
                    "depth_l": info["depth_l"], "symbolic_ms": sym_ms, "numeric_ms": med["numeric"],
                    "forward_ms": med["forward"], "backward_ms": med["backward"],
                    "roofline": {ph: roof(mb[ph], med[ph]) for ph in med}})
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
            "apply_roofline": roof(app_bytes, app_ms, "two products of the incomplete inverses"),
            "gmres_iters": info["iters"], "gmres_relres": info["relres"], "gmres_ms": gi_ms,
            "gmres_with_substitutions": {"iters": ginfo["iters"], "ms": gmres_ms}}


def cpu_baseline(np, A, k, b, restart, rtol, maxit, pat, fout, yout, xg, ginfo, bv, T, ffused=None):
    """The oracle (sequential, one host core) on the headline workload: every
    phase once, the numeric factorization (the headline) median of 3, and the
    GPU's factor, solve and GMRES iterate compared with the oracle's bit for
    bit; with ffused, the GPU's factor in the fused-update mode against the
    oracle's fused elimination too."""
    import oracle as O

    log("cpu baseline: oracle on the n=160000 ILU(2) workload (numeric x3)")
    O.build(force=False)
    times, ref = oracle_phases(O, np, A, b, k, restart, rtol, maxit, numeric_reps=3)
    T.apply(pat, fout, bv, out=yout)
    g = {"pat": pat, "f": fout, "y": yout, "x": xg, "ginfo": ginfo}
    match = bitwise(np, g, ref)
    if ffused is not None:
        vFf, _ = O.numeric(A.n, A.rowptr, A.col, A.val, ref["rpF"], ref["ciF"], fused=True)
        match["factor_fused_update"] = bits_equal(np, ffused.cpu().numpy(), vFf)
    hi = host_info()
    cb = {"value": times["numeric_ms"], "unit": "ms", "cores": 1, "kind": "oracle",
          "sample": "full numeric factorization of the n=160000 ILU(2) workload, median of 3 (pattern "
                    "precomputed); its other phases once",
          "phases_ms": times, "cpu_model": hi["cpu_model"], "nproc": hi["nproc"],
          "usable_cores": hi["usable_cores"]}
    return cb, match


if __name__ == "__main__":
    main()
