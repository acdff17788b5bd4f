#!/usr/bin/env python3
"""Benchmark: numeric supernodal Cholesky factor + solve on one MI355X.

Default workload (the headline): the 3D 27-point, 3-dof elasticity-like
operator on a 48^3 grid (n = 331,776, 2.11e12 flops, kappa ~1e8), 4
right-hand sides, geometric nested dissection.  One step = a plain FP64
refactorization from the values resident in HBM (assemble, panel POTRF/TRSM,
trailing and scatter SYRK/GEMM updates) + the forward and backward solves of
the 4 right-hand sides.  value = FP64 factor GFLOP/s = sum_j colcount_j^2 /
mean factor device time.  Beside it ("vs plain FP64"): the FP32
factorization with FP64 iterative refinement to a backward error of 1e-12
(factor ms, refined-solve p50/p99, steps, backward error).

The printed JSON line also carries a live roofline of the dominant kernel
class (HIP events around each of its launches, in a profiled pass of the
same steps) and the CPU oracle timed on a bounded sample of the same matrix
(whole subtrees of its elimination tree), on all the host's cores (the
oracle's deterministic multi-threaded mode) and on one.

Other workloads: --workload grid3d60 (the 60^3 7-point operator, FP64),
grid2d64, batch512, serving, copy (counter calibration).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--solves", type=int, default=200, help="solves timed for the solve p50/p99 (headline, 60^3)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--grid", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-fp64", action="store_true",
                    help="elast48: the plain FP64 steps only, without the FP32 and BF16-update legs (profiling runs)")
    ap.add_argument("--no-task-baseline", action="store_true",
                    help="skip the paper's task-parallel host factorization of the headline matrix")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target wall time of the oracle's all-cores sample (the one-core sample takes about "
                         "a third of it)")
    ap.add_argument("--workload", default="elast48",
                    choices=["elast48", "grid3d60", "grid2d64", "batch512", "serving", "copy", "cpu_tasks"],
                    help="elast48: the headline, 48^3 elasticity, FP64 factor + solve with the FP32 + FP64 "
                         "refinement leg beside it (default); grid3d60: 60^3 7-point FP64 factor + solve; "
                         "grid2d64: small-system latency; batch512: 512 systems in one schedule; "
                         "serving: request loop; cpu_tasks: the paper's task-parallel host factorization "
                         "(every strategy) on configurations 1-3, no GPU")
    ap.add_argument("--tuning", default="auto", choices=["auto", "default"],
                    help="schedule cut-offs: the autotuner's cache entry for this workload (auto), else defaults")
    ap.add_argument("--seed", type=int, default=0, help="seed of the synthetic inputs (configs 1-3)")
    ap.add_argument("--graph", default="on", choices=["on", "off"],
                    help="replay the factorization from a captured HIP graph (on) or launch it eagerly")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: arrivals per second (0: sweep)")
    ap.add_argument("--requests", type=int, default=300, help="serving: requests per rate")
    ap.add_argument("--capacity-sweep", action="store_true",
                    help="serving: measure capacity (all requests at once), then sweep 0.25-1.1x of it")
    ap.add_argument("--serving-budget-gb", type=float, default=64.0,
                    help="serving: HBM budget for resident factors and work areas (GiB)")
    ap.add_argument("--serving-handover", default="off", choices=["on", "off"],
                    help="serving: the factorizations' in-launch TRSM hand-over (off: no waits inside a launch)")
    return ap.parse_args()


def _subtree_firsts(S):
    """First supernode of each supernode's subtree (a contiguous range in
    postorder ending at the supernode)."""
    sparent = S.sparent
    first = np.arange(S.nsuper, dtype=np.int64)
    for t in range(S.nsuper):
        p = int(sparent[t])
        if p >= 0 and first[t] < first[p]:
            first[p] = first[t]
    return first


def cpu_baseline(s, target_s, name):
    """The oracle (plain C, FP64, no BLAS) on whole subtrees of the same
    matrix's elimination tree: (a) on all host cores (its deterministic
    multi-threaded mode: whole supernodes per thread, level by level), on the
    subtrees of one etree level whose flops fill about target_s; (b) on one
    core, on one subtree of about target_s / 3.  The rate is the sample's
    flops (sum of squared column counts over its columns) over wall time."""
    import oracle
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    cc = S.colcount.astype(np.float64)
    cum = np.concatenate([[0.0], np.cumsum(cc ** 2)])
    sp = S.super_ptr
    first = _subtree_firsts(S)
    sub_flops = cum[sp[1:]] - cum[sp[first]]
    lev = S.level
    one_rate = 1.0e10                    # about what one core reaches on these levels
    all_rate = one_rate * threads * 0.8  # level sync and the top of each subtree cost some parallelism

    def pick(budget, min_roots):
        for L in range(S.sizes["nlevels"] - 1, -1, -1):
            roots = np.nonzero(lev == L)[0]
            if roots.size < min_roots:
                continue
            picks, fl = [], 0.0
            for r in roots:
                if fl + sub_flops[r] > budget and picks:
                    break
                picks.append(int(r))
                fl += sub_flops[r]
            if fl <= budget * 1.3 and len(picks) >= min_roots:
                return L, picks, fl
        return None

    L, roots, fl = pick(target_s * all_rate, min(threads, 8))
    t0 = time.perf_counter()
    S.factor_forest(s.values, roots, threads=threads)
    dt = time.perf_counter() - t0
    used = S.threads_used
    L1, roots1, fl1 = pick(target_s / 3 * one_rate, 1)
    r1 = roots1[:1]
    fl1 = float(sub_flops[r1[0]])
    t0 = time.perf_counter()
    S.factor_subtree(s.values, r1[0])
    dt1 = time.perf_counter() - t0
    import platform
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(fl / dt / 1e9, 4), "unit": "GFLOP/s", "cores": used, "kind": "oracle",
            "sample": f"{len(roots)} whole subtrees rooted at level {L} of the {name} elimination tree, "
                      f"{fl:.3e} flops (sum of squared column counts), {dt:.1f} s on {used} threads "
                      f"(deterministic multi-threaded mode)",
            "seconds": round(dt, 2), "host_cpus": os.cpu_count(), "cpu_model": cpu_model or platform.processor(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "single_core": {"value": round(fl1 / dt1 / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
                            "sample": f"1 whole subtree rooted at level {L1}, {fl1:.3e} flops, {dt1:.1f} s",
                            "seconds": round(dt1, 2)}}


def progress(msg):
    """A line on stderr as each stage of the run ends."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_backward_error(n, colptr, rowidx, values, X, B) -> float:
    """Normwise backward error of the solution X, max over the right-hand
    sides: ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), in FP64 on
    the host with scipy (A symmetric, given by its lower triangle in CSC)."""
    import scipy.sparse as sp
    lower = sp.csc_matrix((np.asarray(values, np.float64), np.asarray(rowidx), np.asarray(colptr)), shape=(n, n))
    A = (lower + sp.tril(lower, -1).T).tocsr()
    X = np.asarray(X, np.float64).reshape(n, -1)
    B = np.asarray(B, np.float64).reshape(n, -1)
    R = B - A @ X
    norm_a = float(np.abs(A).sum(axis=1).max()) if n else 0.0
    worst = 0.0
    for k in range(X.shape[1]):
        den = norm_a * float(np.abs(X[:, k]).max()) + float(np.abs(B[:, k]).max())
        if den > 0:
            worst = max(worst, float(np.abs(R[:, k]).max()) / den)
    return worst


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    modes = {"grid3d60": bench_grid3d, "grid2d64": bench_grid2d, "elast48": bench_elast,
             "batch512": bench_batch, "serving": bench_serving, "copy": bench_copy, "cpu_tasks": bench_cpu_tasks}
    modes[args.workload](args)


def task_leg(s, strategies, threads=None, reps=1):
    """The paper's task-parallel left-looking factorization (Sec. 3-4) on
    the host cores, on the same matrix and analysis: per strategy the best
    of `reps` wall times and GFLOP/s (sum of squared column counts), with
    the update-count statistics of Algorithm 1."""
    from paper_2202_09288_amd import spchol, taskchol
    threads = threads or max(1, min(16, len(os.sched_getaffinity(0))))
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    plan = taskchol.TaskPlan.from_symbolic(sym, s.colptr, s.rowidx)
    st = plan.stats()
    C = plan.update_counts()
    hist = np.bincount(C)
    runs = {}
    for name in strategies:
        best = None
        for _ in range(reps):
            _, info = plan.factor(s.values, name, threads=threads)
            if best is None or info["seconds"] < best["seconds"]:
                best = info
        best["gflops"] = round(st["flops"] / best["seconds"] / 1e9, 3)
        best["seconds"] = round(best["seconds"], 4)
        runs[name] = best
        progress(f"task-parallel host factorization, {name}: {best}")
    if "nonested" in runs:
        for v in runs.values():
            v["speedup_vs_nonested"] = round(runs["nonested"]["seconds"] / v["seconds"], 3)
    plan.close()
    return {"threads": threads, "runs": runs,
            "update_counts": {"nsuper": st["nsuper"], "updates": st["updates"], "max": st["max_updates"],
                              "opt_d": st["opt_d"], "split_under_opt_d": st["split_opt_d"],
                              "tasks": {"nonested": st["tasks_nonested"], "nested": st["tasks_nested"],
                                        "opt_d": st["tasks_opt_d"], "opt_d_cost": st["tasks_opt_d_cost"]},
                              "histogram_head": [int(x) for x in hist[:16]],
                              "avg_supernode_cols": round(st["avg_supernode_cols"], 3),
                              "density": st["density"], "hybrid_choice": st["hybrid_choice"]}}


def bench_cpu_tasks(args):
    """The paper's method on the host: every strategy on configurations 1 and
    2, the hybrid choice and mt-BLAS on configuration 3; no GPU."""
    from paper_2202_09288_amd import workloads as W
    all_s = ["nonested", "nested", "opt_d", "opt_d_cost", "mt_blas", "hybrid"]
    out = {"workload": "cpu_tasks", "configs": {}}
    for name, s, strats, reps in (("64^2 2D 5-point", W.grid2d_unit(), all_s, 5),
                                  ("60^3 3D 7-point", W.grid3d_cond(), all_s, 1),
                                  ("48^3 elasticity", W.elast48(), ["mt_blas", "hybrid"], 1)):
        out["configs"][name] = task_leg(s, strats, reps=reps)
    print(json.dumps(out), flush=True)


def bench_copy(args):
    """Calibration for the HBM byte counters: a plain device-to-device copy
    of a known size (1 GiB read, 1 GiB written per launch), three launches."""
    import torch
    torch.cuda.set_device(0)
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src), 3, 1, torch)
    gbs = 2 * (1 << 30) / (float(np.median(t)) * 1e-3) / 1e9
    print(json.dumps({"workload": "copy", "bytes_read_per_launch": 1 << 30, "bytes_written_per_launch": 1 << 30,
                      "ms_per_launch": round(float(np.median(t)), 4), "GB/s": round(gbs, 1)}), flush=True)


def counted_traffic(kernel: str, precision: str, workload: str = "grid3d60"):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None when
    there is none for it or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"counters_{workload}_{precision}.md")
    try:
        txt = open(path).read()
        src = open(os.path.join(ROOT, "paper_2202_09288_amd", "csrc", "kernels.hip"), "rb").read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and line[:1].islower())
    if fields.get("traffic_kernel") != kernel or fields.get("kernels_source_sha1") != hashlib.sha1(src).hexdigest():
        return None
    return {"bytes": int(fields["traffic_bytes_per_launch"]), "read": int(fields["traffic_read_bytes_per_launch"]),
            "written": int(fields["traffic_written_bytes_per_launch"])}


def head(args, value, unit, dtype, config, ms_per_step, higher=True):
    config.setdefault("seed", args.seed)
    return {"metric": "factor GFLOP/s + solve p50/p99 ms at 1e-12 backward error vs plain FP64",
            "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def solve_times(F, B0, Bw, count, stream, torch):
    """Device ms of `count` solves of the resident factor (events around
    each solve on the library's stream; the right-hand sides are restored
    outside the timed interval)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    for e0, e1 in evs:
        Bw.copy_(B0)
        e0.record(stream)
        F.solve(Bw)
        e1.record(stream)
    torch.cuda.synchronize()
    return np.array([e0.elapsed_time(e1) for e0, e1 in evs])


def timed(fn, steps, warmup, torch):
    """Device time per call of fn() (events on the current stream), ms."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        out.append((e0, e1))
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in out])


def profiled_pass(F, step, nprof):
    """Per kernel class and per etree level: launches, device ms and flops of
    nprof profiled steps (events around every launch on its stream)."""
    F.set_profiling(True)
    prof, lv = {}, None
    for _ in range(nprof):
        step()
        for name, v in F.kernel_stats().items():
            p = prof.setdefault(name, {"launches": 0, "ms": 0.0, "flops": 0.0})
            for key in p:
                p[key] += v[key]
        ls = F.level_stats()
        lv = ls if lv is None else [dict(a, ms=a["ms"] + b["ms"]) for a, b in zip(lv, ls)]
    F.set_profiling(False)
    return prof, lv


def roofline_of(prof, nprof, precision, workload, kernel_names):
    """The dominant kernel class (most device time, assembly aside): its
    algorithmic flops over its summed launch durations, against the dense
    MFMA peak of the precision."""
    dom = max((n for n in prof if n != "assemble"), key=lambda n: prof[n]["ms"])
    peak = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    d = prof[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12 if d["ms"] > 0 else 0.0
    tname = "double" if precision == "fp64" else "float"
    kname = kernel_names[dom].format(t=tname)
    tr = counted_traffic(kname, precision, workload)
    return {"bound": "mfma", "kernel": kname,
            "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": tr["bytes"] if tr else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_read_written": [tr["read"], tr["written"]] if tr else None,
            "launches_per_step": d["launches"] // nprof,
            "avg_launch_ms": round(d["ms"] / max(1, d["launches"]), 4),
            "flops_per_launch": round(d["flops"] / max(1, d["launches"])),
            "classes_ms_per_step": {n: round(v["ms"] / nprof, 3) for n, v in prof.items()}}


def level_rows(lv, nprof):
    """Per etree level (-2: the small-subtree launch, -1: assembly): launches, device ms and TFLOP/s of one
    factorization."""
    return [[v["level"], v["launches"] // nprof, round(v["ms"] / nprof, 3),
             round(v["flops"] / (v["ms"] / nprof * 1e-3) / 1e12, 2) if v["ms"] > 0 else 0.0] for v in lv]


def cutoffs(args, systems, nrhs, precision):
    """The autotuned schedule cut-offs for this workload and precision (from
    the tuner's cache), or {} for the library defaults."""
    if args.tuning != "auto":
        return {}
    from paper_2202_09288_amd import tune
    return tune.load(tune.cache_key(systems, precision, nrhs)) or {}


def bench_grid2d(args):
    """64x64 5-point Laplacian (n = 4,096), FP64: a latency-bound system."""
    import torch
    from paper_2202_09288_amd import spchol
    from paper_2202_09288_amd import workloads as W
    torch.cuda.set_device(0)
    s = W.grid2d_unit(seed=args.seed)
    tuning = cutoffs(args, [s], 1, "fp64")
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning)
    dv = torch.from_numpy(s.values).cuda()
    B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    Bw = torch.empty_like(B0)
    F = spchol.factorize(sym, dv)
    F.sync()
    F.set_graph(args.graph == "on")
    steps, warm = max(args.steps, 50), max(args.warmup, 5)
    fac = timed(lambda: F.refactorize(dv), steps, warm, torch)
    sol = timed(lambda: (Bw.copy_(B0), F.solve(Bw)), steps, warm, torch)
    F.sync()
    berr = host_backward_error(s.n, s.colptr, s.rowidx, s.values, Bw.cpu().numpy().T, s.B)
    flops = float(sym.info["flops"])
    out = head(args, round(flops / (fac.mean() * 1e-3) / 1e9, 3), "GFLOP/s", "f64",
               {"workload": "2D 5-point, 64x64 grid, diagonal = degree + 1e-2, geometric nested dissection, "
                            "1 RHS, plain FP64 factor + solve", "n": s.n, "flops": int(flops),
                "levels": sym.info["levels"], "nsuper": sym.info["nsuper"],
                "schedule_cutoffs": tuning or "library defaults"},
               round(float(fac.mean() + sol.mean()), 4))
    out.update({"factor_us_p50": round(float(np.median(fac)) * 1e3, 1),
                "solve_us_p50": round(float(np.median(sol)) * 1e3, 1),
                "solve_us_p99": round(float(np.percentile(sol, 99)) * 1e3, 1),
                "berr": berr, "berr_ok": bool(berr <= 1e-12)})
    print(json.dumps(out), flush=True)


def bench_elast(args):
    """The headline: 48^3 27-point 3-dof elasticity operator (kappa ~ 1e8),
    4 RHS.  Timed steps: plain FP64 refactorization + solve.  Beside it, the
    FP32 factorization with FP64 refinement to a backward error <= 1e-12."""
    import torch
    from paper_2202_09288_amd import spchol
    from paper_2202_09288_amd import workloads as W
    torch.cuda.set_device(0)
    s = W.elast48(seed=args.seed)
    nrhs = s.B.shape[1]
    progress(f"48^3 elasticity generated, n = {s.n}")
    t0 = time.perf_counter()
    tun64 = cutoffs(args, [s], nrhs, "fp64")
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tun64)
    t_analyze = time.perf_counter() - t0
    info = sym.info
    flops = float(info["flops"])
    dv = torch.from_numpy(s.values).cuda()
    B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    Bw = torch.empty_like(B0)
    stream = torch.cuda.current_stream()

    # ---- plain FP64: the timed steps
    progress(f"analysis done ({t_analyze:.1f} s)")
    F = spchol.factorize(sym, dv, "fp64")
    F.sync()
    F.set_graph(args.graph == "on")
    progress("first FP64 factorization done")

    def step(ev=None):
        Bw.copy_(B0)
        if ev:
            ev[0].record(stream)
        F.refactorize(dv)
        if ev:
            ev[1].record(stream)
        F.solve(Bw)
        if ev:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    F.sync()
    progress(f"{args.warmup} warmup steps done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    F.sync()  # raises if a pivot failed
    fac_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    sol_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    berr64 = host_backward_error(s.n, s.colptr, s.rowidx, s.values, Bw.cpu().numpy().T, s.B)
    # solve latency over more samples than the steps: the p50/p99 reported
    sol_ms = solve_times(F, B0, Bw, args.solves, stream, torch)
    nprof = max(1, min(args.steps, 2))
    progress(f"plain FP64: {args.steps} steps, factor {fac_ms.mean():.2f} ms, {args.solves} solves")
    prof, lv = profiled_pass(F, step, nprof)
    roofline = roofline_of(prof, nprof, "fp64", "elast48", spchol.KERNEL_NAMES)
    F.close()
    fac_mean = float(fac_ms.mean())
    value = flops / (fac_mean * 1e-3) / 1e9

    # ---- FP32 (and BF16-update) factorization + FP64 refinement (the same
    # matrix and right-hand sides)
    tun32 = cutoffs(args, [s], nrhs, "fp32")
    sym32 = sym if tun32 == tun64 else spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tun32)

    def refined_leg(prec):
        F32 = spchol.factorize(sym32, dv, prec)
        F32.sync()
        F32.set_graph(args.graph == "on")
        fac32 = timed(lambda: F32.refactorize(dv), args.steps, args.warmup, torch)
        X = torch.zeros_like(B0)
        rinfo = {}

        def refined():
            rinfo.update(F32.solve_refined(dv, B0, X, tol=1e-12, maxit=200))
        ref = timed(refined, max(3, args.steps // 2), 1, torch)
        F32.sync()
        berr = host_backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
        raised = F32.pivot_floors()
        F32.close()
        f_ms = float(fac32.mean())
        return {"factor_ms": round(f_ms, 3),
                "factor_gflops": round(flops / (f_ms * 1e-3) / 1e9, 1),
                "factor_frac_of_fp32_peak": round(flops / (f_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                "refined_solve_ms_p50": round(float(np.median(ref)), 3),
                "refined_solve_ms_p99": round(float(np.percentile(ref, 99)), 3),
                "refinement_steps": rinfo.get("iterations"), "converged": rinfo.get("converged"),
                "status": spchol._lib.spc_status_string(rinfo.get("status", 0)).decode(),
                "berr": berr, "berr_ok": bool(berr <= 1e-12), "pivots_raised_to_floor": raised,
                "factor_plus_refined_solve_ms": round(f_ms + float(np.median(ref)), 3),
                "schedule_cutoffs": tun32 or "library defaults"}

    if args.only_fp64:
        leg32 = leg16 = None
    else:
        leg32 = refined_leg("fp32")
        progress(f"FP32 + refinement: {leg32['factor_ms']} ms + {leg32['refined_solve_ms_p50']} ms")
        try:
            leg16 = refined_leg("bf16upd")
        except spchol.NotSPD as e:
            leg16 = {"status": "not SPD", "detail": str(e)}
        progress(f"BF16 updates + refinement: {leg16}")
    plain = {"factor_ms": round(fac_mean, 3), "solve_ms_p50": round(float(np.median(sol_ms)), 3),
             "factor_plus_solve_ms": round(fac_mean + float(np.median(sol_ms)), 3)}
    out = head(args, round(value, 2), "GFLOP/s", "f64",
               {"workload": "3D 27-point 3-dof elasticity-like operator, 48^3 grid, kappa ~1e8, 4 RHS, "
                            "geometric nested dissection; plain FP64 supernodal factor + solve",
                "n": s.n, "nnz_lower": s.nnz, "flops": int(flops), "nnz_L": info["nnz_l"],
                "nsuper": info["nsuper"], "levels": info["levels"], "amalg_z": 0.05,
                "schedule_cutoffs": tun64 or "library defaults", "precision": "fp64", "nrhs": nrhs},
               round(wall * 1e3 / args.steps, 3))
    out.update({
        "factor_ms_mean": round(fac_mean, 3),
        "factor_ms_p50": round(float(np.median(fac_ms)), 3),
        "solve_ms_p50": round(float(np.percentile(sol_ms, 50)), 3),
        "solve_ms_p99": round(float(np.percentile(sol_ms, 99)), 3),
        "solves_timed": int(sol_ms.size),
        "berr": berr64, "berr_ok": bool(berr64 <= 1e-12),
        "frac_of_peak": round(value / (FP64_PEAK_TFLOPS * 1e3), 4),
        "analyze_s": round(t_analyze, 2),
        "roofline": roofline,
        "factor_levels": {"columns": ["etree level (-2: the persistent launch over the small subtrees, -1: assembly)",
                                      "launches", "device ms", "TFLOP/s"],
                          "rows": level_rows(lv, nprof)},
        "vs_plain_fp64": {"plain_fp64": plain, "fp32_refined": leg32, "bf16upd_refined": leg16,
                          "speedup_factor_plus_solve": round(plain["factor_plus_solve_ms"] /
                                                             leg32["factor_plus_refined_solve_ms"], 3)
                          if leg32 else None},
    })
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds, "48^3 elasticity")
        progress("CPU oracle sample done")
    if not args.no_task_baseline:
        # the paper's own method on all host cores, whole matrix: its hybrid
        # rule's choice and mt-BLAS
        out["cpu_task_baseline"] = task_leg(s, ["hybrid", "mt_blas"])
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """512 independent systems (2D/3D grids, n from ~1k to ~40k), 16 RHS each,
    merged into one forest: one schedule factors them all (FP32), one batched
    solve; FP64 refinement of all systems together, checked per system."""
    import torch
    from paper_2202_09288_amd import spchol
    from paper_2202_09288_amd import workloads as W
    torch.cuda.set_device(0)
    systems = W.batch512()
    tuning = cutoffs(args, systems, 16, "fp32")
    syms = [spchol.Symbolic(x.colptr, x.rowidx, x.perm, 0.05, tuning) for x in systems]
    flops = float(sum(x.info["flops"] for x in syms))
    dvs = [torch.from_numpy(x.values).cuda() for x in systems]
    Bs0 = [torch.from_numpy(np.ascontiguousarray(x.B.T)).cuda() for x in systems]
    res = {}
    for prec in ("fp32", "fp64"):
        batch = spchol.Batch(syms, prec)
        batch.set_graph(args.graph == "on")
        batch.factorize(dvs)
        batch.sync()
        fac = timed(lambda: batch.factorize(dvs), args.steps, args.warmup, torch)
        Bw = [torch.empty_like(b) for b in Bs0]

        def solve():
            for b, b0 in zip(Bw, Bs0):
                b.copy_(b0)
            batch.solve(Bw)
        sol = timed(solve, max(3, args.steps // 2), 1, torch)
        batch.sync()
        res[prec] = {"factor_ms": round(float(fac.mean()), 3),
                     "factor_gflops": round(flops / (fac.mean() * 1e-3) / 1e9, 1),
                     "batched_solve_ms_p50": round(float(np.median(sol)), 3)}
        # one profiled factorization: device time per kernel class and per
        # etree level of the merged forest (events around every launch)
        batch.set_profiling(True)
        batch.factorize(dvs)
        batch.sync()
        res[prec]["classes_ms"] = {k: round(v["ms"], 3) for k, v in batch.kernel_stats().items()}
        res[prec]["factor_levels"] = {
            "columns": ["etree level (-2: the small-subtree launch, -1: assembly)", "launches", "device ms", "TFLOP/s"],
            "rows": level_rows(batch.level_stats(), 1)}
        batch.set_profiling(False)
        if prec == "fp32":
            # FP64 refinement of all systems at once (one merged solve per
            # step, per-system norms and coefficients)
            Xs = [torch.zeros_like(b) for b in Bs0]
            out = batch.solve_refined(Bs0, Xs, tol=1e-12, maxit=100)
            ref = []
            for _ in range(3):
                t0 = time.perf_counter()
                out = batch.solve_refined(Bs0, Xs, tol=1e-12, maxit=100)
                ref.append(time.perf_counter() - t0)
            iters = [r["iterations"] for r in out["systems"]]
            worst = 0.0
            for i, x in enumerate(systems[:64]):
                worst = max(worst, host_backward_error(x.n, x.colptr, x.rowidx, x.values,
                                                         Xs[i].cpu().numpy().T, x.B))
            res[prec].update({"refine_all_ms": round(1e3 * float(np.median(ref)), 3),
                              "refine_converged_all": bool(out["status"] == spchol.OK),
                              "refine_iterations_max": int(max(iters)),
                              "berr_device_max": max(r["berr"] for r in out["systems"]),
                              "berr_max_first64": worst, "berr_ok": bool(worst <= 1e-12)})
        batch.close()
    r32 = res["fp32"]
    out = head(args, r32["factor_gflops"], "GFLOP/s", "f32",
               {"workload": "batch of 512 SPD systems: 2D 5-point / 3D 7-point grids, sides U[32,200] / "
                            "U[10,34], conductances 10^U[-2,2), shift 1e-2, 16 RHS each; one merged schedule",
                "systems": len(systems), "n_total": int(sum(x.n for x in systems)), "flops": int(flops),
                "schedule_cutoffs": tuning or "library defaults"},
               round(r32["factor_ms"] + r32["batched_solve_ms_p50"], 3))
    out.update({"fp32": res["fp32"], "fp64": res["fp64"]})
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Request loop: Poisson arrivals of factor-then-solve requests from the
    batch size mix (plus 5% 3D 50^3), 30% re-solves with 8 RHS on resident
    factors; p50/p99 latency and solves/s per arrival rate."""
    import torch
    from paper_2202_09288_amd import serving
    torch.cuda.set_device(0)

    def one(rate, count):
        reqs = serving.make_requests(count, rate, seed=args.seed)
        srv = serving.Server(slots=4, hbm_budget=int(args.serving_budget_gb * (1 << 30)), precision="fp32",
                             tol=1e-12, maxit=100, handover=args.serving_handover == "on")
        t0 = time.perf_counter()
        srv.run(reqs)
        wall = time.perf_counter() - t0
        srv.close()
        summ = serving.summarize(reqs, wall)
        summ["peak_device_bytes"] = srv.peak
        summ["rate_hz"] = rate
        print(f"serving rate {rate}: {summ}", file=sys.stderr, flush=True)
        return summ

    runs = []
    capacity = None
    if args.capacity_sweep:
        # capacity: every request at once (arrival rate far above service)
        cap = one(1e6, min(args.requests, 600))
        capacity = cap["requests_per_s"]
        rates = [round(f * capacity, 2) for f in (0.25, 0.5, 0.75, 0.9, 1.0, 1.1)]
    else:
        rates = [args.rate] if args.rate > 0 else [20.0, 50.0, 100.0]
    for rate in rates:
        summ = one(rate, args.requests)
        if capacity:
            summ["fraction_of_capacity"] = round(rate / capacity, 2)
        runs.append(summ)
    best = min(runs, key=lambda r: r["p99_ms"] or 1e30)
    out = head(args, round(best["solves_per_s"], 2), "solves/s", "f32",
               {"workload": "serving: Poisson arrivals, batch size mix + 5% 3D 50^3, 30% re-solves (8 RHS) "
                            "of factors resident when dispatched, FP32 + FP64 refinement to 1e-12, 4 slots, "
                            "analysis in a 2-thread pool, pooled slots refactorized by graph replay",
                "requests_per_rate": args.requests, "hbm_budget_gb": args.serving_budget_gb}, None)
    out.update({"runs": runs, "capacity_requests_per_s": capacity})
    print(json.dumps(out), flush=True)


def bench_grid3d(args):
    import torch
    from paper_2202_09288_amd import spchol
    from paper_2202_09288_amd import workloads as W

    torch.cuda.set_device(0)
    s = W.grid3d_cond(k=args.grid, seed=args.seed)
    tuning = cutoffs(args, [s], 1, args.precision)
    t0 = time.perf_counter()
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning)
    t_analyze = time.perf_counter() - t0
    info = sym.info
    flops = float(info["flops"])
    dv = torch.from_numpy(s.values).cuda()
    B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    Bw = torch.empty_like(B0)
    F = spchol.factorize(sym, dv, args.precision)
    F.sync()
    F.set_graph(args.graph == "on")
    stream = torch.cuda.current_stream()

    def step(ev):
        Bw.copy_(B0)
        ev[0].record(stream)
        F.refactorize(dv)
        ev[1].record(stream)
        F.solve(Bw)
        ev[2].record(stream)

    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True) for _ in range(3)])
    F.sync()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    F.sync()  # raises if a pivot failed
    fac_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    sol_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])

    X = Bw.cpu().numpy().T
    berr = host_backward_error(s.n, s.colptr, s.rowidx, s.values, X, s.B)
    sol_ms = solve_times(F, B0, Bw, args.solves, stream, torch)

    nprof = max(1, min(args.steps, 3))
    prof, lv_ms = profiled_pass(F, lambda: step([torch.cuda.Event(enable_timing=True) for _ in range(3)]), nprof)
    peak = FP64_PEAK_TFLOPS if args.precision == "fp64" else FP32_PEAK_TFLOPS
    roofline = roofline_of(prof, nprof, args.precision, f"grid3d{args.grid}", spchol.KERNEL_NAMES)
    levels = level_rows(lv_ms, nprof)

    fac_mean = float(fac_ms.mean())
    value = flops / (fac_mean * 1e-3) / 1e9
    out = {
        "metric": "factor GFLOP/s + solve p50/p99 ms at 1e-12 backward error vs plain FP64",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point, {args.grid}^3 grid, conductances 10^U[-2,2), shift 1e-6, "
                               "geometric nested dissection, 1 RHS, plain supernodal factor + solve",
                   "n": s.n, "nnz_lower": s.nnz, "flops": int(flops), "nnz_L": info["nnz_l"],
                   "nsuper": info["nsuper"], "levels": info["levels"], "amalg_z": 0.05, "seed": args.seed,
                   "schedule_cutoffs": tuning or "library defaults",
                   "precision": args.precision},
        "factor_ms_mean": round(fac_mean, 3),
        "factor_ms_p50": round(float(np.median(fac_ms)), 3),
        "solve_ms_p50": round(float(np.percentile(sol_ms, 50)), 3),
        "solve_ms_p99": round(float(np.percentile(sol_ms, 99)), 3),
        "solves_timed": int(sol_ms.size),
        "berr": berr,
        "berr_ok": bool(berr <= 1e-12),
        "frac_of_peak": round(value / (peak * 1e3), 4),
        "analyze_s": round(t_analyze, 2),
        "roofline": roofline,
        "factor_levels": {"columns": ["etree level (-2: the persistent launch over the small subtrees, -1: assembly)",
                                      "launches", "device ms", "TFLOP/s"],
                          "rows": levels},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds, f"{args.grid}^3")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
