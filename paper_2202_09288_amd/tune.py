"""Autotuner for the schedule cut-offs of the numeric phase.

The cut-offs decide, per supernode, between batching it with the other
small supernodes of its elimination-tree level (one wave or one workgroup
each) and giving it the blocked whole-device kernels; which scatter updates
take 128x128 tiles; and how many solve levels from the top run as one
persistent launch (the analysis options of spc_analyze).  The tuner times
the refactorization and the solve of a workload on the device for candidate
settings, one group of cut-offs at a time (coordinate descent from the
library defaults), keeps the setting with the smallest factor + solve time,
and stores it in a JSON cache keyed by the workload's size and precision.

    python -m paper_2202_09288_amd.tune --workload grid3d60 --precision fp64

Every trial is checked with the library's own FP64 backward error of the
solve: a setting that misses the bar of its precision is not taken.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import spchol
from . import workloads as W

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

# candidate values per group of cut-offs (the first entry of each group is
# the library default); negative turns a path off
GROUPS = [
    ("tiny", ("tiny_w", "tiny_m"), [(8, 64), (4, 32), (-1, -1)]),
    ("small", ("small_w", "small_m"), [(32, 128), (16, 64), (32, 64), (-1, -1)]),
    ("big", ("big_min", "big_min_k"), [(256, 128), (128, 64), (512, 128), (256, 256), (-1, -1)]),
    ("persist", ("solve_persist_max",), [(1024,), (256,), (4096,)]),
    ("delay", ("delay",), [(1,), (2,), (3,), (4,)]),
    ("handover", ("handover",), [(1,), (-1,), (2,)]),
    ("lookahead", ("lookahead",), [(-1,), (1,)]),
    ("persist", ("persist",), [(-1,), (1,)]),
    ("group", ("group",), [(1,), (-1,)]),
    ("bulk128", ("bulk128",), [(-1,), (1,)]),
]


def workload(name: str):
    """(systems, nrhs) of a named workload (seeded, synthetic)."""
    if name == "grid3d60":
        return [W.grid3d_cond()], 1
    if name == "grid2d64":
        return [W.grid2d_unit()], 1
    if name == "elast48":
        return [W.elast48()], 4
    if name == "batch512":
        return W.batch512(), 16
    raise ValueError(f"unknown workload {name}")


def cache_key(systems, precision: str, nrhs: int) -> str:
    n = sum(int(s.n) for s in systems)
    nnz = sum(int(s.colptr[-1]) for s in systems)
    return f"{precision}:systems={len(systems)}:n={n}:nnz={nnz}:nrhs={nrhs}"


def load(key: str, path: str = CACHE):
    """The cached cut-offs for key, or None."""
    try:
        with open(path) as f:
            entry = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    return None if entry is None else dict(entry["tuning"])


def save(key: str, result: dict, path: str = CACHE) -> None:
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[key] = result
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _berr_bar(precision: str) -> float:
    return {"fp64": 1e-12, "fp32": 1e-5}.get(precision, 1e-2)  # BF16 updates: a rough preconditioner


def measure(systems, nrhs: int, tuning: dict, precision: str, reps: int, torch):
    """Mean device ms of a refactorization and of a solve (a batch: host
    wall time of the batched solve), and the worst FP64 backward error of
    the solve, for one setting."""
    syms = [spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning) for s in systems]
    dvs = [torch.from_numpy(s.values).cuda() for s in systems]
    B0 = [torch.from_numpy(np.ascontiguousarray(s.B[:, :nrhs].T)).cuda() for s in systems]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if len(systems) == 1:
        F = spchol.factorize(syms[0], dvs[0], precision)
        F.sync()
        fac, sol = [], []
        for _ in range(reps + 1):
            F.refactorize(dvs[0])
            F.sync()
            fac.append(F.last_ms())
            X = B0[0].clone()
            ev0.record()
            F.solve(X)
            ev1.record()
            torch.cuda.synchronize()
            sol.append(ev0.elapsed_time(ev1))
        Xs = [X]
    else:
        batch = spchol.Batch(syms, precision)
        batch.factorize(dvs)
        batch.sync()
        fac, sol = [], []
        for _ in range(reps + 1):
            batch.factorize(dvs)
            batch.sync()
            fac.append(batch.last_ms())
            Xs = [b.clone() for b in B0]
            t0 = time.perf_counter()
            batch.solve(Xs)
            sol.append(1e3 * (time.perf_counter() - t0))
    # the library's own FP64 backward error of the plain solve (refinement
    # with no steps)
    if len(systems) == 1:
        X = torch.zeros_like(B0[0])
        worst = F.solve_refined(dvs[0], B0[0], X, tol=0.0, maxit=0)["berr"]
    else:
        out = batch.solve_refined(B0, [torch.zeros_like(b) for b in B0], tol=0.0, maxit=0)
        worst = max(r["berr"] for r in out["systems"])
        batch.close()
    return float(np.mean(fac[1:])), float(np.mean(sol[1:])), worst


def tune(systems, nrhs: int, precision: str = "fp64", reps: int = 5, log=print, passes: int = 2) -> dict:
    """Coordinate descent over GROUPS from the defaults (a second pass goes
    over the groups again from the best setting, since some cut-offs pay
    only together, e.g. the bulk-update depth and the hand-over rule);
    returns the best setting with its times and every trial."""
    import torch
    torch.cuda.set_device(0)
    best = {}
    trials = []

    def run(setting):
        f, s, e = measure(systems, nrhs, setting, precision, reps, torch)
        ok = e <= _berr_bar(precision)
        trials.append({"tuning": dict(setting), "factor_ms": f, "solve_ms": s, "berr": e, "ok": ok})
        log(f"  {setting}: factor {f:.3f} ms, solve {s:.3f} ms, berr {e:.1e}{'' if ok else ' (rejected)'}")
        return (f + s) if ok else float("inf"), f, s

    cost, fbest, sbest = run(best)
    tried = {json.dumps(best, sort_keys=True)}
    for p in range(passes):
        changed = False
        for name, fields, cands in GROUPS:
            log(f"pass {p + 1}, group {name}")
            for vals in cands:
                trial = dict(best)
                trial.update(dict(zip(fields, vals)))
                key = json.dumps(trial, sort_keys=True)
                if key in tried:
                    continue
                tried.add(key)
                c, f, s = run(trial)
                if c < cost:
                    cost, fbest, sbest, best, changed = c, f, s, trial, True
        if not changed:
            break
    return {"tuning": best, "factor_ms": fbest, "solve_ms": sbest, "precision": precision, "nrhs": nrhs,
            "trials": trials}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="grid3d60", choices=["grid3d60", "grid2d64", "elast48", "batch512"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16upd"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--passes", type=int, default=2, help="passes of coordinate descent over the groups")
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args(argv)
    systems, nrhs = workload(a.workload)
    key = cache_key(systems, a.precision, nrhs)
    print(f"tuning {a.workload} ({key})", flush=True)
    res = tune(systems, nrhs, a.precision, a.reps, log=lambda m: print(m, flush=True), passes=a.passes)
    res["workload"] = a.workload
    save(key, res, a.out)
    print(json.dumps({k: v for k, v in res.items() if k != "trials"}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
