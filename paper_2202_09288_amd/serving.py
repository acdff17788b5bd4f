"""Continuous-batching serving loop over the C ABI.

Requests are factor-then-solve (a new SPD system and right-hand sides) or
re-solve (new right-hand sides for a factor kept resident from an earlier
request).  The loop admits requests as slots and device memory free up:

  - a slot is a worker thread with its own HIP stream (default priority), so
    the work of requests in different slots overlaps on the device; the
    library calls release the GIL;
  - the analysis of a pattern (spc_analyze, on the host) runs in a pool of
    analysis threads, off the dispatcher: a factor request whose pattern is
    being analysed waits while the dispatcher admits the requests behind it;
    the result is cached by pattern, so a known pattern is never analysed
    again (the paper's analyze-once, factorize-many, Sec. 1-2);
  - device memory is held in factor slots: a factor, its values buffer and
    the footprint the analysis reports (panels, plan, solve and refinement
    work areas).  A factor request gets a new slot, admitted by footprint,
    while the HBM budget allows; at the budget it takes over the slot of the
    least recently used idle resident factor of its own pattern
    (spc_refactorize into it, replayed from the slot's captured HIP graph:
    the values buffer keeps its address, so a slot's graph is captured once),
    else idle resident factors of other patterns are evicted, least recently
    used first, until it fits.  Residency is bounded by the budget alone;
  - after its request, a factor stays resident: a re-solve picks uniformly
    among the factors resident when it is dispatched (its `pick` in [0, 1)
    indexes them), so it never misses while one is resident.  With
    resolve_policy="fixed" a re-solve instead names its factor request
    (`target`), and one whose factor was evicted is a miss: that system is
    factored again, then solved;
  - every solve is a factor in `precision` plus FP64 refinement to the
    backward-error tolerance, and each request records its latency
    (completion - arrival), whether its pattern was new on arrival (cold)
    and whether it reused a pooled slot.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import hashlib
import queue
import threading
import time
from collections import OrderedDict

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the run
    kind: str                      # "factor" or "resolve"
    system: object = None          # workloads.System for "factor"
    values_scale: float = 1.0      # factor requests scale the system's values
    target: int = -1               # resolve: the factor request it solves with
    pick: float = 0.0              # resolve: which resident factor, in [0, 1)
    nrhs: int = 8
    key: str = ""                  # factor: pattern key
    # filled in by the server
    start: float = -1.0
    done: float = -1.0
    berr: float = float("nan")
    iterations: int = -1
    miss: bool = False             # fixed-target resolve whose factor had been evicted
    cold: bool = False             # factor: pattern first seen at this request's arrival
    pooled: bool = False           # factor: refactorized into an idle slot of its pattern
    status: str = "pending"
    X: object = None               # host solution when keep_solutions
    L: object = None               # host panels (FP64) when export_factors


def pattern_key(s) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(s.colptr).tobytes())
    h.update(np.ascontiguousarray(s.rowidx).tobytes())
    h.update(np.ascontiguousarray(s.perm).tobytes())
    return h.hexdigest()


class Slot:
    """Device memory of one factor: the factor, its values buffer, and the
    bytes admitted for it.  owner: the request whose factor it holds while
    resident, else -1 (idle in its pattern's pool)."""

    def __init__(self, key, sym, nbytes):
        self.key = key
        self.sym = sym
        self.nbytes = nbytes
        self.factor = None
        self.d_values = None
        self.owner = -1
        self.system = None
        self.scale = 1.0
        self.in_use = 0
        self.lock = threading.Lock()

    def close(self):
        if self.factor is not None:
            self.factor.close()
            self.factor = None
        self.d_values = None


class Server:
    """Serve a list of requests with arrival times; see module docstring."""

    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, precision: str = "fp32",
                 tol: float = 1e-12, maxit: int = 50, keep_solutions: bool = False, handover: bool = False,
                 analysis_workers: int = 2, resolve_policy: str = "resident", graph: bool = True,
                 export_factors: bool = False):
        import torch
        from . import spchol
        if resolve_policy not in ("resident", "fixed"):
            raise ValueError("resolve_policy is 'resident' or 'fixed'")
        self.torch = torch
        self.lib = spchol
        self.slots = slots
        self.budget = int(hbm_budget)
        self.precision = precision
        self.tol = tol
        self.maxit = maxit
        self.keep_solutions = keep_solutions
        self.export_factors = export_factors
        self.policy = resolve_policy
        self.graph = graph
        # in-launch TRSM hand-over (waits inside a launch) for the
        # factorizations: safe beside the other slots' work (a wait is only
        # on a running workgroup), but off by default, since its waiting
        # tiles hold CUs that the other slots could use (2,000 requests at
        # 466/s: p50 5.4 / p99 310 ms with it, 5.0 / 209 ms without)
        self.tuning = {"handover": 1 if handover else -1}
        self.sym_cache = {}
        self.analyzing = {}                # key -> future
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=max(1, analysis_workers))
        self.lock = threading.RLock()      # resident, free, used, in_use
        self.resident = OrderedDict()      # owner rid -> Slot (LRU order)
        self.used = 0                      # bytes held by slots
        self.peak = 0
        self.wake = threading.Condition()  # a request finished or an analysis ended
        self.inflight_factors = 0
        self.refactoring = set()           # fixed policy: targets being factored again
        self._factors_pending = False
        self._by_rid = {}

    # ---- memory accounting ------------------------------------------------
    def footprint(self, sym, nrhs: int) -> int:
        i = sym.info
        fac = i["factor_bytes_fp32"] if self.precision != "fp64" else i["factor_bytes_fp64"]
        n = i["n"]
        esz = 8 if self.precision == "fp64" else 4
        work = n * 16 * 3 * esz + n * 16 * 8 * 7  # solve + refinement work areas
        csr = 2 * i["nnz_a"] * 12 + 8 * n
        vals = i["nnz_a"] * 8 + 2 * n * nrhs * 8
        return int(fac + work + csr + vals)

    def _free_slot(self, slot):
        slot.close()
        self.used -= slot.nbytes

    def acquire_slot(self, key, sym, nbytes):
        """Device memory for a factor of pattern `key`: a new slot while the
        budget allows; else the least recently used idle resident factor of
        the same pattern, whose slot is taken over as it is (pooled: no
        allocation, its graph replays); else new room made by evicting idle
        resident factors of other patterns, least recently used first.
        Returns (slot, pooled), or (None, False) if there is no room now."""
        with self.lock:
            if nbytes > self.budget:
                return None, False
            if self.used + nbytes > self.budget:
                rid = next((r for r, sl in self.resident.items() if sl.in_use == 0 and sl.key == key), None)
                if rid is not None:
                    sl = self.resident.pop(rid)
                    sl.owner = -1
                    return sl, True
            while self.used + nbytes > self.budget:
                rid = next((r for r, sl in self.resident.items() if sl.in_use == 0), None)
                if rid is None:
                    return None, False
                self._free_slot(self.resident.pop(rid))
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            return Slot(key, sym, nbytes), False

    def symbolic(self, s):
        """The analysis of s's pattern (synchronously; the loop itself uses
        the analysis pool)."""
        key = pattern_key(s)
        with self.lock:
            sym = self.sym_cache.get(key)
        if sym is None:
            sym = self._analyze(key, s)
        return sym

    def _analyze(self, key, s):
        sym = self.lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, self.tuning)
        with self.lock:
            self.sym_cache.setdefault(key, sym)
            sym = self.sym_cache[key]
        return sym

    def _analysis_done(self, key):
        with self.lock:
            self.analyzing.pop(key, None)
        with self.wake:
            self.wake.notify_all()

    # ---- work of one request (runs in a slot thread) ------------------------
    def _factor_into(self, slot, system, scale, stream):
        """Factor system (values * scale) into the slot on `stream`."""
        torch = self.torch
        vals = torch.from_numpy(system.values * scale)
        if slot.d_values is None:
            slot.d_values = torch.empty(vals.numel(), dtype=torch.float64, device="cuda")
        slot.d_values.copy_(vals)
        if slot.factor is None:
            slot.factor = self.lib.factorize(slot.sym, slot.d_values, self.precision, stream=stream)
            slot.factor.set_graph(self.graph)
        else:
            slot.factor.refactorize(slot.d_values, stream=stream)
        slot.factor.sync()
        slot.system = system
        slot.scale = scale

    def _solve(self, req, slot, stream, B):
        torch = self.torch
        X = torch.zeros_like(B)
        info = slot.factor.solve_refined(slot.d_values, B, X, tol=self.tol, maxit=self.maxit, stream=stream)
        stream.synchronize()
        req.berr = info["berr"]
        req.iterations = info["iterations"]
        req.status = "ok" if info["converged"] else "no-convergence"
        if self.keep_solutions:
            req.X = X.cpu().numpy().T.copy()

    def _run_factor(self, req, slot, stream):
        torch = self.torch
        with slot.lock, torch.cuda.stream(stream):
            self._factor_into(slot, req.system, req.values_scale, stream)
            if self.export_factors:
                req.L = slot.factor.export()
            B = torch.from_numpy(self.rhs(req)).cuda()
            self._solve(req, slot, stream, B)
        with self.lock:
            slot.owner = req.rid
            slot.in_use -= 1
            self.resident[req.rid] = slot
            self.inflight_factors -= 1

    def _run_resolve(self, req, slot, stream):
        torch = self.torch
        with slot.lock, torch.cuda.stream(stream):
            if slot.owner != req.target:  # a miss: factor the target's system again
                tgt = self._by_rid[req.target]
                self._factor_into(slot, tgt.system, tgt.values_scale, stream)
            B = torch.from_numpy(self.rhs(req, slot.system)).cuda()
            self._solve(req, slot, stream, B)
        with self.lock:
            if slot.owner != req.target:
                slot.owner = req.target
                self.resident[req.target] = slot
                self.refactoring.discard(req.target)
            slot.in_use -= 1

    @staticmethod
    def rhs(req: Request, system=None):
        """(nrhs, n) right-hand sides: the system's own for a factor request,
        seeded by the request id for a re-solve."""
        if req.kind == "factor":
            return np.ascontiguousarray(req.system.B[:, :req.nrhs].T)
        from .workloads import uniform, stream_key, W_SERVE, P_RHS
        u = uniform(stream_key(W_SERVE, 0, P_RHS, req.rid), req.nrhs * system.n)
        return np.ascontiguousarray((2.0 * u - 1.0).reshape(req.nrhs, system.n))

    # ---- dispatch ------------------------------------------------------------
    def _dispatch_factor(self, req):
        with self.lock:
            sym = self.sym_cache.get(req.key)
            busy = req.key in self.analyzing
        if sym is None:
            if not busy:
                fut = self.pool.submit(self._analyze, req.key, req.system)
                with self.lock:
                    self.analyzing[req.key] = fut
                fut.add_done_callback(lambda _f, k=req.key: self._analysis_done(k))
            return None
        slot, pooled = self.acquire_slot(req.key, sym, self.footprint(sym, req.nrhs))
        if slot is None:
            return None
        req.pooled = pooled
        with self.lock:
            slot.in_use += 1
            self.inflight_factors += 1
        return (req, "factor", slot)

    def _dispatch_resolve(self, req):
        with self.lock:
            if self.policy == "resident":
                if not self.resident:
                    if self.inflight_factors > 0 or self._factors_pending:
                        return None  # one will be resident soon
                    req.status = "no-resident-factor"
                    return "done"
                owners = sorted(self.resident)
                rid = owners[min(int(req.pick * len(owners)), len(owners) - 1)]
                slot = self.resident[rid]
                req.target = rid
                slot.in_use += 1
                self.resident.move_to_end(rid)
                return (req, "resolve", slot)
            slot = self.resident.get(req.target)
            if slot is not None:
                slot.in_use += 1
                self.resident.move_to_end(req.target)
                return (req, "resolve", slot)
            tgt = self._by_rid.get(req.target)
            if tgt is None or tgt.status not in ("ok", "pending"):
                req.status = "no-resident-factor"
                return "done"
            if tgt.done < 0 or req.target in self.refactoring:
                return None  # its factor request (or another miss on it) is queued or running
        # evicted: a miss, factored again into a slot of its pattern
        got = self._dispatch_factor(Request(rid=-1, arrival=req.arrival, kind="factor", system=tgt.system,
                                            values_scale=tgt.values_scale, key=tgt.key))
        if got is None:
            return None
        _, _, slot = got
        with self.lock:
            self.inflight_factors -= 1
            self.refactoring.add(req.target)
        req.miss = True
        return (req, "resolve", slot)

    # ---- the loop ------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0):
        """Serve `requests` (sorted by arrival); returns them with results.

        Arrival times are in seconds and replayed in real time divided by
        time_scale.
        """
        torch = self.torch
        todo = queue.Queue()
        finished = []
        free_workers = threading.Semaphore(self.slots)
        self._by_rid = {r.rid: r for r in requests}
        for r in requests:
            if r.kind == "factor" and not r.key:
                r.key = pattern_key(r.system)

        def worker():
            stream = torch.cuda.Stream()
            while True:
                item = todo.get()
                if item is None:
                    return
                req, kind, slot = item
                req.start = time.perf_counter() - t0
                try:
                    if kind == "factor":
                        self._run_factor(req, slot, stream)
                    else:
                        self._run_resolve(req, slot, stream)
                except Exception as e:  # recorded, the loop goes on
                    req.status = f"error: {e}"
                    with self.lock:
                        slot.in_use = max(0, slot.in_use - 1)
                        if kind == "factor":
                            self.inflight_factors -= 1
                req.done = time.perf_counter() - t0
                finished.append(req)
                free_workers.release()
                with self.wake:
                    self.wake.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for th in threads:
            th.start()
        pending = list(requests)
        seen = set(self.sym_cache)
        waiting = []
        t0 = time.perf_counter()
        i = 0
        while i < len(pending) or waiting:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival / time_scale <= now:
                r = pending[i]
                if r.kind == "factor":
                    r.cold = r.key not in seen
                    seen.add(r.key)
                waiting.append(r)
                i += 1
            self._factors_pending = any(r.kind == "factor" for r in waiting)
            progressed = False
            for req in list(waiting):
                if not free_workers.acquire(blocking=False):
                    break
                got = self._dispatch_factor(req) if req.kind == "factor" else self._dispatch_resolve(req)
                if got is None:
                    free_workers.release()
                    continue
                waiting.remove(req)
                progressed = True
                if got == "done":
                    free_workers.release()
                    req.done = time.perf_counter() - t0
                    finished.append(req)
                    continue
                todo.put(got)
            if not progressed:
                nxt = pending[i].arrival / time_scale - now if i < len(pending) else 0.01
                with self.wake:
                    self.wake.wait(timeout=max(0.0002, min(0.002, nxt)))
        for _ in threads:
            todo.put(None)
        for th in threads:
            th.join()
        return sorted(finished, key=lambda r: r.rid)

    def close(self):
        with self.lock:
            for sl in self.resident.values():
                sl.close()
            self.resident.clear()
            self.used = 0
        self.pool.shutdown(wait=True)


def _pcts(lat):
    lat = np.asarray(lat, dtype=np.float64)
    if not lat.size:
        return {"count": 0, "p50_ms": None, "p99_ms": None}
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99))}


def summarize(reqs, wall: float) -> dict:
    ok = [r for r in reqs if r.status == "ok"]
    lat = {r.rid: (r.done - r.arrival) * 1e3 for r in ok}
    solves = sum(r.nrhs for r in ok)
    res = [r for r in reqs if r.kind == "resolve"]
    out = {
        "requests": len(reqs), "ok": len(ok),
        "failed": sorted({r.status for r in reqs if r.status != "ok"}),
        "misses": sum(r.miss for r in reqs),
        "resolve_hit_rate": (sum(not r.miss for r in res if r.status == "ok") / len(res)) if res else None,
        "p50_ms": float(np.percentile(list(lat.values()), 50)) if lat else None,
        "p99_ms": float(np.percentile(list(lat.values()), 99)) if lat else None,
        "mean_ms": float(np.mean(list(lat.values()))) if lat else None,
        "solves_per_s": solves / wall if wall > 0 else None,
        "requests_per_s": len(ok) / wall if wall > 0 else None,
        "max_berr": float(max((r.berr for r in ok), default=float("nan"))),
        "factor_requests": sum(r.kind == "factor" for r in ok),
        "resolve_requests": sum(r.kind == "resolve" for r in ok),
        "pooled_factor_requests": sum(r.pooled for r in ok if r.kind == "factor"),
        "cold": _pcts([lat[r.rid] for r in ok if r.kind == "factor" and r.cold]),
        "warm": _pcts([lat[r.rid] for r in ok if r.kind == "factor" and not r.cold]),
        "resolve": _pcts([lat[r.rid] for r in ok if r.kind == "resolve"]),
    }
    return out


def make_requests(count: int, rate_hz: float, seed: int = 0, system_fn=None, max_side=None):
    """Requests of the serving mix (workloads.serving_requests): factor
    requests carry their system (built by system_fn(kind, side), cached per
    pattern); a re-solve carries its `pick` (which resident factor) and, for
    the fixed policy, a target chosen with the same pick among the factor
    requests before it.  max_side clamps grid sides (smaller tests)."""
    from . import workloads as W
    specs = W.serving_requests(count, rate_hz, seed)
    cache = {}
    out = []
    factors = []
    for sp in specs:
        if sp["kind"] == "factor":
            kind, side = sp["sys"]
            if max_side is not None:
                side = min(side, max_side[kind])
            key = (kind, side)
            if key not in cache:
                sysm = system_fn(kind, side) if system_fn else W.batch_system(
                    len(cache), kind, side, seed, nrhs=sp["nrhs"], workload=W.W_SERVE)
                cache[key] = (sysm, pattern_key(sysm))
            scale = 1.0 + 0.5 * ((sp["id"] * 0.6180339887498949) % 1.0)
            r = Request(rid=sp["id"], arrival=sp["t"], kind="factor", system=cache[key][0],
                        values_scale=scale, nrhs=sp["nrhs"], key=cache[key][1])
            factors.append(r.rid)
        else:
            if not factors:
                continue
            tgt = factors[min(int(sp["pick"] * len(factors)), len(factors) - 1)]
            r = Request(rid=sp["id"], arrival=sp["t"], kind="resolve", target=tgt, pick=sp["pick"],
                        nrhs=sp["nrhs"])
        out.append(r)
    return out
