"""Continuous-batching serving loop over the C ABI.

Requests are factor-then-solve (a new SPD system and right-hand sides) or
re-solve (new right-hand sides for a factor kept resident from an earlier
request).  The loop admits requests as slots and device memory free up:

  - a slot is a worker thread with its own HIP stream (default priority), so
    the work of requests in different slots overlaps on the device; the
    library calls release the GIL;
  - admission is by footprint: a factor request needs the factor bytes the
    analysis reports (plus solve and refinement workspace), and it waits
    while admitting it would exceed the HBM budget; resident factors that
    are not in use are evicted (least recently used first) to make room;
  - the analysis of a pattern is cached (keyed by the pattern), so repeated
    patterns skip the host analysis;
  - every solve is FP32 factor + FP64 refinement to the backward-error
    tolerance, and the result records latency (completion - arrival).

The paper's analyze/factorize/solve phases (Sec. 1-2) are the unit of work;
keeping factors for repeated solves is the resident-factor cache.
"""
from __future__ import annotations

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
    target: int = -1               # resolve requests: rid of the factor request
    nrhs: int = 8
    # filled in by the server
    start: float = -1.0
    done: float = -1.0
    berr: float = float("nan")
    iterations: int = -1
    factor_key: int = -1
    miss: bool = False             # resolve whose factor had been evicted
    status: str = "pending"
    X: object = None               # host solution when keep_solutions


def pattern_key(s) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(s.colptr).tobytes())
    h.update(np.ascontiguousarray(s.rowidx).tobytes())
    h.update(np.ascontiguousarray(s.perm).tobytes())
    return h.hexdigest()


class Resident:
    def __init__(self, key, factor, d_values, system, nbytes, scale):
        self.key = key
        self.factor = factor
        self.d_values = d_values
        self.system = system
        self.nbytes = nbytes
        self.scale = scale
        self.lock = threading.Lock()
        self.in_use = 0


class Server:
    """Serve a list of requests with arrival times; see module docstring."""

    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, precision: str = "fp32",
                 tol: float = 1e-12, maxit: int = 50, keep_solutions: bool = False,
                 max_resident: int = 64, handover: bool = False):
        import torch
        from . import spchol
        self.torch = torch
        self.lib = spchol
        self.slots = slots
        self.budget = int(hbm_budget)
        self.precision = precision
        self.tol = tol
        self.maxit = maxit
        self.keep_solutions = keep_solutions
        self.max_resident = max_resident
        # in-launch TRSM hand-over (waits inside a launch) for the
        # factorizations; off by default, since the slots' factorizations
        # share the device on several streams
        self.tuning = {"handover": 1 if handover else -1}
        self.sym_cache = {}
        self.sym_lock = threading.Lock()
        self.resident = OrderedDict()      # key -> Resident (LRU order)
        self.res_lock = threading.Lock()
        self.used = 0                      # bytes admitted or resident
        self.mem_cv = threading.Condition()
        self.refactoring = set()           # targets being factored again

    # ---- memory accounting ------------------------------------------------
    def footprint(self, sym, nrhs: int) -> int:
        i = sym.info
        fac = i["factor_bytes_fp32"] if self.precision == "fp32" else i["factor_bytes_fp64"]
        n = i["n"]
        work = n * 16 * (3 * (4 if self.precision == "fp32" else 8)) + n * 16 * 8 * 7  # solve + refine
        csr = 2 * i["nnz_a"] * 12 + 8 * n
        vals = i["nnz_a"] * 8 + 2 * n * nrhs * 8
        return int(fac + work + csr + vals)

    def _reserve(self, nbytes: int) -> bool:
        """Reserve device bytes, evicting idle resident factors (LRU)."""
        with self.mem_cv:
            while self.used + nbytes > self.budget:
                victim = None
                with self.res_lock:
                    for k, r in self.resident.items():
                        if r.in_use == 0:
                            victim = k
                            break
                    if victim is not None:
                        r = self.resident.pop(victim)
                if victim is None:
                    return False
                r.factor.close()
                self.used -= r.nbytes
            self.used += nbytes
            return True

    def _release(self, nbytes: int):
        with self.mem_cv:
            self.used -= nbytes
            self.mem_cv.notify_all()

    def symbolic(self, s):
        key = pattern_key(s)
        with self.sym_lock:
            sym = self.sym_cache.get(key)
            if sym is None:
                sym = self.lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, self.tuning)
                self.sym_cache[key] = sym
        return sym

    # ---- work of one request (runs in a slot thread) ------------------------
    def _run_factor(self, req: Request, stream, sym, nbytes, hold: bool = False):
        torch = self.torch
        s = req.system
        with torch.cuda.stream(stream):
            dv = torch.from_numpy(s.values * req.values_scale).to("cuda", non_blocking=False)
            F = self.lib.factorize(sym, dv, self.precision, stream=stream)
            B = torch.from_numpy(self.rhs(req)).cuda()
            X = torch.zeros_like(B)
            F.sync()
            info = F.solve_refined(dv, B, X, tol=self.tol, maxit=self.maxit, stream=stream)
            stream.synchronize()
        req.berr = info["berr"]
        req.iterations = info["iterations"]
        req.status = "ok" if info["converged"] else "no-convergence"
        if self.keep_solutions:
            req.X = X.cpu().numpy().T.copy()
        victims = []
        with self.res_lock:  # never take mem_cv while holding res_lock
            key = req.target if req.kind == "resolve" else req.rid
            old = self.resident.get(key)
            if old is not None and old.in_use > 0:
                # a user still holds the current one: keep it, drop ours
                if hold:
                    old.in_use += 1
                new = old
                victims.append(Resident(key, F, dv, s, nbytes, req.values_scale))
            else:
                if old is not None:
                    victims.append(self.resident.pop(key))
                new = Resident(key, F, dv, s, nbytes, req.values_scale)
                new.in_use = 1 if hold else 0  # held: not evictable until released
                self.resident[key] = new
            req.factor_key = key
            # cap the number of resident factors
            while len(self.resident) > self.max_resident:
                k0 = next((k for k, r in self.resident.items() if r.in_use == 0), None)
                if k0 is None:
                    break
                victims.append(self.resident.pop(k0))
        for r in victims:
            r.factor.close()
            self._release(r.nbytes)
        return new

    def _run_refactor(self, req: Request, stream, sym, nbytes, tgt: Request):
        """A re-solve whose factor was evicted: factor the target's system
        again (it becomes resident under the target's id) and solve."""
        shadow = Request(rid=tgt.rid, arrival=req.arrival, kind="factor", system=tgt.system,
                         values_scale=tgt.values_scale, nrhs=req.nrhs)
        try:
            res = self._run_factor(shadow, stream, sym, nbytes, hold=True)
        finally:
            self.refactoring.discard(tgt.rid)
        try:
            self._run_resolve(req, stream, res)
        finally:
            with self.res_lock:
                res.in_use -= 1

    def _run_resolve(self, req: Request, stream, res: Resident):
        torch = self.torch
        s = res.system
        with res.lock, torch.cuda.stream(stream):
            B = torch.from_numpy(self.rhs(req, s)).cuda()
            X = torch.zeros_like(B)
            info = res.factor.solve_refined(res.d_values, B, X, tol=self.tol, maxit=self.maxit, stream=stream)
            stream.synchronize()
        req.berr = info["berr"]
        req.iterations = info["iterations"]
        req.status = "ok" if info["converged"] else "no-convergence"
        req.factor_key = res.key
        if self.keep_solutions:
            req.X = X.cpu().numpy().T.copy()

    @staticmethod
    def rhs(req: Request, system=None):
        """(nrhs, n) right-hand sides: the system's own for a factor request,
        seeded by the request id for a re-solve."""
        if req.kind == "factor":
            return np.ascontiguousarray(req.system.B[:, :req.nrhs].T)
        from .workloads import uniform, stream_key, W_SERVE, P_RHS
        u = uniform(stream_key(W_SERVE, 0, P_RHS, req.rid), req.nrhs * system.n)
        return np.ascontiguousarray((2.0 * u - 1.0).reshape(req.nrhs, system.n))

    # ---- the loop ------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0):
        """Serve `requests` (sorted by arrival); returns them with results.

        Arrival times are in seconds and replayed in real time divided by
        time_scale.  Re-solve requests that arrive before any factor is
        resident wait for one.
        """
        torch = self.torch
        todo = queue.Queue()
        finished = []
        fin_lock = threading.Lock()
        slot_free = threading.Semaphore(self.slots)

        def worker(idx):
            stream = torch.cuda.Stream()
            while True:
                item = todo.get()
                if item is None:
                    return
                req, payload = item
                req.start = time.perf_counter() - t0
                try:
                    if req.kind == "factor":
                        sym, nbytes = payload
                        self._run_factor(req, stream, sym, nbytes)
                    elif isinstance(payload, tuple):
                        _, sym, nbytes, tgt = payload
                        self._run_refactor(req, stream, sym, nbytes, tgt)
                    else:
                        try:
                            self._run_resolve(req, stream, payload)
                        finally:
                            with self.res_lock:
                                payload.in_use -= 1
                except Exception as e:  # recorded, the loop goes on
                    req.status = f"error: {e}"
                    if isinstance(payload, tuple):
                        self._release(payload[-2] if len(payload) == 4 else payload[1])
                req.done = time.perf_counter() - t0
                with fin_lock:
                    finished.append(req)
                slot_free.release()

        threads = [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(self.slots)]
        for th in threads:
            th.start()
        pending = list(requests)
        by_rid = {r.rid: r for r in pending}
        waiting = []
        t0 = time.perf_counter()
        i = 0
        while i < len(pending) or waiting:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival / time_scale <= now:
                waiting.append(pending[i])
                i += 1
            if not waiting:
                nxt = pending[i].arrival / time_scale
                time.sleep(max(0.0, min(0.01, nxt - now)))
                continue
            req = waiting[0]
            if req.kind == "resolve":
                with self.res_lock:
                    res = self.resident.get(req.target)
                    if res is not None:
                        res.in_use += 1
                        self.resident.move_to_end(req.target)
                if res is None:
                    tgt = by_rid.get(req.target)
                    if tgt is not None and tgt.done < 0 and tgt.status == "pending":
                        # its factor is queued or in flight: serve others first
                        nxt_req = next((r for r in waiting if r.kind == "factor"), None)
                        if nxt_req is not None:
                            waiting.remove(nxt_req)
                            waiting.insert(0, nxt_req)
                        else:
                            time.sleep(0.0005)
                        continue
                    if tgt is None or tgt.status != "ok":
                        req.status = "no-resident-factor"
                        waiting.pop(0)
                        with fin_lock:
                            finished.append(req)
                        continue
                    if req.target in self.refactoring:
                        time.sleep(0.0005)  # another re-solve is refactoring it
                        continue
                    # evicted: factor the target's system again (a miss)
                    req.miss = True
                    sym = self.symbolic(tgt.system)
                    nbytes = self.footprint(sym, req.nrhs)
                    if not self._reserve(nbytes):
                        with self.mem_cv:
                            self.mem_cv.wait(timeout=0.01)
                        continue
                    slot_free.acquire()
                    waiting.pop(0)
                    self.refactoring.add(req.target)
                    todo.put((req, ("refactor", sym, nbytes, tgt)))
                    continue
                slot_free.acquire()
                waiting.pop(0)
                todo.put((req, res))
                continue
            sym = self.symbolic(req.system)
            nbytes = self.footprint(sym, req.nrhs)
            if nbytes > self.budget:
                req.status = "rejected: footprint above budget"
                waiting.pop(0)
                finished.append(req)
                continue
            if not self._reserve(nbytes):
                with self.mem_cv:
                    self.mem_cv.wait(timeout=0.01)
                continue
            slot_free.acquire()
            waiting.pop(0)
            todo.put((req, (sym, nbytes)))
        for _ in threads:
            todo.put(None)
        for th in threads:
            th.join()
        return sorted(finished, key=lambda r: r.rid)

    def close(self):
        with self.res_lock:
            for r in self.resident.values():
                r.factor.close()
            self.resident.clear()
        self.used = 0


def summarize(reqs, wall: float) -> dict:
    ok = [r for r in reqs if r.status == "ok"]
    lat = np.array([r.done - r.arrival for r in ok]) * 1e3
    solves = sum(r.nrhs for r in ok)
    return {
        "requests": len(reqs), "ok": len(ok),
        "failed": sorted({r.status for r in reqs if r.status != "ok"}),
        "misses": sum(r.miss for r in reqs),
        "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_ms": float(lat.mean()) if lat.size else None,
        "solves_per_s": solves / wall if wall > 0 else None,
        "requests_per_s": len(ok) / wall if wall > 0 else None,
        "max_berr": float(max((r.berr for r in ok), default=float("nan"))),
        "factor_requests": sum(r.kind == "factor" for r in ok),
        "resolve_requests": sum(r.kind == "resolve" for r in ok),
    }


def make_requests(count: int, rate_hz: float, seed: int = 0, system_fn=None, max_side=None):
    """Requests of the serving mix (workloads.serving_requests): factor
    requests carry their system (built by system_fn(kind, side), cached per
    pattern), re-solves target an earlier factor request, chosen uniformly
    from those before it.  max_side clamps grid sides (smaller tests)."""
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
                cache[key] = system_fn(kind, side) if system_fn else W.batch_system(
                    len(cache), kind, side, seed, nrhs=sp["nrhs"], workload=W.W_SERVE)
            scale = 1.0 + 0.5 * ((sp["id"] * 0.6180339887498949) % 1.0)
            r = Request(rid=sp["id"], arrival=sp["t"], kind="factor", system=cache[key],
                        values_scale=scale, nrhs=sp["nrhs"])
            factors.append(r.rid)
        else:
            if not factors:
                continue
            tgt = factors[min(int(sp["pick"] * len(factors)), len(factors) - 1)]
            r = Request(rid=sp["id"], arrival=sp["t"], kind="resolve", target=tgt, nrhs=sp["nrhs"])
        out.append(r)
    return out
