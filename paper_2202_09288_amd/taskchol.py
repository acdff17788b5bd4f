"""Python binding of libtaskchol.so (include/taskchol.h): the paper's
task-parallel supernodal Cholesky on the host cores, the multicore CPU
baseline beside the GPU library.  Argument marshalling only.

    plan = TaskPlan.from_symbolic(sym, colptr, rowidx)   # sym: spchol.Symbolic
    Lx, run = plan.factor(values, "opt_d_cost", threads=16)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtaskchol.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2202_09288_amd/build.py")
_lib = ctypes.CDLL(LIB_PATH)

STRATEGIES = {"nonested": 0, "nested": 1, "opt_d": 2, "opt_d_cost": 3, "mt_blas": 4, "hybrid": 5}
NAMES = {v: k for k, v in STRATEGIES.items()}


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n", "nsuper", "nnz_a_full", "updates", "max_updates", "opt_d", "split_opt_d", "tasks_nonested",
        "tasks_nested", "tasks_opt_d", "tasks_opt_d_cost")] + [
        ("avg_supernode_cols", ctypes.c_double), ("density", ctypes.c_double),
        ("hybrid_choice", ctypes.c_int32), ("flops", ctypes.c_double)]


class _Run(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("strategy", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("d", ctypes.c_int64), ("inner_tasks", ctypes.c_int64), ("bad_column", ctypes.c_int64)]


_P = ctypes.c_void_p
_lib.tch_plan_create.argtypes = [ctypes.c_int64, ctypes.c_int32] + [_P] * 8 + [ctypes.POINTER(_P)]
_lib.tch_plan_create.restype = ctypes.c_int
_lib.tch_plan_stats.argtypes = [_P, ctypes.POINTER(_Stats)]
_lib.tch_plan_stats.restype = ctypes.c_int
_lib.tch_plan_update_counts.argtypes = [_P, _P]
_lib.tch_plan_update_counts.restype = ctypes.c_int
_lib.tch_opt_d.argtypes = [ctypes.c_int64, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64)]
_lib.tch_opt_d.restype = ctypes.c_int
_lib.tch_hybrid_choice.argtypes = [ctypes.c_double, ctypes.c_double]
_lib.tch_hybrid_choice.restype = ctypes.c_int
_lib.tch_factor.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                            ctypes.POINTER(_Run)]
_lib.tch_factor.restype = ctypes.c_int
_lib.tch_plan_free.argtypes = [_P]
_lib.tch_plan_free.restype = None
EXPORTS = ("tch_plan_create", "tch_plan_stats", "tch_plan_update_counts", "tch_opt_d", "tch_hybrid_choice",
           "tch_factor", "tch_plan_free")


class NotSPD(RuntimeError):
    def __init__(self, column):
        super().__init__(f"matrix is not positive definite at permuted column {column}")
        self.column = column


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def opt_d(n: int, C) -> int:
    """Algorithm 1 (Opt-D) on the update counts C."""
    c = np.ascontiguousarray(C, dtype=np.int32)
    d = ctypes.c_int64(0)
    if _lib.tch_opt_d(int(n), int(c.size), _ptr(c), ctypes.byref(d)) != 0:
        raise ValueError("tch_opt_d: invalid input")
    return int(d.value)


def hybrid_choice(avg_supernode_cols: float, density: float) -> str:
    return NAMES[_lib.tch_hybrid_choice(float(avg_supernode_cols), float(density))]


class TaskPlan:
    def __init__(self, n, perm, super_ptr, sparent, rptr, rows, colcount, colptr, rowidx):
        self._keep = [np.ascontiguousarray(a, dtype=dt) for a, dt in (
            (perm, np.int32), (super_ptr, np.int32), (sparent, np.int32), (rptr, np.int64), (rows, np.int32),
            (colcount, np.int32), (colptr, np.int64), (rowidx, np.int32))]
        h = _P()
        ns = self._keep[1].size - 1
        rc = _lib.tch_plan_create(int(n), int(ns), *[_ptr(a) for a in self._keep], ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"tch_plan_create failed ({rc})")
        self._h = h
        self.n = int(n)
        self.nsuper = int(ns)
        rp = self._keep[3]; sp = self._keep[1]
        self.panel_entries = int(np.sum(np.diff(rp) * np.diff(sp).astype(np.int64)))

    @classmethod
    def from_symbolic(cls, sym, colptr, rowidx):
        """The structure of a GPU-library analysis (spchol.Symbolic)."""
        e = sym.export
        return cls(sym.n, e("perm"), e("super_ptr"), e("sparent"), e("rptr"), e("rows"), e("colcount"),
                   colptr, rowidx)

    def stats(self) -> dict:
        st = _Stats()
        _lib.tch_plan_stats(self._h, ctypes.byref(st))
        out = {k: getattr(st, k) for k, _ in _Stats._fields_}
        out["hybrid_choice"] = NAMES[out["hybrid_choice"]]
        return out

    def update_counts(self) -> np.ndarray:
        C = np.zeros(max(self.nsuper, 1), dtype=np.int32)
        _lib.tch_plan_update_counts(self._h, _ptr(C))
        return C[: self.nsuper]

    def factor(self, values, strategy: str = "hybrid", threads: int = 0, d: int = 0, cost: float = 0.0):
        v = np.ascontiguousarray(values, dtype=np.float64)
        Lx = np.zeros(max(self.panel_entries, 1), dtype=np.float64)
        run = _Run()
        rc = _lib.tch_factor(self._h, _ptr(v), _ptr(Lx), STRATEGIES[strategy], int(threads), int(d), float(cost),
                             ctypes.byref(run))
        if rc == -2:
            raise NotSPD(int(run.bad_column))
        if rc != 0:
            raise ValueError(f"tch_factor failed ({rc})")
        info = {"seconds": run.seconds, "strategy": NAMES[run.strategy], "threads": run.threads, "d": run.d,
                "inner_tasks": run.inner_tasks}
        return Lx[: self.panel_entries], info

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.tch_plan_free(self._h)
            self._h = None

    def __del__(self):
        self.close()
