"""Python binding of libspchol.so (the C ABI in include/spchol.h).

Argument marshalling only: every numeric step runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device and the
stream is torch's current stream unless one is given.  Importing this module
loads the library and fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspchol.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2202_09288_amd/build.py "
                      "(or __graft_entry__.build())")

# torch ships its own HIP runtime and refers to it by a name the loader does
# not match against an already loaded /opt/rocm copy; loading torch first
# makes libspchol.so bind to torch's runtime, so the process holds one HIP
# runtime and both see the device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, INVALID_INPUT, NOT_SPD, OUT_OF_MEMORY, NO_CONVERGENCE, DEVICE_ERROR, BAD_HANDLE, NO_DEVICE = \
    0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32, FP32_BF16UPD = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "bf16upd": FP32_BF16UPD, FP64: FP64, FP32: FP32, FP32_BF16UPD: FP32_BF16UPD}

EXPORTS = ("spc_analyze", "spc_symbolic_info", "spc_symbolic_verify", "spc_symbolic_export", "spc_factorize",
           "spc_refactorize", "spc_factorize_batch", "spc_solve", "spc_solve_refined", "spc_sync",
           "spc_factor_export", "spc_factor_last_ms", "spc_factor_set_profiling",
           "spc_factor_kernel_stats", "spc_free_symbolic", "spc_free_factor", "spc_status_string",
           "spc_last_error_message", "spc_batch_create", "spc_batch_factorize", "spc_batch_factor",
           "spc_batch_solve", "spc_batch_sync", "spc_batch_last_ms", "spc_batch_info", "spc_free_batch",
           "spc_batch_set_profiling", "spc_batch_kernel_stats", "spc_batch_solve_refined",
           "spc_factor_set_graph", "spc_batch_set_graph", "spc_factor_level_stats", "spc_batch_level_stats",
           "spc_factor_set_wait_limit", "spc_solve_noalloc", "spc_factor_pivot_floors", "spc_order")
KERNEL_CLASSES = {"assemble": 0, "potrf": 1, "trsm": 2, "trailing": 3, "scatter": 4, "scatter_big": 5,
                  "small": 6, "tiny": 7, "small_trees": 8}
# kernel behind each class (as rocprofv3 names it, precision filled in)
KERNEL_NAMES = {"potrf": "k_potrf<{t}, false>", "trsm": "k_tiles<{t}, 2, false>", "trailing": "k_tiles<{t}, 0, false>",
                "scatter": "k_tiles<{t}, 1, false>", "scatter_big": "k_tiles128<{t}, false, false>", "small": "k_small<{t}>",
                "tiny": "k_tiny<{t}>", "small_trees": "k_persist_small<{t}>",
                "assemble": "k_zero<{t}> + k_assemble<{t}>"}


# schedule cut-offs of spc_options (0: library default, < 0: path off)
TUNING_FIELDS = ("tiny_w", "tiny_m", "small_w", "small_m", "big_min", "big_min_k", "solve_persist_max",
                 "handover", "delay", "persist", "ordering", "group", "bulk128", "lookahead")


class _Options(ctypes.Structure):
    _fields_ = [("amalg_z", ctypes.c_double)] + [(k, ctypes.c_int32) for k in TUNING_FIELDS] + [
        ("hbm_budget", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n", "nnz_a", "nsuper", "nnz_l", "panel_entries", "flops", "levels", "rows_total",
        "max_width", "max_rows", "factor_bytes_fp64", "factor_bytes_fp32", "solve_levels",
        "solve_persistent_levels", "solve_block_tasks", "solve_tiny_tasks", "updates_total",
        "solve_handovers")]


class _KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("flops", ctypes.c_double)]


class _RefineInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("berr", ctypes.c_double)]


_P = ctypes.c_void_p
_i64 = ctypes.c_int64
_lib.spc_analyze.argtypes = [_i64, _P, _P, _P, ctypes.POINTER(_Options), ctypes.POINTER(_P)]
_lib.spc_symbolic_info.argtypes = [_P, ctypes.POINTER(_Info)]
_lib.spc_order.argtypes = [_i64, _P, _P, ctypes.c_int, _P]
_lib.spc_symbolic_verify.argtypes = [_P]
_lib.spc_symbolic_export.argtypes = [_P, ctypes.c_int, _P]
_lib.spc_factorize.argtypes = [_P, _P, ctypes.c_int, _P, ctypes.POINTER(_P)]
_lib.spc_refactorize.argtypes = [_P, _P, _P]
_lib.spc_factorize_batch.argtypes = [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int,
                                     _P, ctypes.POINTER(_P)]
_lib.spc_solve.argtypes = [_P, _P, ctypes.c_int, _i64, _P]
_lib.spc_solve_noalloc.argtypes = [_P, _P, ctypes.c_int, _i64, _P]
_lib.spc_solve_refined.argtypes = [_P, _P, _P, _P, ctypes.c_int, _i64, ctypes.c_double, ctypes.c_int, _P,
                                   ctypes.POINTER(_RefineInfo)]
_lib.spc_sync.argtypes = [_P, ctypes.POINTER(_i64)]
_lib.spc_factor_export.argtypes = [_P, _P]
_lib.spc_factor_last_ms.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.spc_factor_set_profiling.argtypes = [_P, ctypes.c_int]
_lib.spc_factor_kernel_stats.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_KernelStats)]
_lib.spc_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P)]
_lib.spc_batch_factorize.argtypes = [_P, ctypes.POINTER(_P), _P]
_lib.spc_batch_factor.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_P)]
_lib.spc_batch_solve.argtypes = [_P, ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_i64), _P]
_lib.spc_batch_solve_refined.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int,
                                         ctypes.POINTER(_i64), ctypes.c_double, ctypes.c_int, _P,
                                         ctypes.POINTER(_RefineInfo)]
_lib.spc_factor_set_graph.argtypes = [_P, ctypes.c_int]
_lib.spc_factor_set_wait_limit.argtypes = [_P, ctypes.c_int32]
_lib.spc_factor_pivot_floors.argtypes = [_P, ctypes.POINTER(_i64)]
_lib.spc_factor_level_stats.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_KernelStats)]
_lib.spc_batch_level_stats.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_KernelStats)]
_lib.spc_batch_set_graph.argtypes = [_P, ctypes.c_int]
_lib.spc_batch_sync.argtypes = [_P, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.spc_batch_last_ms.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.spc_batch_info.argtypes = [_P, ctypes.POINTER(_Info)]
_lib.spc_batch_set_profiling.argtypes = [_P, ctypes.c_int]
_lib.spc_batch_kernel_stats.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_KernelStats)]
_lib.spc_free_batch.argtypes = [_P]
_lib.spc_free_batch.restype = None
_lib.spc_free_symbolic.argtypes = [_P]
_lib.spc_free_symbolic.restype = None
_lib.spc_free_factor.argtypes = [_P]
_lib.spc_free_factor.restype = None
_lib.spc_status_string.argtypes = [ctypes.c_int]
_lib.spc_status_string.restype = ctypes.c_char_p
_lib.spc_last_error_message.argtypes = []
_lib.spc_last_error_message.restype = ctypes.c_char_p
for _name in EXPORTS:
    if _name not in ("spc_free_symbolic", "spc_free_factor", "spc_status_string", "spc_last_error_message",
                     "spc_free_batch"):
        getattr(_lib, _name).restype = ctypes.c_int


class SpcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = _lib.spc_status_string(status).decode()
        if status in (DEVICE_ERROR, OUT_OF_MEMORY):
            detail = _lib.spc_last_error_message().decode()
            if detail:
                msg += f" [{detail}]"
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


class NotSPD(SpcError):
    def __init__(self, column: int, system: int = -1):
        where = f"system {system}, " if system >= 0 else ""
        super().__init__(NOT_SPD, f"pivot failed at {where}permuted column {column}")
        self.column = column
        self.system = system


def _check(rc: int, what: str):
    if rc != OK:
        raise SpcError(rc, what)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device (cuda/hip) torch tensor")
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _values_ptr(sym: "Symbolic", t):
    """Device pointer of a value array of sym's pattern: float64, at least
    one entry per stored entry of the lower CSC (the library reads the first
    nnz(lower A) of them)."""
    p = _dev_ptr(t, "torch.float64")
    if t.numel() < sym.info["nnz_a"]:
        raise ValueError(f"values must hold nnz(lower A) = {sym.info['nnz_a']} entries, got {t.numel()}")
    return p


def _rhs_count(B, n: int, what: str = "B") -> int:
    """Right-hand sides of a (n,) or (nrhs, n) tensor."""
    if B.dim() not in (1, 2) or B.shape[-1] != n:
        raise ValueError(f"{what} must have shape (n,) or (nrhs, n) with n = {n}, got {tuple(B.shape)}")
    return 1 if B.dim() == 1 else int(B.shape[0])


def _batch_rhs(syms, Bs, what: str = "Bs") -> int:
    """Common right-hand-side count of one tensor per system of a batch."""
    if len(Bs) != len(syms):
        raise ValueError(f"{what}: expected {len(syms)} tensors (one per system), got {len(Bs)}")
    counts = {_rhs_count(b, s.n, f"{what}[{i}]") for i, (s, b) in enumerate(zip(syms, Bs))}
    if len(counts) > 1:
        raise ValueError(f"{what}: every system needs the same number of right-hand sides")
    return counts.pop() if counts else 0


_EXPORT_ARRAYS = {"perm": (0, np.int32, "n"), "parent": (1, np.int32, "n"),
                  "colcount": (2, np.int32, "n"), "super_ptr": (3, np.int32, "ns1"),
                  "sparent": (4, np.int32, "ns"), "rptr": (5, np.int64, "ns1"),
                  "rows": (6, np.int32, "rows_total"), "lptr": (7, np.int64, "ns1"),
                  "level": (8, np.int32, "ns"), "uptr": (9, np.int64, "ns1"),
                  "ulist": (10, np.int32, "updates_total")}


class Symbolic:
    """spc_analyze: host-only symbolic analysis of a lower-CSC pattern."""

    def __init__(self, colptr, rowidx, perm=None, amalg_z: float = 0.05, tuning=None, hbm_budget: int = 0):
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        self._perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        n = self._colptr.size - 1
        if n < 0:
            raise ValueError("colptr needs n + 1 entries")
        if self._rowidx.size < max(int(self._colptr[-1]), 0):
            raise ValueError("rowidx is shorter than colptr[n]")
        if self._perm is not None and self._perm.size != n:
            raise ValueError(f"perm must have n = {n} entries")
        opts = _Options(amalg_z=float(amalg_z), hbm_budget=int(hbm_budget))
        self.tuning = dict(tuning or {})
        for k, v in self.tuning.items():
            if k not in TUNING_FIELDS:
                raise ValueError(f"unknown schedule cut-off {k!r}")
            setattr(opts, k, int(v))
        h = _P()
        rc = _lib.spc_analyze(n, _np_ptr(self._colptr), _np_ptr(self._rowidx),
                              _np_ptr(self._perm) if self._perm is not None else None,
                              ctypes.byref(opts), ctypes.byref(h))
        _check(rc, "spc_analyze")
        self._h = h
        info = _Info()
        _check(_lib.spc_symbolic_info(self._h, ctypes.byref(info)), "spc_symbolic_info")
        self.info = {k: int(getattr(info, k)) for k, _ in _Info._fields_}
        self._cache = {}

    @property
    def handle(self):
        return self._h

    @property
    def n(self) -> int:
        return self.info["n"]

    def verify(self) -> None:
        """Host check of the schedule's invariants (spc_symbolic_verify);
        raises SpcError naming the first violation."""
        rc = _lib.spc_symbolic_verify(self._h)
        if rc != 0:
            raise SpcError(rc, "spc_symbolic_verify: " + _lib.spc_last_error_message().decode())

    def export(self, name: str) -> np.ndarray:
        if name not in self._cache:
            which, dt, sz = _EXPORT_ARRAYS[name]
            i = self.info
            count = {"n": i["n"], "ns": i["nsuper"], "ns1": i["nsuper"] + 1,
                     "rows_total": i["rows_total"], "updates_total": i["updates_total"]}[sz]
            a = np.zeros(max(count, 1), dtype=dt)
            _check(_lib.spc_symbolic_export(self._h, which, _np_ptr(a)), "spc_symbolic_export")
            self._cache[name] = a[:count]
        return self._cache[name]

    def close(self):
        # (at interpreter exit the module's globals may already be gone)
        if getattr(self, "_h", None) and _lib is not None:
            _lib.spc_free_symbolic(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Factor:
    """A device-resident factor (spc_factorize)."""

    def __init__(self, sym: Symbolic, handle, precision: int):
        self.sym = sym
        self._h = handle
        self.precision = precision

    @property
    def handle(self):
        return self._h

    def refactorize(self, d_values, stream=None):
        _check(_lib.spc_refactorize(self._h, _values_ptr(self.sym, d_values), _stream_ptr(stream)),
               "spc_refactorize")

    def sync(self):
        bad = _i64(-1)
        rc = _lib.spc_sync(self._h, ctypes.byref(bad))
        if rc == NOT_SPD:
            raise NotSPD(int(bad.value))
        _check(rc, "spc_sync")

    def export(self) -> np.ndarray:
        out = np.zeros(max(self.sym.info["panel_entries"], 1), dtype=np.float64)
        _check(_lib.spc_factor_export(self._h, _np_ptr(out)), "spc_factor_export")
        return out[: self.sym.info["panel_entries"]]

    def last_ms(self) -> float:
        v = ctypes.c_float(0)
        _check(_lib.spc_factor_last_ms(self._h, ctypes.byref(v)), "spc_factor_last_ms")
        return float(v.value)

    def set_profiling(self, on: bool = True):
        _check(_lib.spc_factor_set_profiling(self._h, 1 if on else 0), "spc_factor_set_profiling")

    def level_stats(self) -> list:
        """Per elimination-tree level (-2 = the persistent launch over the
        small subtrees, -1 = the assembly, then levels 0..): launches, device
        ms and flops of the last profiled factorization."""
        out = []
        for lv in range(-2, self.sym.info["levels"]):
            st = _KernelStats()
            _check(_lib.spc_factor_level_stats(self._h, lv, ctypes.byref(st)), "spc_factor_level_stats")
            out.append({"level": lv, "launches": int(st.launches), "ms": float(st.total_ms),
                        "flops": float(st.flops)})
        return out

    def set_graph(self, on: bool = True):
        """Capture the factorization into a HIP graph and replay it."""
        _check(_lib.spc_factor_set_graph(self._h, 1 if on else 0), "spc_factor_set_graph")

    def pivot_floors(self) -> int:
        """BF16 updates: pivots of the last factorization raised to their
        floor (spc_factor_pivot_floors)."""
        v = _i64(0)
        _check(_lib.spc_factor_pivot_floors(self._h, ctypes.byref(v)), "spc_factor_pivot_floors")
        return int(v.value)

    def set_wait_limit(self, polls: int):
        """Polls before a bounded wait on another workgroup gives up
        (spc_factor_set_wait_limit; 0: every such wait gives up at once)."""
        _check(_lib.spc_factor_set_wait_limit(self._h, int(polls)), "spc_factor_set_wait_limit")

    def kernel_stats(self) -> dict:
        """Per kernel class: launches, total device ms and algorithmic flops of
        the last profiled factorization."""
        out = {}
        for name, cls in KERNEL_CLASSES.items():
            st = _KernelStats()
            _check(_lib.spc_factor_kernel_stats(self._h, cls, ctypes.byref(st)), "spc_factor_kernel_stats")
            out[name] = {"launches": int(st.launches), "ms": float(st.total_ms), "flops": float(st.flops)}
        return out

    def solve(self, B, stream=None):
        """In-place solve. B: float64 device tensor of shape (n,) or (nrhs, n)
        (each row one right-hand side, i.e. column-major n x nrhs)."""
        n = self.sym.n
        nrhs = _rhs_count(B, n)
        _check(_lib.spc_solve(self._h, _dev_ptr(B, "torch.float64"), nrhs, n, _stream_ptr(stream)),
               "spc_solve")
        return B

    def solve_noalloc(self, B, stream=None):
        """spc_solve_noalloc: the in-place solve of solve(), with its work in
        the library's fixed scratch array (no device allocation)."""
        n = self.sym.n
        nrhs = _rhs_count(B, n)
        rc = _lib.spc_solve_noalloc(self._h, _dev_ptr(B, "torch.float64"), nrhs, n, _stream_ptr(stream))
        if rc != OK:
            raise SpcError(rc, "spc_solve_noalloc: " + _lib.spc_last_error_message().decode())
        return B

    def solve_refined(self, d_values, B, X, tol: float = 1e-12, maxit: int = 10, stream=None):
        n = self.sym.n
        nrhs = _rhs_count(B, n)
        if tuple(X.shape) != tuple(B.shape):
            raise ValueError(f"X must have the shape of B {tuple(B.shape)}, got {tuple(X.shape)}")
        info = _RefineInfo()
        rc = _lib.spc_solve_refined(self._h, _values_ptr(self.sym, d_values),
                                    _dev_ptr(B, "torch.float64"), _dev_ptr(X, "torch.float64"),
                                    nrhs, n, float(tol), int(maxit), _stream_ptr(stream),
                                    ctypes.byref(info))
        res = {"iterations": int(info.iterations), "converged": bool(info.converged),
               "berr": float(info.berr)}
        if rc not in (OK, NO_CONVERGENCE):
            _check(rc, "spc_solve_refined")
        res["status"] = rc
        return res

    def close(self):
        # (at interpreter exit the module's globals may already be gone)
        if getattr(self, "_h", None) and _lib is not None:
            _lib.spc_free_factor(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Several systems merged into one elimination forest and one device
    schedule (spc_batch_*): factored and solved level by level together."""

    def __init__(self, syms, precision="fp64"):
        self.syms = list(syms)
        self.precision = _PREC[precision]
        hs = (_P * len(self.syms))(*[x.handle for x in self.syms])
        h = _P()
        _check(_lib.spc_batch_create(len(self.syms), hs, self.precision, ctypes.byref(h)), "spc_batch_create")
        self._h = h
        info = _Info()
        _check(_lib.spc_batch_info(self._h, ctypes.byref(info)), "spc_batch_info")
        self.info = {k: int(getattr(info, k)) for k, _ in _Info._fields_}

    def factorize(self, d_values_list, stream=None):
        if len(d_values_list) != len(self.syms):
            raise ValueError(f"expected {len(self.syms)} value arrays (one per system), got {len(d_values_list)}")
        vs = (_P * len(self.syms))(*[_values_ptr(s, v) for s, v in zip(self.syms, d_values_list)])
        _check(_lib.spc_batch_factorize(self._h, vs, _stream_ptr(stream)), "spc_batch_factorize")

    def factor(self, i: int) -> "Factor":
        h = _P()
        _check(_lib.spc_batch_factor(self._h, int(i), ctypes.byref(h)), "spc_batch_factor")
        return Factor(self.syms[i], h, self.precision)

    def solve(self, Bs, stream=None):
        """Bs[i]: float64 device tensor (nrhs, n_i), solved in place."""
        nrhs = _batch_rhs(self.syms, Bs)
        ptrs = (_P * len(Bs))(*[_dev_ptr(b, "torch.float64") for b in Bs])
        lds = (_i64 * len(Bs))(*[x.n for x in self.syms])
        _check(_lib.spc_batch_solve(self._h, ptrs, nrhs, lds, _stream_ptr(stream)), "spc_batch_solve")
        return Bs

    def solve_refined(self, Bs, Xs, tol: float = 1e-12, maxit: int = 10, stream=None):
        """Refined solve of every system (against the values of the last
        factorize): Bs[i], Xs[i] float64 device tensors (nrhs, n_i); returns
        the status and one {iterations, converged, berr} per system."""
        count = len(self.syms)
        nrhs = _batch_rhs(self.syms, Bs)
        if _batch_rhs(self.syms, Xs, "Xs") != nrhs:
            raise ValueError("Xs must have the right-hand-side count of Bs")
        bp = (_P * count)(*[_dev_ptr(b, "torch.float64") for b in Bs])
        xp = (_P * count)(*[_dev_ptr(x, "torch.float64") for x in Xs])
        lds = (_i64 * count)(*[x.n for x in self.syms])
        infos = (_RefineInfo * count)()
        rc = _lib.spc_batch_solve_refined(self._h, bp, xp, nrhs, lds, float(tol), int(maxit),
                                          _stream_ptr(stream), infos)
        if rc not in (OK, NO_CONVERGENCE):
            _check(rc, "spc_batch_solve_refined")
        per = [{"iterations": int(r.iterations), "converged": bool(r.converged), "berr": float(r.berr)}
               for r in infos]
        return {"status": rc, "systems": per}

    def sync(self):
        sy, col = _i64(-1), _i64(-1)
        rc = _lib.spc_batch_sync(self._h, ctypes.byref(sy), ctypes.byref(col))
        if rc == NOT_SPD:
            raise NotSPD(int(col.value), int(sy.value))
        _check(rc, "spc_batch_sync")

    def last_ms(self) -> float:
        v = ctypes.c_float(0)
        _check(_lib.spc_batch_last_ms(self._h, ctypes.byref(v)), "spc_batch_last_ms")
        return float(v.value)

    def set_profiling(self, on: bool = True):
        _check(_lib.spc_batch_set_profiling(self._h, 1 if on else 0), "spc_batch_set_profiling")

    def set_graph(self, on: bool = True):
        _check(_lib.spc_batch_set_graph(self._h, 1 if on else 0), "spc_batch_set_graph")

    def level_stats(self) -> list:
        """As Factor.level_stats, for the last profiled batch factorization."""
        out = []
        for lv in range(-2, self.info["levels"]):
            st = _KernelStats()
            _check(_lib.spc_batch_level_stats(self._h, lv, ctypes.byref(st)), "spc_batch_level_stats")
            out.append({"level": lv, "launches": int(st.launches), "ms": float(st.total_ms),
                        "flops": float(st.flops)})
        return out

    def kernel_stats(self) -> dict:
        out = {}
        for name, cls in KERNEL_CLASSES.items():
            st = _KernelStats()
            _check(_lib.spc_batch_kernel_stats(self._h, cls, ctypes.byref(st)), "spc_batch_kernel_stats")
            out[name] = {"launches": int(st.launches), "ms": float(st.total_ms), "flops": float(st.flops)}
        return out

    def close(self):
        # (at interpreter exit the module's globals may already be gone)
        if getattr(self, "_h", None) and _lib is not None:
            _lib.spc_free_batch(self._h)
            self._h = None

    def __del__(self):
        self.close()


ORDERINGS = {"natural": 0, "nd": 1, "md": 2}


def order(colptr, rowidx, method: str = "nd") -> np.ndarray:
    """spc_order: a fill-reducing order (perm[k] = original index of the
    k-th pivot) of a lower-CSC pattern without coordinates."""
    cp = np.ascontiguousarray(colptr, dtype=np.int64)
    ri = np.ascontiguousarray(rowidx, dtype=np.int32)
    n = cp.size - 1
    perm = np.zeros(max(n, 1), dtype=np.int32)
    rc = _lib.spc_order(n, _np_ptr(cp), _np_ptr(ri), ORDERINGS[method], _np_ptr(perm))
    if rc != OK:
        raise SpcError(rc, "spc_order: " + _lib.spc_last_error_message().decode())
    return perm[:n]


def analyze(colptr, rowidx, perm=None, amalg_z: float = 0.05, tuning=None) -> Symbolic:
    return Symbolic(colptr, rowidx, perm, amalg_z, tuning)


def factorize(sym: Symbolic, d_values, precision="fp64", stream=None) -> Factor:
    prec = _PREC[precision]
    h = _P()
    _check(_lib.spc_factorize(sym.handle, _values_ptr(sym, d_values), prec,
                              _stream_ptr(stream), ctypes.byref(h)), "spc_factorize")
    return Factor(sym, h, prec)


def factorize_batch(syms, d_values_list, precision="fp64", stream=None):
    prec = _PREC[precision]
    count = len(syms)
    if len(d_values_list) != count:
        raise ValueError(f"expected {count} value arrays (one per system), got {len(d_values_list)}")
    hs = (_P * count)(*[s.handle for s in syms])
    vs = (_P * count)(*[_values_ptr(s, v) for s, v in zip(syms, d_values_list)])
    outs = (_P * count)()
    _check(_lib.spc_factorize_batch(count, hs, vs, prec, _stream_ptr(stream), outs),
           "spc_factorize_batch")
    return [Factor(s, _P(outs[i]), prec) for i, s in enumerate(syms)]


def solve(F: Factor, B, stream=None):
    return F.solve(B, stream)
