"""Plain FP64 CPU oracle for supernodal sparse Cholesky (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads ``liboracle.so`` built from ``oracle.c`` (plain
C, no BLAS) and exposes:

    Symbolic(colptr, rowidx, perm, z)   analyze: etree, counts, supernodes
    Symbolic.factor(values)             left-looking numeric factorization
    Symbolic.solve(Lx, B)               L y = b, L^T x = y
    metrics: rel_frobenius, backward_error, residual helpers

The file header of ``oracle.c`` states what each step follows in the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.orc_analyze.restype = P
        lib.orc_analyze.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double]
        lib.orc_free.argtypes = [P]
        lib.orc_free.restype = None
        lib.orc_sizes.argtypes = [P, P]
        lib.orc_sizes.restype = None
        lib.orc_get.argtypes = [P, ctypes.c_int, P]
        lib.orc_get.restype = ctypes.c_int
        lib.orc_factor.argtypes = [P, P, P, P]
        lib.orc_factor.restype = ctypes.c_int
        lib.orc_solve.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64]
        lib.orc_solve.restype = None
        lib.orc_factor_parallel.argtypes = [P, P, P, P, ctypes.c_int, P, P, ctypes.c_int32]
        lib.orc_factor_parallel.restype = ctypes.c_int
        lib.orc_factor_subtree.argtypes = [P, P, ctypes.c_int32, P, P, P]
        lib.orc_factor_subtree.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


SIZE_KEYS = ("n", "nsuper", "nfund", "rows_total", "panel_entries", "flops", "nnzL",
             "nlevels", "updates_total", "zeros")
_GET = {"perm": (0, np.int32, "n"), "parent": (1, np.int32, "n"), "colcount": (2, np.int32, "n"),
        "super_ptr": (3, np.int32, "ns1"), "sparent": (4, np.int32, "ns"),
        "rptr": (5, np.int64, "ns1"), "rows": (6, np.int32, "rows_total"),
        "lptr": (7, np.int64, "ns1"), "uptr": (8, np.int64, "ns1"),
        "ulist": (9, np.int32, "updates_total"), "level": (10, np.int32, "ns"),
        "post": (11, np.int32, "n"), "Lp": (12, np.int64, "n1"), "Li": (13, np.int32, "Li"),
        "fund_ptr": (14, np.int32, "nf1")}

NOT_SPD = -2


class NotSPD(Exception):
    def __init__(self, column):
        super().__init__(f"matrix is not positive definite at permuted column {column}")
        self.column = column


class Symbolic:
    """Oracle analyze phase; arrays are fetched lazily by attribute name."""

    def __init__(self, colptr, rowidx, perm, z: float = 0.05):
        lib = _load()
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        self._perm = np.ascontiguousarray(perm, dtype=np.int32)
        n = self._colptr.size - 1
        self._h = lib.orc_analyze(n, _ptr(self._colptr), _ptr(self._rowidx), _ptr(self._perm),
                                  float(z))
        if not self._h:
            raise ValueError("oracle: malformed input")
        out = np.zeros(len(SIZE_KEYS), dtype=np.int64)
        lib.orc_sizes(self._h, _ptr(out))
        self.sizes = {k: int(v) for k, v in zip(SIZE_KEYS, out)}
        self.z = z
        self._cache = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    @property
    def n(self):
        return self.sizes["n"]

    @property
    def nsuper(self):
        return self.sizes["nsuper"]

    def get(self, name: str) -> np.ndarray:
        if name not in self._cache:
            which, dt, sz = _GET[name]
            s = self.sizes
            count = {"n": s["n"], "ns": s["nsuper"], "ns1": s["nsuper"] + 1, "n1": s["n"] + 1,
                     "rows_total": s["rows_total"], "updates_total": s["updates_total"],
                     "Li": s["nnzL"] - s["n"], "nf1": s["nfund"] + 1}[sz]
            a = np.zeros(count, dtype=dt)
            if count:
                _load().orc_get(self._h, which, _ptr(a))
            self._cache[name] = a
        return self._cache[name]

    def __getattr__(self, name):
        if name in _GET:
            return self.get(name)
        raise AttributeError(name)

    def factor(self, values, threads: int = 0) -> np.ndarray:
        """Left-looking factorization; threads > 0 runs the deterministic
        multi-threaded mode (whole supernodes per thread, level by level),
        whose result is bit-identical to the sequential one."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        Lx = np.zeros(max(self.sizes["panel_entries"], 1), dtype=np.float64)
        bad = np.zeros(1, dtype=np.int64)
        if threads > 0:
            used = np.zeros(1, dtype=np.int32)
            rc = _load().orc_factor_parallel(self._h, _ptr(v), _ptr(Lx), _ptr(bad), int(threads), _ptr(used),
                                             None, 0)
            self.threads_used = int(used[0])
        else:
            rc = _load().orc_factor(self._h, _ptr(v), _ptr(Lx), _ptr(bad))
            self.threads_used = 1
        if rc == NOT_SPD:
            raise NotSPD(int(bad[0]))
        return Lx[: self.sizes["panel_entries"]]

    def factor_subtree(self, values, root: int):
        """Panels of the subtree rooted at supernode ``root``.

        Returns (Lx, first): Lx holds the exact panels of supernodes
        first..root (zeros elsewhere).
        """
        v = np.ascontiguousarray(values, dtype=np.float64)
        Lx = np.zeros(max(self.sizes["panel_entries"], 1), dtype=np.float64)
        bad = np.zeros(1, dtype=np.int64)
        first = np.zeros(1, dtype=np.int32)
        rc = _load().orc_factor_subtree(self._h, _ptr(v), int(root), _ptr(Lx), _ptr(bad),
                                        _ptr(first))
        if rc == NOT_SPD:
            raise NotSPD(int(bad[0]))
        if rc != 0:
            raise ValueError("bad subtree root")
        return Lx[: self.sizes["panel_entries"]], int(first[0])

    def factor_forest(self, values, roots, threads: int = 1):
        """Panels of the subtrees of the supernodes ``roots`` (the rest of
        the returned array is zero), factored by the multi-threaded mode on
        ``threads`` threads; self.threads_used holds the count it ran with."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        r = np.ascontiguousarray(roots, dtype=np.int32)
        Lx = np.zeros(max(self.sizes["panel_entries"], 1), dtype=np.float64)
        bad = np.zeros(1, dtype=np.int64)
        used = np.zeros(1, dtype=np.int32)
        rc = _load().orc_factor_parallel(self._h, _ptr(v), _ptr(Lx), _ptr(bad), int(threads), _ptr(used),
                                         _ptr(r), int(r.size))
        self.threads_used = int(used[0])
        if rc == NOT_SPD:
            raise NotSPD(int(bad[0]))
        if rc != 0:
            raise ValueError("bad subtree root")
        return Lx[: self.sizes["panel_entries"]]

    def solve(self, Lx: np.ndarray, B: np.ndarray) -> np.ndarray:
        """Return A^{-1} B; B is (n, nrhs) or (n,)."""
        Lx = np.ascontiguousarray(Lx, dtype=np.float64)
        one = B.ndim == 1
        Bm = B[:, None] if one else B
        X = np.asfortranarray(Bm, dtype=np.float64).copy(order="F")
        _load().orc_solve(self._h, _ptr(Lx), _ptr(X), X.shape[1], X.shape[0])
        return X[:, 0] if one else X

    # ---- views of the supernodal storage ---------------------------------
    def panel(self, Lx: np.ndarray, s: int) -> np.ndarray:
        """Supernode s as an (m_s, w_s) array (rows R_s, columns cols(s))."""
        sp, rp, lp = self.super_ptr, self.rptr, self.lptr
        w = int(sp[s + 1] - sp[s]); m = int(rp[s + 1] - rp[s])
        return Lx[lp[s]:lp[s + 1]].reshape(w, m).T

    def lower_mask(self) -> np.ndarray:
        """True for stored entries on or below the diagonal of each block."""
        sp, rp = self.super_ptr, self.rptr
        mask = np.ones(self.sizes["panel_entries"], dtype=bool)
        lp = self.lptr
        for s in range(self.nsuper):
            w = int(sp[s + 1] - sp[s]); m = int(rp[s + 1] - rp[s])
            blk = mask[lp[s]:lp[s + 1]].reshape(w, m)
            blk[np.tril_indices(w, -1)] = False  # (col c, row i) with i < c
        return mask

    def to_dense_L(self, Lx: np.ndarray) -> np.ndarray:
        """Dense n x n lower factor (tiny problems only)."""
        n = self.n
        L = np.zeros((n, n))
        sp, rp = self.super_ptr, self.rptr
        for s in range(self.nsuper):
            P = self.panel(Lx, s)
            R = self.rows[rp[s]:rp[s + 1]]
            for c in range(P.shape[1]):
                j = sp[s] + c
                L[R[c:], j] = P[c:, c]
        return L


# ---- metrics ----------------------------------------------------------------

def full_csr(n, colptr, rowidx, values):
    """Full symmetric matrix (scipy CSR) from the lower CSC triple."""
    import scipy.sparse as sp
    c = np.repeat(np.arange(n), np.diff(colptr))
    r = rowidx.astype(np.int64)
    off = r != c
    rows = np.concatenate([r, c[off]]); cols = np.concatenate([c, r[off]])
    vals = np.concatenate([values, values[off]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def backward_error(n, colptr, rowidx, values, X, B) -> float:
    """max over RHS of ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), FP64."""
    A = full_csr(n, colptr, rowidx, values)
    X = X.reshape(n, -1); B = B.reshape(n, -1)
    R = B - A @ X
    normA = float(np.max(np.abs(A).sum(axis=1))) if n else 0.0
    eta = 0.0
    for k in range(X.shape[1]):
        den = normA * np.max(np.abs(X[:, k])) + np.max(np.abs(B[:, k]))
        eta = max(eta, float(np.max(np.abs(R[:, k])) / den) if den > 0 else 0.0)
    return eta


def rel_frobenius(Lx, Lref, mask=None) -> float:
    """||L - L_ref||_F / ||L_ref||_F over the lower parts of the panels."""
    a = np.asarray(Lx, dtype=np.float64); b = np.asarray(Lref, dtype=np.float64)
    if mask is not None:
        a = a[mask]; b = b[mask]
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def supernode_rel_errors(Lx, Lref, lptr, mask=None) -> np.ndarray:
    """Per supernode s: ||L_s - L_ref,s||_F / ||L_ref,s||_F over the entries
    lptr[s]..lptr[s+1]-1 of the panel storage (the lower parts where mask is
    given); a supernode whose reference is all zero gets ||L_s||_F.  So that
    an error confined to one small supernode cannot hide under the norm of
    the whole factor."""
    a = np.asarray(Lx, dtype=np.float64); b = np.asarray(Lref, dtype=np.float64)
    lptr = np.asarray(lptr, dtype=np.int64)
    d2 = (a - b) ** 2
    r2 = b ** 2
    if mask is not None:
        d2 = np.where(mask, d2, 0.0); r2 = np.where(mask, r2, 0.0)
    ns = lptr.size - 1
    num = np.zeros(ns); den = np.zeros(ns)
    nonempty = lptr[1:] > lptr[:-1]
    starts = lptr[:-1][nonempty]
    if starts.size:
        num[nonempty] = np.add.reduceat(d2, starts)[: starts.size]
        den[nonempty] = np.add.reduceat(r2, starts)[: starts.size]
    num = np.sqrt(num); den = np.sqrt(den)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)

