"""C-ABI contract on the host: the library loads, exports every function the
header declares, validates input and handles, and never needs a device for
the analyze phase."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2202_09288_amd import workloads as W

from paper_2202_09288_amd import spchol  # noqa: E402  (conftest builds it when missing)
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "spchol.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spc_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(spchol.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(spchol.EXPORTS)


def analyze_raw(n, colptr, rowidx, perm=None):
    h = ctypes.c_void_p()
    cp = np.ascontiguousarray(colptr, dtype=np.int64)
    ri = np.ascontiguousarray(rowidx, dtype=np.int32)
    pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    rc = spchol._lib.spc_analyze(n, cp.ctypes.data_as(ctypes.c_void_p), ri.ctypes.data_as(ctypes.c_void_p),
                                 None if pp is None else pp.ctypes.data_as(ctypes.c_void_p), None,
                                 ctypes.byref(h))
    if rc == 0:
        spchol._lib.spc_free_symbolic(h)
    return rc


def good():
    # columns: 0 -> rows [0, 1, 3], 1 -> [1], 2 -> [2, 3], 3 -> [3]
    return (np.array([0, 3, 4, 6, 7], np.int64), np.array([0, 1, 3, 1, 2, 3, 3], np.int32),
            np.array([4, -1, -1, 4, 4, -1, 4.0]))


def test_valid_input_ok():
    c, r, _ = good()
    assert analyze_raw(4, c, r) == spchol.OK
    assert analyze_raw(0, np.zeros(1, np.int64), np.zeros(0, np.int32)) == spchol.OK


BAD = {
    "unsorted": ([0, 3, 4, 6, 7], [0, 3, 1, 1, 2, 3, 3]),
    "duplicate": ([0, 3, 4, 6, 7], [0, 1, 1, 1, 2, 3, 3]),
    "upper": ([0, 3, 4, 7, 8], [0, 1, 3, 1, 1, 2, 3, 3]),
    "out_of_range": ([0, 3, 4, 6, 7], [0, 1, 9, 1, 2, 3, 3]),
    "no_diag": ([0, 3, 3, 5, 6], [0, 1, 3, 2, 3, 3]),
    "bad_colptr": ([1, 3, 4, 6, 7], [0, 1, 3, 1, 2, 3, 3]),
    "decreasing_colptr": ([0, 3, 2, 6, 7], [0, 1, 3, 1, 2, 3, 3]),
}


@pytest.mark.parametrize("mutate", sorted(BAD) + ["negative_n"])
def test_malformed_csc(mutate):
    if mutate == "negative_n":
        c, r, _ = good()
        assert analyze_raw(-1, c, r) == spchol.INVALID_INPUT
        return
    c, r = BAD[mutate]
    assert analyze_raw(4, np.array(c), np.array(r)) == spchol.INVALID_INPUT


@pytest.mark.parametrize("perm", [[0, 1, 2, 2], [0, 1, 2, 4], [-1, 0, 1, 2]])
def test_bad_permutation(perm):
    c, r, _ = good()
    assert analyze_raw(4, c, r, perm) == spchol.INVALID_INPUT


def test_null_handles_and_double_free():
    lib = spchol._lib
    info = spchol._Info()
    assert lib.spc_symbolic_info(None, ctypes.byref(info)) == spchol.BAD_HANDLE
    assert lib.spc_sync(None, None) == spchol.BAD_HANDLE
    assert lib.spc_solve(None, None, 1, 1, None) == spchol.BAD_HANDLE
    assert lib.spc_refactorize(None, None, None) == spchol.BAD_HANDLE
    assert lib.spc_factor_export(None, None) == spchol.BAD_HANDLE
    assert lib.spc_factorize(None, None, 0, None, None) == spchol.INVALID_INPUT
    out = ctypes.c_void_p()
    assert lib.spc_factorize(None, None, 0, None, ctypes.byref(out)) == spchol.BAD_HANDLE
    lib.spc_free_symbolic(None)
    lib.spc_free_factor(None)
    assert lib.spc_analyze(4, None, None, None, None, None) == spchol.INVALID_INPUT


def test_status_strings():
    for st in range(-7, 1):
        assert spchol._lib.spc_status_string(st)
    assert b"positive definite" in spchol._lib.spc_status_string(spchol.NOT_SPD)


def test_info_and_export():
    s = W.laplacian((12, 10), "5pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    S = spchol.Symbolic(s.colptr, s.rowidx, s.perm)
    i = S.info
    assert i["n"] == s.n and i["nnz_a"] == s.nnz
    assert i["panel_entries"] == int(S.export("lptr")[-1])
    assert i["factor_bytes_fp64"] > 8 * i["panel_entries"]
    assert i["factor_bytes_fp32"] > 4 * i["panel_entries"]
    with pytest.raises(KeyError):
        S.export("nope")
    assert spchol._lib.spc_symbolic_export(S.handle, 99, ctypes.c_void_p(1)) == spchol.INVALID_INPUT


@pytest.mark.parametrize("field,value", [("tiny_w", 9), ("tiny_m", 65), ("small_w", 33), ("small_m", 129),
                                         ("handover", 3), ("group", 2), ("bulk128", 2), ("lookahead", 2)])
def test_cutoffs_beyond_kernel_limits_rejected(field, value):
    s = W.laplacian((6, 5), "5pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    with pytest.raises(spchol.SpcError) as e:
        spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {field: value})
    assert e.value.status == spchol.INVALID_INPUT


def test_nan_amalgamation_threshold_rejected():
    s = W.laplacian((6, 5), "5pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    with pytest.raises(spchol.SpcError) as e:
        spchol.Symbolic(s.colptr, s.rowidx, s.perm, float("nan"))
    assert e.value.status == spchol.INVALID_INPUT


def test_binding_checks_host_array_sizes():
    """The binding refuses host arrays shorter than the pattern says (the
    library reads colptr[n] row indices and n permutation entries)."""
    s = W.laplacian((6, 5), "5pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    with pytest.raises(ValueError):
        spchol.Symbolic(s.colptr, s.rowidx[:-1], s.perm)
    with pytest.raises(ValueError):
        spchol.Symbolic(s.colptr, s.rowidx, s.perm[:-1])
    with pytest.raises(ValueError):
        spchol.Symbolic(np.zeros(0, dtype=np.int64), s.rowidx)


def test_cutoffs_shape_the_schedule():
    """Schedule cut-offs from the analysis options: turning the one-wave
    path off empties the one-wave solve list; no persistent levels when the
    threshold is off, all of them when it is huge; an unknown name is
    refused by the binding.  The structure of L does not depend on them."""
    s = W.laplacian((30, 30, 30), "7pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    base = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    no_tiny = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"tiny_w": -1})
    assert base.info["solve_tiny_tasks"] > 0 and no_tiny.info["solve_tiny_tasks"] == 0
    none = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"solve_persist_max": -1})
    assert none.info["solve_persistent_levels"] == 0
    allp = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"solve_persist_max": 1 << 30})
    assert allp.info["solve_persistent_levels"] == allp.info["solve_levels"]
    for other in (no_tiny, none, allp):
        for name in ("super_ptr", "rows", "lptr"):
            assert np.array_equal(other.export(name), base.export(name))
    with pytest.raises(ValueError):
        spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"tile": 3})


def test_hbm_budget_refuses_before_the_device():
    """A factorization over the analysis's device budget is refused with
    SPC_OUT_OF_MEMORY before any allocation (no device needed), with both
    sizes in the error message; a budget at the footprint is not refused by
    the budget check."""
    s = W.laplacian((6, 5, 4), "7pt", 1, 0, unit=False, shift=1e-2, nrhs=1)
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, hbm_budget=1000)
    need = {1: sym.info["factor_bytes_fp32"], 0: sym.info["factor_bytes_fp64"]}
    assert need[1] > 1000 and need[0] > need[1]
    dummy = ctypes.c_void_p(16)  # never dereferenced: the budget check comes first
    for prec in (spchol.FP64, spchol.FP32, spchol.FP32_BF16UPD):
        h = ctypes.c_void_p()
        rc = spchol._lib.spc_factorize(sym.handle, dummy, prec, None, ctypes.byref(h))
        assert rc == spchol.OUT_OF_MEMORY and not h.value
        msg = spchol._lib.spc_last_error_message().decode()
        assert str(need[0 if prec == 0 else 1]) in msg and "1000" in msg
    # at the FP32 footprint: FP32 passes the budget check, FP64 does not
    sym2 = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, hbm_budget=need[1])
    h = ctypes.c_void_p()
    assert spchol._lib.spc_factorize(sym2.handle, dummy, spchol.FP64, None,
                                     ctypes.byref(h)) == spchol.OUT_OF_MEMORY
