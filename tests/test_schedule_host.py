"""Host checks of the device schedule (spc_symbolic_verify, no device): every
64-column block of the blocked path gets the rows below its diagonal solved
exactly once, by a TRSM launch or by the tiles of the step before that take
its TRSM inside the trailing launch; every tile that waits inside a launch
sits after its block's diagonal tile and carries the task that tile runs
(it runs it itself when it claims the block's factorization).  The schedule
is the one the GPU parity tests run."""
import numpy as np
import pytest

from paper_2202_09288_amd import workloads as W

from paper_2202_09288_amd import spchol  # noqa: E402  (conftest builds it when missing)

TUNINGS = [None, {"handover": -1}, {"tiny_w": -1, "small_w": -1}, {"big_min": 1, "big_min_k": 1},
           {"tiny_w": 4, "tiny_m": 32, "small_w": 16, "small_m": 64}, {"delay": 2}, {"delay": 3},
           {"delay": 4, "handover": -1}, {"persist": 1}, {"persist": 1, "tiny_w": 4, "tiny_m": 32},
           {"group": -1}, {"persist": 1, "group": -1}, {"handover": 2}, {"delay": 3, "handover": 2},
           {"delay": 3, "bulk128": 1}, {"delay": 2, "bulk128": 1, "handover": 2},
           {"delay": 3, "lookahead": 1}, {"delay": 4, "lookahead": 1, "handover": 2}]


@pytest.mark.parametrize("dims", [(20, 20, 20), (30, 24, 28), (37, 23), (200, 150), (12, 9, 11)])
@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "defaults" if t is None else ",".join(t))
def test_schedule_invariants_grids(dims, tuning):
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    for z in (0.05, -1.0, 0.5):
        spchol.Symbolic(s.colptr, s.rowidx, s.perm, z, tuning).verify()


@pytest.mark.parametrize("n", [64, 65, 130, 203, 320])
def test_schedule_invariants_dense(n):
    """One supernode: every block of the root hands over to tiles that all
    share one residue, the case with the most no-op entries."""
    r, c = np.tril_indices(n)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    colptr, rowidx, v = W.lower_csc(n, r, c, A[r, c])
    perm = np.arange(n, dtype=np.int32)
    for tuning in (None, {"handover": -1}, {"tiny_w": -1, "small_w": -1}, {"delay": 2}, {"delay": 4}):
        spchol.Symbolic(colptr, rowidx, perm, 0.05, tuning).verify()


def test_schedule_invariants_headline_grid():
    """The 60^3 grid of the benchmark, as analysed for it."""
    s = W.grid3d_cond()
    spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05).verify()


def test_schedule_invariants_elasticity():
    s = W.elasticity27((6, 5, 7), 88, 0, kappa=1e6, nrhs=1, power_iters=5)
    spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05).verify()


def test_solve_handovers_counted():
    """Consecutive column blocks of a supernode hand over directly only in
    the persistent solve sweeps: one dense supernode of 10 blocks has 9
    hand-overs when every solve level is persistent and none when none is."""
    n = 611
    r, c = np.tril_indices(n)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    colptr, rowidx, v = W.lower_csc(n, r, c, A[r, c])
    perm = np.arange(n, dtype=np.int32)
    every = spchol.Symbolic(colptr, rowidx, perm, 0.05, {"solve_persist_max": 1 << 30})
    every.verify()
    assert every.info["nsuper"] == 1 and every.info["solve_handovers"] == 9
    assert spchol.Symbolic(colptr, rowidx, perm, 0.05, {"solve_persist_max": -1}).info["solve_handovers"] == 0
