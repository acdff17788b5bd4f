"""Library analyze phase vs the oracle, bit for bit (host only, no GPU).

The library finds the elimination tree by Liu's algorithm and the column
counts / row lists by row-subtree traversal; the oracle uses the column-merge
recurrence.  Both apply the same ordering, postorder and amalgamation rules,
so every exported array must agree exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import workloads as W

from paper_2202_09288_amd import spchol  # noqa: E402  (conftest builds it when missing)

NAMES = ("perm", "parent", "colcount", "super_ptr", "sparent", "rptr", "rows", "lptr", "level", "uptr", "ulist")


def compare(colptr, rowidx, perm, z):
    S = oracle.Symbolic(colptr, rowidx, perm, z)
    L = spchol.Symbolic(colptr, rowidx, perm, z)
    for name in NAMES:
        a = L.export(name)
        b = S.get(name)
        assert a.dtype == b.dtype, name
        assert np.array_equal(a, b), name
    assert L.info["flops"] == S.sizes["flops"]
    assert L.info["nnz_l"] == S.sizes["nnzL"]
    assert L.info["nsuper"] == S.nsuper
    assert L.info["levels"] == S.sizes["nlevels"]
    assert L.info["panel_entries"] == S.sizes["panel_entries"]
    assert L.info["updates_total"] == S.sizes["updates_total"]
    return S, L


def small_cases():
    for n, dens, seed in [(1, 0.5, 0), (2, 1.0, 1), (9, 0.3, 2), (30, 0.1, 3), (64, 0.05, 4),
                          (100, 0.03, 5), (50, 0.0, 6)]:
        c, r, v = W.random_spd_pattern(n, dens, seed)
        yield f"rand{n}_{seed}", c, r, np.random.default_rng(seed).permutation(n).astype(np.int32)
    for dims in [(1, 1), (2, 3), (7, 7), (16, 9), (3, 3, 3), (6, 5, 4), (10, 10, 10)]:
        s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
        yield s.name, s.colptr, s.rowidx, s.perm
    s = W.elasticity27((4, 3, 5), 77, 0, kappa=1e8, nrhs=1, power_iters=5)
    yield s.name, s.colptr, s.rowidx, s.perm


CASES = list(small_cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("z", [-1.0, 0.0, 0.05, 0.5])
def test_small(case, z):
    _, c, r, p = case
    compare(c, r, p, z)


def test_identity_perm_is_null_perm():
    s = W.laplacian((9, 8), "5pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    a = spchol.Symbolic(s.colptr, s.rowidx, None, 0.05)
    b = spchol.Symbolic(s.colptr, s.rowidx, np.arange(s.n, dtype=np.int32), 0.05)
    for name in NAMES:
        assert np.array_equal(a.export(name), b.export(name))


def test_grid2d_64():
    s = W.grid2d_unit()
    compare(s.colptr, s.rowidx, s.perm, 0.05)


def test_batch_members():
    specs = W.batch_specs(512, 0)
    picks = [i for i, (k, side) in enumerate(specs) if side <= (60 if k == "2d" else 14)][:6]
    for i in picks:
        s = W.batch_system(i, *specs[i])
        compare(s.colptr, s.rowidx, s.perm, 0.05)


@pytest.mark.slow
def test_grid3d_60():
    s = W.grid3d_cond()
    S, L = compare(s.colptr, s.rowidx, s.perm, 0.05)
    assert S.sizes["flops"] == 279230799993


@pytest.mark.parametrize("dims,expect_tiny", [((8, 8), False), ((30, 30, 30), True), ((150, 150), True)])
def test_solve_schedule_split(dims, expect_tiny):
    """The solve schedule: levels with few tasks at the top run persistently;
    below them, tiny supernodes (w <= 8, m <= 64) leave the block-task list
    for the one-wave kernels.  A small grid is persistent throughout; the
    30^3 and 150^2 grids have wide bottom levels full of tiny supernodes."""
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    L = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    info = L.info
    w = np.diff(L.export("super_ptr"))
    m = np.diff(L.export("rptr"))
    tiny = int(((w <= 8) & (m <= 64)).sum())
    assert 1 <= info["solve_persistent_levels"] <= info["solve_levels"]
    assert info["solve_tiny_tasks"] <= tiny
    # every column block keeps at least one block task unless it went to the
    # one-wave list: blocks = sum over supernodes of ceil(w / 64)
    blocks = int(((w + 63) // 64).sum())
    assert info["solve_block_tasks"] + info["solve_tiny_tasks"] >= blocks
    if expect_tiny:
        assert info["solve_persistent_levels"] < info["solve_levels"]
        assert info["solve_tiny_tasks"] > tiny // 2
    else:
        assert info["solve_persistent_levels"] == info["solve_levels"] and info["solve_tiny_tasks"] == 0
