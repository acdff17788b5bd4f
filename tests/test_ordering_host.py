"""Fill-reducing orderings without coordinates (spc_order) on the host:
valid permutations on every kind of pattern, minimum degree on graphs
worked by hand, the nested-dissection separator of a path, and the fill of
both against the natural order and the coordinate nested dissection of the
grid workloads (R1).  Parity of factor and solve under these orders is in
the GPU tests (the solution does not depend on the order)."""
import numpy as np
import pytest

from paper_2202_09288_amd import spchol
from paper_2202_09288_amd import workloads as W


def graph_csc(n, edges):
    r = np.array([max(a, b) for a, b in edges] + list(range(n)), dtype=np.int64)
    c = np.array([min(a, b) for a, b in edges] + list(range(n)), dtype=np.int64)
    v = np.where(r == c, 4.0, -1.0)
    colptr, rowidx, _ = W.lower_csc(n, r, c, v)
    return colptr, rowidx


def test_minimum_degree_hand_values():
    """A star with its hub at 0 and leaves 1-5: the leaves (degree 1) go in
    index order while the hub's degree exceeds 1; once only leaf 5 is left
    the hub has degree 1 too, and the tie goes to the lower index, 0.  A path: the end 0 (degree 1, lowest index),
    then 1, which becomes an end, and so on.  A 5-cycle: all of degree 2,
    so 0 first; its neighbours 1 and 4 then join, every degree is 2 again,
    and the lowest index goes next each time."""
    cp, ri = graph_csc(6, [(0, k) for k in range(1, 6)])
    assert spchol.order(cp, ri, "md").tolist() == [1, 2, 3, 4, 0, 5]
    cp, ri = graph_csc(5, [(k, k + 1) for k in range(4)])
    assert spchol.order(cp, ri, "md").tolist() == [0, 1, 2, 3, 4]
    cp, ri = graph_csc(5, [(k, (k + 1) % 5) for k in range(5)])
    assert spchol.order(cp, ri, "md").tolist() == [0, 1, 2, 3, 4]


def test_nested_dissection_path_separator():
    """A path of 200 vertices: the level structure from its end 0 has one
    vertex per level; the first level leaving a third of the path on each
    side is level 67, so vertex 67 is the top separator, ordered last."""
    n = 200
    cp, ri = graph_csc(n, [(k, k + 1) for k in range(n - 1)])
    p = spchol.order(cp, ri, "nd")
    assert p[-1] == 67
    assert sorted(p.tolist()) == list(range(n))


@pytest.mark.parametrize("method", ["natural", "nd", "md"])
def test_orders_are_permutations(method):
    cases = [graph_csc(1, []), graph_csc(7, []),  # isolated vertices
             graph_csc(9, [(0, 1), (1, 2), (5, 6), (6, 7), (7, 8)])]  # disconnected
    for n, dens, seed in [(40, 0.1, 1), (150, 0.02, 2)]:
        cp, ri, _ = W.random_spd_pattern(n, dens, seed)
        cases.append((cp, ri))
    s = W.laplacian((17, 13, 11), "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    cases.append((s.colptr, s.rowidx))
    for cp, ri in cases:
        n = cp.size - 1
        p = spchol.order(cp, ri, method)
        assert sorted(p.tolist()) == list(range(n))
        if method == "natural":
            assert p.tolist() == list(range(n))


def test_order_errors_and_empty():
    assert spchol.order(np.zeros(1, np.int64), np.zeros(0, np.int32), "nd").size == 0
    cp, ri = graph_csc(4, [(0, 1)])
    bad = ri.copy()
    bad[1] = 9  # row out of range
    with pytest.raises(spchol.SpcError):
        spchol.order(cp, bad, "nd")
    s = W.laplacian((25, 25, 25), "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    with pytest.raises(spchol.SpcError):  # minimum degree is limited to n <= 10,000
        spchol.order(s.colptr, s.rowidx, "md")


@pytest.mark.parametrize("dims", [(64, 64), (30, 30, 30)])
def test_fill_against_natural_and_coordinate_nd(dims):
    """Graph nested dissection fills far less than the natural order and no
    more than the coordinate nested dissection of the grid workloads (on
    these grids it measured 0.6-0.8 of its entries of L)."""
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    nnz = {}
    for name, perm in [("coord", s.perm), ("natural", None), ("nd", spchol.order(s.colptr, s.rowidx, "nd"))]:
        nnz[name] = spchol.Symbolic(s.colptr, s.rowidx, perm, 0.05).info["nnz_l"]
    assert nnz["nd"] <= nnz["coord"]
    assert nnz["nd"] * 2 < nnz["natural"]
    if s.n <= 10000:
        md = spchol.Symbolic(s.colptr, s.rowidx, spchol.order(s.colptr, s.rowidx, "md"), 0.05).info["nnz_l"]
        assert md * 2 < nnz["natural"]


def test_analyze_orders_when_no_perm_given():
    s = W.laplacian((20, 19, 18), "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    a = spchol.Symbolic(s.colptr, s.rowidx, None, 0.05, {"ordering": 1})
    b = spchol.Symbolic(s.colptr, s.rowidx, spchol.order(s.colptr, s.rowidx, "nd"), 0.05)
    assert np.array_equal(a.export("perm"), b.export("perm"))
    assert a.info == b.info
