"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check below is independent of the oracle's own code: a brute-force
elimination game, dense LAPACK Cholesky, closed forms, invariants of
elimination trees, and the worked example of Sec. 3, Fig. 1.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import workloads as W
from tests.bruteforce import dense_lower, elimination_game, permuted_dense

HERE = os.path.dirname(os.path.abspath(__file__))


def lower_from_dense_pattern(P, values=None):
    n = P.shape[0]
    r, c = np.nonzero(np.tril(P))
    v = values[r, c] if values is not None else np.ones(r.size)
    return W.lower_csc(n, r, c, v)


def random_cases():
    for n, dens, seed in [(1, 0.5, 0), (2, 1.0, 1), (7, 0.3, 2), (16, 0.15, 3), (33, 0.08, 4),
                          (48, 0.05, 5), (64, 0.04, 6), (64, 0.2, 7), (40, 0.0, 8)]:
        colptr, rowidx, values = W.random_spd_pattern(n, dens, seed)
        perm = np.arange(n, dtype=np.int32)[::-1].copy() if seed % 2 else np.arange(n, dtype=np.int32)
        yield f"rand{n}_{seed}", n, colptr, rowidx, values, perm
    for dims in [(3, 3), (5, 4), (8, 8), (4, 4, 4), (5, 3, 6), (8, 8, 8)]:
        s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
        yield s.name, s.n, s.colptr, s.rowidx, s.values, s.perm


CASES = list(random_cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("z", [-1.0, 0.0, 0.05, 0.3])
def test_structure_vs_elimination_game(case, z):
    _, n, colptr, rowidx, values, perm = case
    S = oracle.Symbolic(colptr, rowidx, perm, z)
    G = permuted_dense(n, colptr, rowidx, np.ones(colptr[-1]), S.perm) != 0
    parent, cols = elimination_game(G)
    assert np.array_equal(S.parent, parent)
    assert np.array_equal(S.colcount, np.array([c.size + 1 for c in cols]))
    Lp, Li = S.Lp, S.Li
    for j in range(n):
        assert np.array_equal(Li[Lp[j]:Lp[j + 1]], cols[j])
    assert S.sizes["nnzL"] == sum(c.size + 1 for c in cols)
    assert S.sizes["flops"] == sum((c.size + 1) ** 2 for c in cols)
    # final order is a permutation; parent(j) > j; subtrees are contiguous
    assert np.array_equal(np.sort(S.perm), np.arange(n))
    assert np.all((parent == -1) | (parent > np.arange(n)))
    size = np.ones(n, dtype=int)
    for j in range(n):
        if parent[j] != -1:
            size[parent[j]] += size[j]
    for j in range(n):
        lo = j - size[j] + 1
        for k in range(lo, j):
            a = k
            while a != -1 and a < j:
                a = parent[a]
            assert a == j, "postorder: subtree of j must be [j-size+1, j]"


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("z", [-1.0, 0.0, 0.05, 0.3])
def test_supernode_invariants(case, z):
    _, n, colptr, rowidx, values, perm = case
    S = oracle.Symbolic(colptr, rowidx, perm, z)
    sp, rp, rows, par = S.super_ptr, S.rptr, S.rows, S.parent
    cc = S.colcount
    Lp, Li = S.Lp, S.Li
    snode = np.repeat(np.arange(S.nsuper), np.diff(sp))
    fp = S.fund_ptr
    # fundamental supernodes: columns j, j+1 together iff the textbook rule
    for j in range(n - 1):
        together = snode_of(fp, j) == snode_of(fp, j + 1)
        rule = par[j] == j + 1 and np.sum(par == j + 1) == 1 and cc[j] == cc[j + 1] + 1
        assert together == rule
    # every final supernode is a union of consecutive fundamental ones
    assert set(sp.tolist()) <= set(fp.tolist())
    zeros_total = 0
    for s in range(S.nsuper):
        R = rows[rp[s]:rp[s + 1]]
        f, l = sp[s], sp[s + 1] - 1
        w, m = l - f + 1, R.size
        assert np.all(np.diff(R) > 0)
        assert np.array_equal(R[:w], np.arange(f, l + 1))
        stored = 0
        exact = 0
        for j in range(f, l + 1):
            col = Li[Lp[j]:Lp[j + 1]]
            assert np.all(np.isin(col, R)), "pattern of L inside R_s"
            stored += m - (j - f)
            exact += col.size + 1
        zeros_total += stored - exact
        assert float(stored - exact) <= max(z, 0.0) * float(stored)
    assert zeros_total == S.sizes["zeros"]
    # U_s is the set of d < s with R_d meeting cols(s); R_d below f_s inside R_s
    U = {s: S.ulist[S.uptr[s]:S.uptr[s + 1]] for s in range(S.nsuper)}
    for s in range(S.nsuper):
        f, l = sp[s], sp[s + 1] - 1
        want = [d for d in range(s) if np.any((rows[rp[d]:rp[d + 1]] >= f) & (rows[rp[d]:rp[d + 1]] <= l))]
        assert U[s].tolist() == want
        Rs = set(rows[rp[s]:rp[s + 1]].tolist())
        for d in want:
            Rd = rows[rp[d]:rp[d + 1]]
            assert set(Rd[Rd >= f].tolist()) <= Rs
    # levels: 0 at leaves, else 1 + max over children
    sparent = S.sparent
    lev = np.zeros(S.nsuper, dtype=int)
    for s in range(S.nsuper):
        if sparent[s] != -1:
            lev[sparent[s]] = max(lev[sparent[s]], lev[s] + 1)
            assert sparent[s] == snode[par[sp[s + 1] - 1]]
    assert np.array_equal(S.level, lev)


def snode_of(ptr, j):
    return int(np.searchsorted(ptr, j, side="right") - 1)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_factor_vs_dense_cholesky(case):
    _, n, colptr, rowidx, values, perm = case
    S = oracle.Symbolic(colptr, rowidx, perm, 0.05)
    Lx = S.factor(values)
    Ah = permuted_dense(n, colptr, rowidx, values, S.perm)
    Lref = np.linalg.cholesky(Ah)
    L = S.to_dense_L(Lx)
    assert np.linalg.norm(L - Lref) <= 1e-13 * np.linalg.norm(Lref)
    assert np.linalg.norm(Ah - L @ L.T) <= 4 * n * 2.2e-16 * np.linalg.norm(Ah)
    # explicit zeros of amalgamated supernodes stay exactly zero
    mask = S.lower_mask()
    stored = np.zeros((n, n), dtype=bool)
    for s in range(S.nsuper):
        R = S.rows[S.rptr[s]:S.rptr[s + 1]]
        for c in range(S.super_ptr[s + 1] - S.super_ptr[s]):
            stored[R[c:], S.super_ptr[s] + c] = True
    exact = np.zeros((n, n), dtype=bool)
    for j in range(n):
        exact[j, j] = True
        exact[S.Li[S.Lp[j]:S.Lp[j + 1]], j] = True
    assert np.all(L[stored & ~exact] == 0.0)
    assert mask.sum() == S.sizes["panel_entries"] - sum(
        (w * (w - 1)) // 2 for w in np.diff(S.super_ptr))


def test_scaling_gives_sqrt_alpha():
    s = W.laplacian((6, 5), "5pt", 77, 3, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    L1 = S.factor(s.values)
    L4 = S.factor(4.0 * s.values)
    assert np.array_equal(L4, 2.0 * L1)  # scaling by 4 is exact in binary


def test_closed_form_diagonal():
    n = 9
    colptr, rowidx, values = W.lower_csc(n, np.arange(n), np.arange(n), np.arange(1, n + 1, dtype=float))
    S = oracle.Symbolic(colptr, rowidx, np.arange(n, dtype=np.int32), 0.05)
    assert np.all(S.parent == -1)
    assert np.all(S.colcount == 1)
    assert S.nsuper == n and S.sizes["nlevels"] == 1
    Lx = S.factor(values)
    assert np.allclose(np.sort(Lx), np.sqrt(np.arange(1, n + 1)), rtol=0, atol=1e-15)


def test_closed_form_tridiagonal():
    n = 12
    r = np.concatenate([np.arange(n), np.arange(1, n)])
    c = np.concatenate([np.arange(n), np.arange(n - 1)])
    v = np.concatenate([np.full(n, 2.0), np.full(n - 1, -1.0)])
    colptr, rowidx, values = W.lower_csc(n, r, c, v)
    S = oracle.Symbolic(colptr, rowidx, np.arange(n, dtype=np.int32), 0.05)
    assert np.array_equal(S.parent, np.append(np.arange(1, n), -1))
    assert np.array_equal(S.colcount, np.append(np.full(n - 1, 2), 1))
    assert S.sizes["nfund"] == n - 1
    L = S.to_dense_L(S.factor(values))
    j = np.arange(n)
    assert np.allclose(np.diag(L), np.sqrt((j + 2) / (j + 1)), rtol=1e-15, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt((j[:-1] + 1) / (j[:-1] + 2)), rtol=1e-15, atol=0)


def test_closed_form_dense():
    n = 20
    rng = np.random.default_rng(0)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    colptr, rowidx, values = lower_from_dense_pattern(np.ones((n, n), bool), A)
    S = oracle.Symbolic(colptr, rowidx, np.arange(n, dtype=np.int32), 0.05)
    assert S.nsuper == 1
    assert np.array_equal(S.colcount, n - np.arange(n))
    assert S.sizes["flops"] == n * (n + 1) * (2 * n + 1) // 6
    L = S.to_dense_L(S.factor(values))
    assert np.allclose(L, np.linalg.cholesky(A), rtol=0, atol=1e-13 * np.abs(A).max())


def test_closed_form_arrow():
    n = 10
    r = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
    c = np.concatenate([np.arange(n), np.arange(n - 1)])
    v = np.concatenate([np.full(n, float(n)), np.full(n - 1, -1.0)])
    colptr, rowidx, values = W.lower_csc(n, r, c, v)
    S = oracle.Symbolic(colptr, rowidx, np.arange(n, dtype=np.int32), 0.0)
    assert np.array_equal(S.parent, np.append(np.full(n - 1, n - 1), -1))  # a star
    assert np.array_equal(S.colcount, np.append(np.full(n - 1, 2), 1))
    assert S.sizes["nlevels"] == 2


@pytest.mark.parametrize("k", [3, 4, 5, 7, 9])
def test_closed_form_lexicographic_grid(k):
    """k x k 5-point grid in lexicographic order fills its band."""
    s = W.laplacian((k, k), "5pt", 77, 0, unit=True, shift=1e-2, nrhs=1)
    n = k * k
    S = oracle.Symbolic(s.colptr, s.rowidx, np.arange(n, dtype=np.int32), 0.0)
    j = np.arange(n)
    want = np.where(j <= k - 2, j + 3, np.minimum(k, n - 1 - j) + 1)
    assert np.array_equal(S.colcount, want)


def test_fig1_schedule_golden():
    """Levels reproduce the schedule printed for Fig. 1 (Sec. 3)."""
    txt = open(os.path.join(HERE, "golden", "fig1_tree.txt")).read().splitlines()
    edges = [tuple(int(x) for x in e.split("->")) for e in
             next(l for l in txt if l.startswith("edges:")).split(":", 1)[1].split()]
    sched = [set(int(x) for x in g.split()) for g in
             next(l for l in txt if l.startswith("schedule:")).split(":", 1)[1].split("|")]
    n = 6
    r = [p - 1 for (_, p) in edges]; c = [ch - 1 for (ch, _) in edges]
    colptr, rowidx, values = W.lower_csc(n, np.concatenate([np.arange(n), r]),
                                         np.concatenate([np.arange(n), c]),
                                         np.concatenate([np.full(n, 4.0), -np.ones(len(r))]))
    # z < 0 turns amalgamation off: the six supernodes of the figure stay apart
    S = oracle.Symbolic(colptr, rowidx, np.arange(n, dtype=np.int32), -1.0)
    assert S.nsuper == n
    groups = {}
    for k in range(n):  # supernode k holds pivot k = original column perm[k]
        groups.setdefault(int(S.level[k]), set()).add(int(S.perm[k]) + 1)
    assert [groups[l] for l in sorted(groups)] == sched


@pytest.mark.parametrize("dims", [(8, 8), (12, 9), (5, 5, 5)])
def test_solve_backward_error_and_manufactured(dims):
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 1, unit=False, shift=1e-2, nrhs=3)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lx = S.factor(s.values)
    X = S.solve(Lx, s.B)
    assert oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X, s.B) < 1e-15
    # manufactured: b = A x* with integer x*
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values)
    xs = np.arange(s.n, dtype=float) % 7 - 3
    x = S.solve(Lx, A @ xs)
    cond = np.linalg.cond(A.toarray())
    assert np.max(np.abs(x - xs)) <= 10 * cond * 2.2e-16 * np.max(np.abs(xs))
    # a different ordering gives the same solution within kappa * u
    S2 = oracle.Symbolic(s.colptr, s.rowidx, np.arange(s.n, dtype=np.int32), 0.0)
    X2 = S2.solve(S2.factor(s.values), s.B)
    assert np.max(np.abs(X2 - X)) <= 10 * cond * 2.2e-16 * np.max(np.abs(X))


def test_not_spd_reports_pivot():
    s = W.laplacian((7, 6), "5pt", 77, 2, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    iperm = np.argsort(S.perm)
    for r in (0, 17, s.n - 1):
        v = s.values.copy()
        diag_pos = s.colptr[r]  # rows sorted, diagonal first in its column
        assert s.rowidx[diag_pos] == r
        v[diag_pos] = -v[diag_pos]
        with pytest.raises(oracle.NotSPD) as e:
            S.factor(v)
        assert e.value.column == iperm[r]
    v = s.values.copy(); v[s.colptr[5]] = np.nan
    with pytest.raises(oracle.NotSPD) as e:
        S.factor(v)
    assert e.value.column == iperm[5]


def test_workload_sizes_2d64():
    """The 64x64 5-point workload: n = 4096, 20,224 stored entries in full."""
    s = W.grid2d_unit()
    assert s.n == 4096 and 2 * s.nnz - s.n == 20224
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values)
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    assert np.allclose(d - off, 1e-2, rtol=0, atol=1e-12)


def test_subtree_factor_matches_full():
    s = W.laplacian((9, 9, 9), "7pt", 77, 4, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lx = S.factor(s.values)
    for lev in (1, 3):
        root = int(np.nonzero(S.level == lev)[0][-1])
        Ls, first = S.factor_subtree(s.values, root)
        sl = slice(S.lptr[first], S.lptr[root + 1])
        assert np.array_equal(Ls[sl], Lx[sl])
        anc = root
        for k in range(first, root + 1):  # every supernode in range descends from root
            a = k
            while a != -1 and a < root:
                a = S.sparent[a]
            assert a == root


def test_backward_error_hand_values():
    """Normwise backward error in the infinity norm on cases worked by hand:
    A = [2], b = [3], x = [1]: |3 - 2| / (2 * 1 + 3) = 1/5.  A = [[2, -1],
    [-1, 2]] (||A|| = 3), b = [1, 1]: x = [1, 1] is exact (0); x = [1, 0]
    leaves r = [-1, 2], so 2 / (3 * 1 + 1) = 1/2.  Several right-hand sides
    take the largest."""
    one = (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.0]))
    assert oracle.backward_error(1, *one, np.array([1.0]), np.array([3.0])) == pytest.approx(0.2, abs=1e-16)
    cp, ri, v = np.array([0, 2, 3], np.int64), np.array([0, 1, 1], np.int32), np.array([2.0, -1.0, 2.0])
    b = np.array([1.0, 1.0])
    assert oracle.backward_error(2, cp, ri, v, np.array([1.0, 1.0]), b) == 0.0
    assert oracle.backward_error(2, cp, ri, v, np.array([1.0, 0.0]), b) == pytest.approx(0.5, abs=1e-16)
    X = np.column_stack([[1.0, 1.0], [1.0, 0.0]])
    B = np.column_stack([b, b])
    assert oracle.backward_error(2, cp, ri, v, X, B) == pytest.approx(0.5, abs=1e-16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_error_is_the_smallest_consistent_perturbation(seed):
    """Rigal-Gaches: eta is attained (A + dA) x = b + db with ||dA|| = eta
    ||A|| and ||db|| = eta ||b||, through dA = c r z^T, db = -d r, with z
    picking the largest entry of x; and no consistent perturbation is
    smaller: for (A + E) x = b + f, max(||E||/||A||, ||f||/||b||) >= eta."""
    s = W.laplacian((6, 5), "5pt", 77, seed, unit=False, shift=1e-2, nrhs=1)
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values).toarray()
    b = s.B[:, 0]
    rng = np.random.default_rng(seed)
    x = np.linalg.solve(A, b) * (1.0 + 1e-3 * rng.standard_normal(s.n))
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, x, b)
    nA, nx, nb = np.abs(A).sum(axis=1).max(), np.abs(x).max(), np.abs(b).max()
    r = b - A @ x
    k = int(np.argmax(np.abs(x)))
    z = np.zeros(s.n)
    z[k] = np.sign(x[k])
    den = nA * nx + nb
    dA = (nA / den) * np.outer(r, z)
    db = -(nb / den) * r
    assert np.max(np.abs((A + dA) @ x - (b + db))) <= 1e-13 * nA * nx
    assert np.abs(dA).sum(axis=1).max() == pytest.approx(eta * nA, rel=1e-12)
    assert np.abs(db).max() == pytest.approx(eta * nb, rel=1e-12)
    for _ in range(20):
        E = rng.standard_normal((s.n, s.n)) * 1e-4 * rng.random()
        f = (A + E) @ x - b
        eps = max(np.abs(E).sum(axis=1).max() / nA, np.abs(f).max() / nb)
        assert eps >= eta * (1 - 1e-12)


def test_rel_frobenius_hand_values():
    """relF = ||L - L_ref||_F / ||L_ref||_F over the masked entries, worked
    by hand: L_ref = [3, 4, 0, 12], L = [3, 4, 99, 25] with entry 2 masked
    out leaves the difference [0, 0, 13] against ||[3, 4, 12]|| = 13, so
    relF = 1; without the mask the difference is [0, 0, 99, 13], so relF =
    sqrt(99^2 + 13^2) / 13.  An all-zero reference gives ||L||_F, and
    L = 2 L_ref gives 1."""
    ref = np.array([3.0, 4.0, 0.0, 12.0])
    got = np.array([3.0, 4.0, 99.0, 25.0])
    mask = np.array([True, True, False, True])
    assert oracle.rel_frobenius(got, ref, mask) == 1.0
    assert oracle.rel_frobenius(got, ref) == pytest.approx(np.sqrt(99.0 ** 2 + 13.0 ** 2) / 13.0, rel=1e-15)
    assert oracle.rel_frobenius(np.array([3.0, 4.0]), np.zeros(2)) == 5.0
    assert oracle.rel_frobenius(2 * ref, ref) == 1.0
    assert oracle.rel_frobenius(ref, ref, mask) == 0.0


def test_lower_mask_hand_values():
    """The mask keeps each panel's lower trapezoid and drops the strict upper
    triangle of its diagonal block.  A dense 3x3 matrix is one supernode, a
    3x3 column-major panel: entries (row, col) = (0,1), (0,2), (1,2) are out.
    On a grid the mask holds sum_s (m_s w_s - w_s (w_s - 1) / 2) entries."""
    A = np.array([[4.0, 1.0, 1.0], [1.0, 4.0, 1.0], [1.0, 1.0, 4.0]])
    colptr, rowidx, values = lower_from_dense_pattern(np.ones((3, 3), bool), A)
    S = oracle.Symbolic(colptr, rowidx, np.arange(3, dtype=np.int32), 0.05)
    assert S.nsuper == 1
    assert S.lower_mask().tolist() == [True, True, True, False, True, True, False, False, True]
    s = W.laplacian((7, 6, 5), "7pt", 77, 0, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    w = np.diff(S.super_ptr).astype(np.int64)
    m = np.diff(S.rptr).astype(np.int64)
    assert int(S.lower_mask().sum()) == int(np.sum(m * w - w * (w - 1) // 2))


def test_supernode_rel_errors_hand_values():
    """Per-supernode relative error, by hand: panels [0, 2) and [2, 6) with
    L_ref = [1, 0 | 3, 4, 0, 0] and L = [1, 0 | 3, 4, 0, 5]: supernode 0 is
    exact, supernode 1 differs by 5 against ||[3, 4]|| = 5, so 1.  A
    supernode whose reference is zero reports ||L_s||."""
    lptr = np.array([0, 2, 6])
    ref = np.array([1.0, 0.0, 3.0, 4.0, 0.0, 0.0])
    got = np.array([1.0, 0.0, 3.0, 4.0, 0.0, 5.0])
    assert oracle.supernode_rel_errors(got, ref, lptr).tolist() == [0.0, 1.0]
    mask = np.array([True, True, True, True, True, False])
    assert oracle.supernode_rel_errors(got, ref, lptr, mask).tolist() == [0.0, 0.0]
    assert oracle.supernode_rel_errors(np.array([0.5, 2.0]), np.array([0.0, 2.0]),
                                       np.array([0, 1, 2])).tolist() == [0.5, 0.0]
    # an empty supernode (no entries) reports 0
    assert oracle.supernode_rel_errors(np.array([2.0]), np.array([2.0]), np.array([0, 0, 1])).tolist() == [0.0, 0.0]


def test_supernode_errors_expose_a_local_error():
    """A relative error of 1e-8 planted in one entry of the smallest-norm
    supernode of a grid factor stays below the 1e-10 bar in the global relF
    but shows above it in that supernode's error, which is what the
    per-supernode bar of the GPU tests is for."""
    s = W.laplacian((14, 13, 12), "7pt", 77, 1, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lref = S.factor(s.values)
    mask = S.lower_mask()
    lp = S.lptr
    norms = np.sqrt(np.add.reduceat(np.where(mask, Lref, 0.0) ** 2, lp[:-1]))
    t = int(np.argmin(norms))
    Lbad = Lref.copy()
    Lbad[lp[t]] *= 1.0 + 1e-8  # the diagonal entry of its first column
    assert oracle.rel_frobenius(Lbad, Lref, mask) < 1e-10
    e = oracle.supernode_rel_errors(Lbad, Lref, lp, mask)
    assert e[t] > 1e-9 and np.count_nonzero(e) == 1


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_oracle_is_bit_identical(threads):
    """The multi-threaded mode (whole supernodes per thread, level by level)
    runs each supernode's steps on the same inputs as the sequential loop,
    so its factor equals the sequential one bit for bit."""
    for dims in [(9, 8, 7), (33, 31)]:
        s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 2, unit=False, shift=1e-2, nrhs=1)
        S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        assert np.array_equal(S.factor(s.values), S.factor(s.values, threads=threads))


def test_parallel_oracle_not_spd_same_column():
    """A failing pivot is reported at the column the sequential loop stops
    at, also when a later supernode on another branch fails too."""
    s = W.laplacian((9, 9, 9), "7pt", 77, 3, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    v = s.values.copy()
    # make two diagonal entries negative: permuted columns a < b on different branches
    iperm = np.empty(S.n, dtype=np.int64)
    iperm[S.perm] = np.arange(S.n)
    lev0 = np.nonzero(S.level == 0)[0]
    cols = [int(S.super_ptr[lev0[3]]), int(S.super_ptr[lev0[-2]])]
    for pc in cols:
        j = int(S.perm[pc])
        v[s.colptr[j]] = -1.0  # first entry of column j is its diagonal
    with pytest.raises(oracle.NotSPD) as e1:
        S.factor(v)
    with pytest.raises(oracle.NotSPD) as e2:
        S.factor(v, threads=4)
    assert e1.value.column == e2.value.column == min(cols)


def test_parallel_forest_matches_subtrees():
    """The multi-threaded mode restricted to a forest of subtrees gives the
    panels of each subtree exactly as the full sequential factorization."""
    s = W.laplacian((10, 9, 8), "7pt", 77, 5, unit=False, shift=1e-2, nrhs=1)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lx = S.factor(s.values)
    roots = np.nonzero(S.level == 2)[0]
    Lf = S.factor_forest(s.values, roots, threads=4)
    for r in roots:
        _, first = S.factor_subtree(s.values, int(r))
        sl = slice(S.lptr[first], S.lptr[r + 1])
        assert np.array_equal(Lf[sl], Lx[sl])
