"""GPU parity: the HIP path through the C ABI vs the CPU oracle.

Bars (written here, from the paper's method being exact up to rounding):
  FP64 factor:  ||L - L_ref||_F / ||L_ref||_F <= 1e-10 over the lower parts,
                for the whole factor and for every supernode on its own
                (factor_error), so an error confined to one small supernode
                cannot hide under the norm of the whole factor
  FP64 solve:   max-over-RHS normwise backward error <= 1e-12 (host FP64)
  structure:    bit-exact (covered on the host by test_symbolic_parity)
"""
import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_F_FP64 = 1e-10
BERR_FP64 = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def lib(torch_dev):
    from paper_2202_09288_amd import spchol  # fails loudly if the library is missing
    return spchol


def factor_error(Lg, Lref, S, first=0, last=None):
    """The larger of relF over supernodes first..last (all by default) and
    the largest relF of one of them alone."""
    last = S.nsuper - 1 if last is None else last
    sl = slice(int(S.lptr[first]), int(S.lptr[last + 1]))
    mask = S.lower_mask()[sl]
    glob = oracle.rel_frobenius(Lg[sl], Lref[sl], mask)
    per = oracle.supernode_rel_errors(Lg[sl], Lref[sl], S.lptr[first:last + 2] - S.lptr[first], mask)
    worst = int(np.argmax(per)) if per.size else 0
    print(f"  relF {glob:.3e}, worst supernode {first + worst}: {per[worst] if per.size else 0.0:.3e}", flush=True)
    return max(glob, float(per.max()) if per.size else 0.0)


def run_case(torch, lib, colptr, rowidx, values, perm, B, z=0.05, precision="fp64"):
    """relF: for FP64 factor_error (whole factor and every supernode), for
    FP32 the whole factor's relF."""
    print(f"case n={colptr.size - 1} nnz={colptr[-1]} nrhs={B.shape[1]} z={z} {precision}", flush=True)
    S = oracle.Symbolic(colptr, rowidx, perm, z)
    Lref = S.factor(values)
    sym = lib.Symbolic(colptr, rowidx, perm, z)
    dv = torch.from_numpy(values).cuda()
    F = lib.factorize(sym, dv, precision)
    F.sync()
    Lg = F.export()
    mask = S.lower_mask()
    relF = factor_error(Lg, Lref, S) if precision == "fp64" else oracle.rel_frobenius(Lg, Lref, mask)
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    F.solve(Bt)
    X = Bt.cpu().numpy().T
    eta = oracle.backward_error(S.n, colptr, rowidx, values, X, B)
    return relF, eta, F, S


def grid(dims, seed=0, nrhs=1, shift=1e-2):
    return W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 88, seed, unit=False, shift=shift,
                       nrhs=nrhs)


CASES = [
    ("2d-8x8", lambda: grid((8, 8))),
    ("2d-37x23-ragged", lambda: grid((37, 23), nrhs=3)),
    ("3d-9x7x11", lambda: grid((9, 7, 11), nrhs=2)),
    ("3d-16", lambda: grid((16, 16, 16))),
    ("3d-20-17rhs", lambda: grid((20, 20, 20), nrhs=17)),
    ("2d-64-unit", lambda: W.grid2d_unit()),
    ("elast-5x4x6", lambda: W.elasticity27((5, 4, 6), 88, 0, kappa=1e6, nrhs=4, power_iters=20)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity(torch_dev, lib, name, make):
    s = make()
    relF, eta, _, _ = run_case(torch_dev, lib, s.colptr, s.rowidx, s.values, s.perm, s.B)
    print(f"{name}: relF={relF:.3e} eta={eta:.3e}")
    assert relF <= REL_F_FP64
    assert eta <= BERR_FP64


@pytest.mark.parametrize("dims,nrhs,precision", [((30, 30, 30), 1, "fp64"), ((30, 30, 30), 16, "fp64"),
                                                 ((150, 150), 5, "fp64"), ((30, 30, 30), 16, "fp32"),
                                                 ((150, 150), 1, "fp32")])
def test_solve_wide_levels_one_wave_path(torch_dev, lib, dims, nrhs, precision):
    """Grids whose bottom solve levels hold thousands of tiny supernodes, so
    the one-wave forward/backward kernels carry most of the solve; 16 and 5
    right-hand sides take the MFMA form and its clamped columns."""
    s = grid(dims, seed=9, nrhs=nrhs)
    sym_info = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05).info
    assert sym_info["solve_tiny_tasks"] > 1000
    relF, eta, _, _ = run_case(torch_dev, lib, s.colptr, s.rowidx, s.values, s.perm, s.B, precision=precision)
    print(f"one-wave path {dims} nrhs={nrhs} {precision}: relF={relF:.2e} eta={eta:.2e}")
    if precision == "fp64":
        assert relF <= REL_F_FP64 and eta <= BERR_FP64
    else:
        assert relF <= 1e-4 and eta <= 1e-5


SCHEDULES = {
    "blocked only": {"tiny_w": -1, "small_w": -1},
    "tiny 4x32, small 16x64": {"tiny_w": 4, "tiny_m": 32, "small_w": 16, "small_m": 64},
    "128-tiles everywhere": {"big_min": 1, "big_min_k": 1},
    "no 128-tiles": {"big_min": -1},
    "solve levels only": {"solve_persist_max": -1},
    "no in-launch TRSM hand-over": {"handover": -1},
    "solve all persistent": {"solve_persist_max": 1 << 30},
    "bulk updates every 2 blocks": {"delay": 2},
    "bulk updates every 4 blocks, no hand-over": {"delay": 4, "handover": -1},
    "bulk updates every 3 blocks": {"delay": 3},
    "small subtrees in one persistent launch": {"persist": 1},
    "small subtrees persistent, one-wave path off": {"persist": 1, "tiny_w": -1},
    "hand-over where its waits spread": {"handover": 2},
    "hand-over where its waits spread, bulk every 3 blocks": {"delay": 3, "handover": 2},
    "tiny supernodes one wave each": {"group": -1},
    "bulk every 3 blocks, far columns in the next group's steps": {"delay": 3, "lookahead": 1},
    "bulk every 2 blocks, far columns in the next group's steps, hand-over where it spreads":
        {"delay": 2, "lookahead": 1, "handover": 2},
    "bulk updates every 3 blocks on 128-tiles": {"delay": 3, "bulk128": 1},
    "bulk updates every 2 blocks on 128-tiles, hand-over where it spreads": {"delay": 2, "bulk128": 1, "handover": 2},
    "small subtrees persistent, tiny one wave each": {"persist": 1, "group": -1},
}


@pytest.mark.parametrize("name", list(SCHEDULES))
def test_schedule_cutoffs_same_factor(torch_dev, lib, name):
    """Every choice of the schedule cut-offs (what the autotuner varies)
    gives the oracle's factor and a solve at the FP64 bar, 1 and 16 RHS."""
    torch = torch_dev
    s = grid((22, 21, 20), seed=11, nrhs=16)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, SCHEDULES[name])
    F = lib.factorize(sym, torch.from_numpy(s.values).cuda())
    F.sync()
    relF = factor_error(F.export(), S.factor(s.values), S)
    for q in (1, 16):
        Bt = torch.from_numpy(np.ascontiguousarray(s.B[:, :q].T)).cuda()
        F.solve(Bt)
        eta = oracle.backward_error(S.n, s.colptr, s.rowidx, s.values, Bt.cpu().numpy().T, s.B[:, :q])
        print(f"schedule {name}: relF={relF:.2e} eta({q})={eta:.2e}", flush=True)
        assert eta <= BERR_FP64
    assert relF <= REL_F_FP64


def test_factor_graph_replay_matches_eager(torch_dev, lib):
    """The captured factorization replays like the eager one: several
    replays with eager solves and synchronizations between them; values
    changed in place under the same pointer (the replay reads them); a new
    values pointer (captured again)."""
    torch = torch_dev
    s = grid((20, 19, 18), seed=12, nrhs=2)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    mask = S.lower_mask()
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    Fe = lib.factorize(sym, dv)
    Fe.sync()
    Le = Fe.export()
    Fg = lib.factorize(sym, dv)
    Fg.sync()
    Fg.set_graph(True)
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    for rep in range(6):
        if rep == 3:
            dv.mul_(4.0)  # same pointer, new values: L doubles
        if rep == 5:
            dv = dv.clone()  # new pointer
        Fg.refactorize(dv)
        Fg.sync()
        scale = 1.0 if rep < 3 else 2.0
        relF = oracle.rel_frobenius(Fg.export(), scale * Le, mask)
        X = B.clone()
        Fg.solve(X)  # eager work between replays
        torch.cuda.synchronize()
        eta = oracle.backward_error(S.n, s.colptr, s.rowidx, (scale * scale) * s.values, X.cpu().numpy().T, s.B)
        print(f"graph replay {rep}: relF={relF:.2e} eta={eta:.2e}", flush=True)
        assert relF <= 1e-13 and eta <= BERR_FP64


def test_batch_graph_replay_matches_eager(torch_dev, lib):
    torch = torch_dev
    systems = small_batch(6, seed=4, nrhs=1)
    syms = [lib.Symbolic(x.colptr, x.rowidx, x.perm, 0.05) for x in systems]
    dvs = [torch.from_numpy(x.values).cuda() for x in systems]
    eager = lib.Batch(syms, "fp64")
    eager.factorize(dvs)
    eager.sync()
    ref = [eager.factor(i).export() for i in range(len(systems))]
    g = lib.Batch(syms, "fp64")
    g.set_graph(True)
    for rep in range(3):
        g.factorize(dvs)
        g.sync()
        for i, x in enumerate(systems):
            S = oracle.Symbolic(x.colptr, x.rowidx, x.perm, 0.05)
            assert oracle.rel_frobenius(g.factor(i).export(), ref[i], S.lower_mask()) <= 1e-13
        Bs = [torch.from_numpy(np.ascontiguousarray(x.B.T)).cuda() for x in systems]
        g.solve(Bs)  # eager work between replays


@pytest.mark.parametrize("z", [-1.0, 0.0, 0.5])
def test_fp64_amalgamation_settings(torch_dev, lib, z):
    s = grid((14, 13, 12), seed=3, nrhs=2)
    relF, eta, _, _ = run_case(torch_dev, lib, s.colptr, s.rowidx, s.values, s.perm, s.B, z=z)
    assert relF <= REL_F_FP64 and eta <= BERR_FP64


def test_dense_wide_supernode(torch_dev, lib):
    """One supernode wider than several panel blocks, with a ragged edge."""
    n = 203
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    r, c = np.tril_indices(n)
    colptr, rowidx, values = W.lower_csc(n, r, c, A[r, c])
    B = rng.standard_normal((n, 2))
    relF, eta, _, S = run_case(torch_dev, lib, colptr, rowidx, values, np.arange(n, dtype=np.int32), B)
    assert S.nsuper == 1
    assert relF <= REL_F_FP64 and eta <= BERR_FP64


def test_arrow_and_diagonal(torch_dev, lib):
    n = 300  # star etree: many leaves updating one root
    r = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
    c = np.concatenate([np.arange(n), np.arange(n - 1)])
    v = np.concatenate([np.full(n, float(n)), -np.linspace(0.1, 1.0, n - 1)])
    colptr, rowidx, values = W.lower_csc(n, r, c, v)
    B = np.linspace(-1, 1, n)[:, None]
    relF, eta, _, _ = run_case(torch_dev, lib, colptr, rowidx, values, np.arange(n, dtype=np.int32), B)
    assert relF <= REL_F_FP64 and eta <= BERR_FP64
    colptr, rowidx, values = W.lower_csc(5, np.arange(5), np.arange(5), np.arange(1.0, 6.0))
    relF, eta, _, _ = run_case(torch_dev, lib, colptr, rowidx, values, np.arange(5, dtype=np.int32),
                               np.ones((5, 1)))
    assert relF <= REL_F_FP64 and eta <= BERR_FP64


def test_single_unknown(torch_dev, lib):
    colptr, rowidx, values = W.lower_csc(1, [0], [0], [4.0])
    relF, eta, _, _ = run_case(torch_dev, lib, colptr, rowidx, values, np.zeros(1, np.int32),
                               np.array([[2.0]]))
    assert relF <= REL_F_FP64 and eta <= BERR_FP64


def test_not_spd_pivot(torch_dev, lib):
    s = grid((11, 9, 7), seed=2)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    iperm = np.argsort(S.perm)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    for r in (3, s.n // 2, s.n - 1):
        v = s.values.copy()
        v[s.colptr[r]] = -v[s.colptr[r]]
        with pytest.raises(oracle.NotSPD) as eo:
            S.factor(v)
        F = lib.factorize(sym, torch_dev.from_numpy(v).cuda())
        with pytest.raises(lib.NotSPD) as eg:
            F.sync()
        assert eg.value.column == eo.value.column == iperm[r]
    v = s.values.copy()
    v[s.colptr[7]] = np.nan
    F = lib.factorize(sym, torch_dev.from_numpy(v).cuda())
    with pytest.raises(lib.NotSPD) as eg:
        F.sync()
    assert eg.value.column == iperm[7]


def test_not_spd_pivot_in_handed_over_block(torch_dev, lib):
    """A failing pivot inside a 64-column block that a trailing launch
    factors while handing its panels to the tiles below (blocks 1.. of a wide
    supernode): the status names the oracle's column, the tiles below do not
    wait in vain, and the same factor object factors good values again."""
    torch = torch_dev
    n = 300
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    r, c = np.tril_indices(n)
    colptr, rowidx, v0 = W.lower_csc(n, r, c, A[r, c])
    perm = np.arange(n, dtype=np.int32)
    S = oracle.Symbolic(colptr, rowidx, perm, 0.05)
    iperm = np.argsort(S.perm)
    for handover in (1, -1):
        sym = lib.Symbolic(colptr, rowidx, perm, 0.05, {"handover": handover})
        sym.verify()
        F = None
        for col in (70, 150, 255, 299):
            print(f"case not-SPD column {col} handover {handover}", flush=True)
            v = v0.copy()
            v[colptr[col]] = -v[colptr[col]]
            with pytest.raises(oracle.NotSPD) as eo:
                S.factor(v)
            dv = torch.from_numpy(v).cuda()
            if F is None:
                F = lib.factorize(sym, dv)
            else:
                F.refactorize(dv)
            with pytest.raises(lib.NotSPD) as eg:
                F.sync()
            assert eg.value.column == eo.value.column == iperm[col]
        F.refactorize(torch.from_numpy(v0).cuda())
        F.sync()
        assert oracle.rel_frobenius(F.export(), S.factor(v0), S.lower_mask()) <= REL_F_FP64


def test_refactorize_and_repeat(torch_dev, lib):
    s = grid((15, 15, 15), seed=4, nrhs=1)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch_dev.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv)
    F.sync()
    L1 = F.export()
    F.refactorize(dv * 4.0)
    F.sync()
    L2 = F.export()
    assert np.max(np.abs(L2 - 2.0 * L1)) <= 1e-12 * np.max(np.abs(L1))
    F.refactorize(dv)
    F.sync()
    L3 = F.export()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    assert oracle.rel_frobenius(L3, L1, S.lower_mask()) <= 1e-14


def test_refactorize_new_values_wide(torch_dev, lib):
    """One pattern refactorized with unrelated values, alternately.  The
    blocks of a wide supernode hand their inverses to the tiles below inside
    one launch, so nothing may survive from the previous factorization."""
    n = 300
    rng = np.random.default_rng(11)
    r, c = np.tril_indices(n)
    vals = []
    for _ in range(2):
        X = rng.standard_normal((n, n))
        A = X @ X.T + n * np.eye(n)
        colptr, rowidx, v = W.lower_csc(n, r, c, A[r, c])
        vals.append(v)
    perm = np.arange(n, dtype=np.int32)
    sym = lib.Symbolic(colptr, rowidx, perm, 0.05)
    S = oracle.Symbolic(colptr, rowidx, perm, 0.05)
    refs = [S.factor(v) for v in vals]
    dvs = [torch_dev.from_numpy(v).cuda() for v in vals]
    F = lib.factorize(sym, dvs[0])
    for k in (1, 0, 1, 1, 0):
        F.refactorize(dvs[k])
        F.sync()
        assert oracle.rel_frobenius(F.export(), refs[k], S.lower_mask()) <= REL_F_FP64


def test_handover_concurrent_streams(torch_dev, lib):
    """Factorizations with the in-launch hand-over on four streams at once,
    so that trailing launches with waiting tiles share the device: every
    factor matches the oracle's, refactorization after refactorization.
    (The waiting tiles sit on the XCD of the tile they wait for, which
    spc_symbolic_verify checks, so no wait depends on another launch.)"""
    torch = torch_dev
    s = grid((30, 28, 26), seed=7)
    print(f"case concurrent hand-over n={s.n}", flush=True)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"handover": 1})
    sym.verify()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    ref = S.factor(s.values)
    dv = torch.from_numpy(s.values).cuda()
    streams = [torch.cuda.Stream() for _ in range(4)]
    facs = []
    for st in streams:
        facs.append(lib.factorize(sym, dv, "fp64", stream=st))
    for rep in range(3):
        for F, st in zip(facs, streams):
            F.refactorize(dv, stream=st)
    torch.cuda.synchronize()
    for F in facs:
        F.sync()  # raises if a pivot failed or a wait gave up
        assert oracle.rel_frobenius(F.export(), ref, S.lower_mask()) <= REL_F_FP64


def test_zero_rhs_and_empty(torch_dev, lib):
    s = grid((6, 6))
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm)
    F = lib.factorize(sym, torch_dev.from_numpy(s.values).cuda())
    F.sync()
    B = torch_dev.zeros((0, s.n), dtype=torch_dev.float64, device="cuda")
    F.solve(B)
    colptr = np.zeros(1, np.int64)
    sym0 = lib.Symbolic(colptr, np.zeros(0, np.int32), None)
    F0 = lib.factorize(sym0, torch_dev.zeros(1, dtype=torch_dev.float64, device="cuda"))
    F0.sync()


def test_batch_members_fp64(torch_dev, lib):
    specs = W.batch_specs(512, 0)
    picks = [i for i, (k, side) in enumerate(specs) if side <= (70 if k == "2d" else 16)][:4]
    for i in picks:
        s = W.batch_system(i, *specs[i], nrhs=3)
        relF, eta, _, _ = run_case(torch_dev, lib, s.colptr, s.rowidx, s.values, s.perm, s.B)
        assert relF <= REL_F_FP64 and eta <= BERR_FP64


def test_grid3d_60_full_size(torch_dev, lib):
    """The 60^3 7-point workload at full size, in the benchmark's launch
    configuration.  The oracle checks (a) a sampled subtree whose panels it
    computes exactly, (b) the backward error of the solve, (c) the factor
    residual A - L L^T on sampled columns, all in FP64 on the host."""
    torch = torch_dev
    s = W.grid3d_cond()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv)
    F.sync()
    Lg = F.export()
    # (a) subtree of a supernode at level 8 (a few seconds in the oracle)
    lev = S.level
    root = int(np.nonzero(lev == 8)[0][0])
    Ls, first = S.factor_subtree(s.values, root)
    sl = slice(int(S.lptr[first]), int(S.lptr[root + 1]))
    mask = S.lower_mask()[sl]
    assert factor_error(Lg, Ls, S, first, root) <= REL_F_FP64
    # (b) solve
    Bt = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    F.solve(Bt)
    X = Bt.cpu().numpy().T
    eta = oracle.backward_error(S.n, s.colptr, s.rowidx, s.values, X, s.B)
    print(f"60^3: eta={eta:.3e}")
    assert eta <= BERR_FP64
    # (c) sampled columns of Ahat - L L^T, relative to ||Ahat||
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values)
    P = S.perm
    Ah = A[P][:, P].tocsc()
    rng = np.random.default_rng(0)
    cols = np.concatenate([rng.choice(S.n, 40, replace=False), np.arange(S.n - 10, S.n)])
    sp, rp, rows, lp = S.super_ptr, S.rptr, S.rows, S.lptr
    snode = np.repeat(np.arange(S.nsuper), np.diff(sp))

    # L column j as sparse vector
    def lcol(j):
        t = snode[j]
        m = rp[t + 1] - rp[t]
        c = j - sp[t]
        vals = Lg[lp[t] + c * m: lp[t] + (c + 1) * m][c:]
        return rows[rp[t]:rp[t + 1]][c:], vals

    import scipy.sparse as ssp
    import scipy.sparse.linalg  # noqa: F401  (norm)
    # assemble L (CSC) from panels, then check columns of L L^T
    indptr = [0]; ind = []; dat = []
    for j in range(S.n):
        r_, v_ = lcol(j)
        ind.append(r_); dat.append(v_); indptr.append(indptr[-1] + r_.size)
    Lm = ssp.csc_matrix((np.concatenate(dat), np.concatenate(ind), np.array(indptr)), shape=(S.n, S.n))
    E = (Lm @ Lm[cols, :].T) - Ah[:, cols]
    res = ssp.linalg.norm(E) / ssp.linalg.norm(Ah[:, cols])
    print(f"60^3: sampled ||A - LL^T||/||A|| = {res:.3e}")
    assert res <= 1e-12


# ---- FP32 factorization and FP64 refinement ---------------------------------

def refined(torch, lib, s, precision, tol=1e-12, maxit=50, z=0.05):
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, z)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, precision)
    F.sync()
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    X = torch.zeros_like(B)
    info = F.solve_refined(dv, B, X, tol=tol, maxit=maxit)
    Xh = X.cpu().numpy().T
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Xh, s.B)
    print(f"refine {precision}: {info}, host eta={eta:.3e}", flush=True)
    return info, eta, F


def test_fp32_factor_error_vs_oracle(torch_dev, lib):
    """FP32 panels: the error against the FP64 oracle is reported; for this
    well-conditioned grid it must be of the order of FP32 rounding."""
    s = grid((18, 17, 16), seed=5, nrhs=2)
    relF, eta, _, _ = run_case(torch_dev, lib, s.colptr, s.rowidx, s.values, s.perm, s.B, precision="fp32")
    print(f"fp32 relF={relF:.3e} eta={eta:.3e}")
    assert relF <= 1e-4
    assert eta <= 1e-5


def test_fp32_refined_to_1e12(torch_dev, lib):
    s = grid((20, 19, 18), seed=6, nrhs=3)
    info, eta, _ = refined(torch_dev, lib, s, "fp32")
    assert info["converged"] and info["status"] == lib.OK
    assert eta <= 1e-12 and info["berr"] <= 1e-12


def test_fp32_refined_ill_conditioned_elasticity(torch_dev, lib):
    """27-point 3-dof operator with kappa = 1e8: kappa * u_fp32 > 1, so the
    classical steps stall and the FP64 CG phase must finish the job."""
    s = W.elasticity27((7, 6, 5), 88, 1, kappa=1e8, nrhs=4, power_iters=50)
    info, eta, _ = refined(torch_dev, lib, s, "fp32", maxit=200)
    assert info["converged"], info
    assert eta <= 1e-12


def test_fp64_refined_and_no_convergence_status(torch_dev, lib):
    s = grid((12, 12, 12), seed=7, nrhs=2)
    info, eta, F = refined(torch_dev, lib, s, "fp64")
    assert info["converged"] and eta <= 1e-12 and info["iterations"] <= 1
    s2 = W.elasticity27((6, 5, 5), 88, 2, kappa=1e8, nrhs=1, power_iters=50)
    info2, eta2, _ = refined(torch_dev, lib, s2, "fp32", tol=1e-15, maxit=0)
    assert info2["status"] == lib.NO_CONVERGENCE and not info2["converged"]
    assert info2["iterations"] == 0 and info2["berr"] > 0


# ---- batches: many systems in one level-scheduled pass ----------------------

def small_batch(count, seed=0, nrhs=2):
    specs = W.batch_specs(count * 8, seed)
    chosen = [(i, k, sd) for i, (k, sd) in enumerate(specs) if sd <= (60 if k == "2d" else 14)][:count]
    return [W.batch_system(i, k, sd, seed, nrhs=nrhs) for i, k, sd in chosen]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_factor_and_solve(torch_dev, lib, precision):
    torch = torch_dev
    systems = small_batch(12)
    syms = [lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05) for s in systems]
    batch = lib.Batch(syms, precision)
    dvs = [torch.from_numpy(s.values).cuda() for s in systems]
    batch.factorize(dvs)
    batch.sync()
    Bs = [torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda() for s in systems]
    batch.solve(Bs)
    for i, s in enumerate(systems):
        S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        F = batch.factor(i)
        relF = oracle.rel_frobenius(F.export(), S.factor(s.values), S.lower_mask())
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Bs[i].cpu().numpy().T, s.B)
        print(f"batch {precision} {s.name}: relF={relF:.2e} eta={eta:.2e}")
        if precision == "fp64":
            assert relF <= REL_F_FP64 and eta <= BERR_FP64
        else:
            assert relF <= 1e-4 and eta <= 1e-5
            X = torch.zeros_like(Bs[i])
            B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
            info = F.solve_refined(dvs[i], B0, X, tol=1e-12, maxit=30)
            assert info["converged"]
            assert oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B) <= 1e-12


def test_batch_alone_equals_in_mix(torch_dev, lib):
    """A system factored alone and inside a batch gives the same factor."""
    torch = torch_dev
    systems = small_batch(6, seed=1, nrhs=1)
    syms = [lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05) for s in systems]
    views = lib.factorize_batch(syms, [torch.from_numpy(s.values).cuda() for s in systems])
    for i, s in enumerate(systems):
        F = lib.factorize(syms[i], torch.from_numpy(s.values).cuda())
        F.sync()
        views[i].sync()
        a, b = F.export(), views[i].export()
        S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        assert oracle.rel_frobenius(b, a, S.lower_mask()) <= 1e-13


@pytest.mark.parametrize("nrhs", [3, 17])
def test_batch_solve_refined_per_system(torch_dev, lib, nrhs):
    """Merged refinement of an FP32 batch: a system that needs the CG phase
    (3-dof operator, kappa = 1e8) sits among grids that converge in a few
    classical steps; each must reach tol on its own, with its own reported
    error and step count, and 17 right-hand sides span two chunks."""
    torch = torch_dev
    systems = small_batch(5, seed=3, nrhs=nrhs)
    systems.insert(2, W.elasticity27((6, 5, 5), 88, 4, kappa=1e8, nrhs=nrhs, power_iters=50))
    syms = [lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05) for s in systems]
    batch = lib.Batch(syms, "fp32")
    batch.factorize([torch.from_numpy(s.values).cuda() for s in systems])
    batch.sync()
    Bs = [torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda() for s in systems]
    Xs = [torch.zeros_like(b) for b in Bs]
    out = batch.solve_refined(Bs, Xs, tol=1e-12, maxit=200)
    assert out["status"] == lib.OK, out
    for i, s in enumerate(systems):
        r = out["systems"][i]
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Xs[i].cpu().numpy().T, s.B)
        print(f"batch refine {s.name}: {r} host eta={eta:.2e}", flush=True)
        assert r["converged"] and r["berr"] <= 1e-12
        assert eta <= 1e-12
        # B is left as given
        assert np.array_equal(Bs[i].cpu().numpy().T, s.B)
    hard = out["systems"][2]["iterations"]
    easy = max(out["systems"][i]["iterations"] for i in range(len(systems)) if i != 2)
    assert easy < hard
    out0 = batch.solve_refined(Bs, Xs, tol=1e-15, maxit=0)
    assert out0["status"] == lib.NO_CONVERGENCE
    assert all(r["iterations"] == 0 for r in out0["systems"])


def test_batch_not_spd_names_system(torch_dev, lib):
    torch = torch_dev
    systems = small_batch(5, seed=2, nrhs=1)
    syms = [lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05) for s in systems]
    vals = [s.values.copy() for s in systems]
    bad = 3
    r = systems[bad].n // 3
    vals[bad][systems[bad].colptr[r]] *= -1.0
    batch = lib.Batch(syms, "fp64")
    batch.factorize([torch.from_numpy(v).cuda() for v in vals])
    with pytest.raises(lib.NotSPD) as e:
        batch.sync()
    S = oracle.Symbolic(systems[bad].colptr, systems[bad].rowidx, systems[bad].perm, 0.05)
    assert e.value.system == bad
    assert e.value.column == np.argsort(S.perm)[r]
    views = [batch.factor(i) for i in range(len(systems))]
    batch.close()  # views outlive the batch handle
    views[0].sync()
    with pytest.raises(lib.NotSPD):
        views[bad].sync()


# ---- serving: continuous batching -------------------------------------------

def test_serving_alone_equals_in_mix(torch_dev, lib):
    """Each request's solution is the same served alone (one slot) and in
    the mix (four slots, overlapping on the device), and every one reaches
    the 1e-12 backward error."""
    from paper_2202_09288_amd import serving as SV
    reqs_a = SV.make_requests(24, 200.0, 3, max_side={"2d": 48, "3d": 12})
    reqs_b = SV.make_requests(24, 200.0, 3, max_side={"2d": 48, "3d": 12})
    # re-solves name their factor request, so both runs pair the same systems
    alone = SV.Server(slots=1, keep_solutions=True, resolve_policy="fixed").run(reqs_a, time_scale=1.0)
    mix = SV.Server(slots=4, keep_solutions=True, resolve_policy="fixed").run(reqs_b, time_scale=1.0)
    assert [r.rid for r in alone] == [r.rid for r in mix]
    systems = {r.rid: r.system for r in alone if r.kind == "factor"}
    scales = {r.rid: r.values_scale for r in alone if r.kind == "factor"}
    kappas = {}
    for a, b in zip(alone, mix):
        assert a.status == "ok" and b.status == "ok", (a.status, b.status)
        assert a.berr <= 1e-12 and b.berr <= 1e-12
        s = systems[a.rid if a.kind == "factor" else a.target]
        sc = scales[a.rid if a.kind == "factor" else a.target]
        Bh = SV.Server.rhs(a, s).T if a.kind == "resolve" else s.B[:, :a.nrhs]
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values * sc, b.X, Bh)
        assert eta <= 1e-12
        # two solutions with backward error <= 1e-12 differ by at most
        # about 2 kappa(A) 1e-12 relatively (kappa in the infinity norm)
        key = a.rid if a.kind == "factor" else a.target
        if key not in kappas:
            Ad = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values * sc).toarray()
            kappas[key] = np.linalg.cond(Ad, np.inf)
        diff = np.max(np.abs(a.X - b.X)) / np.max(np.abs(a.X))
        assert diff <= 4 * kappas[key] * 1e-12, (diff, kappas[key])


def test_serving_admission_budget(torch_dev, lib):
    """A budget that holds about one factor forces queuing and eviction;
    nothing above the budget is admitted and results stay correct."""
    from paper_2202_09288_amd import serving as SV
    reqs = SV.make_requests(16, 1000.0, 4, max_side={"2d": 40, "3d": 10})
    srv = SV.Server(slots=3)
    one = max(srv.footprint(srv.symbolic(r.system), r.nrhs) for r in reqs if r.kind == "factor")
    srv.budget = int(one * 1.5)
    out = srv.run(reqs)
    srv.close()
    bad = [(r.rid, r.kind, r.status) for r in out if r.status != "ok"]
    assert not bad, bad
    assert 0 < srv.peak <= srv.budget
    assert all(r.berr <= 1e-12 for r in out)


def test_binding_rejects_mismatched_sizes(torch_dev, lib):
    """The library takes bare device pointers, so the binding checks every
    tensor's size against the analysis before a call: a value array shorter
    than nnz(lower A), right-hand sides whose length is not n, a result
    of another shape, and batch lists of the wrong length are refused on the
    host (ValueError) with no launch."""
    torch = torch_dev
    s = grid((7, 6), nrhs=2)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm)
    dv = torch.from_numpy(s.values).cuda()
    print("binding size checks", flush=True)
    with pytest.raises(ValueError):
        lib.factorize(sym, dv[:-1])
    F = lib.factorize(sym, dv)
    F.sync()
    with pytest.raises(ValueError):
        F.refactorize(dv[:1])
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    with pytest.raises(ValueError):
        F.solve(B[:, :-1].contiguous())
    with pytest.raises(ValueError):
        F.solve(B.reshape(1, 2, -1))
    with pytest.raises(ValueError):
        F.solve_refined(dv, B, torch.zeros_like(B[:1]))
    with pytest.raises(ValueError):
        F.solve_refined(dv[:-1], B, torch.zeros_like(B))
    batch = lib.Batch([sym, sym])
    with pytest.raises(ValueError):
        batch.factorize([dv])
    with pytest.raises(ValueError):
        batch.factorize([dv, dv[:-1]])
    batch.factorize([dv, dv])
    batch.sync()
    with pytest.raises(ValueError):
        batch.solve([B.clone()])
    with pytest.raises(ValueError):
        batch.solve([B.clone(), B[:1].clone()])
    with pytest.raises(ValueError):
        batch.solve_refined([B, B], [torch.zeros_like(B), torch.zeros_like(B[:1])])
    with pytest.raises(ValueError):
        lib.factorize_batch([sym, sym], [dv])
    # the checked calls still work after the refusals
    X = B.clone()
    F.solve(X)
    Xh = X.cpu().numpy().T
    assert oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Xh, s.B[:, :2]) <= BERR_FP64
    batch.close()


# ---- full-size workloads in the benchmark's launch configuration ----------

@pytest.mark.timeout(400)
def test_elasticity48_full_size(torch_dev, lib):
    """The 48^3 27-point 3-dof workload at full size (n = 331,776, kappa
    ~1e8, 4 RHS) with the cut-offs the benchmark takes for it: the FP32
    factor refined in FP64 reaches a host backward error of 1e-12 on every
    right-hand side; the FP64 factor of the same analysis matches the oracle
    on a sampled subtree, and its plain solve has a host backward error
    below 1e-12; the BF16-update factor, refined in FP64, either reaches
    1e-12 (checked on the host) or reports SPC_NO_CONVERGENCE with its best
    backward error, and its distance from the oracle on the same subtree is
    reported (parity unpinned: BF16 operands carry 8 significant bits)."""
    from paper_2202_09288_amd import tune
    torch = torch_dev
    print("elasticity 48^3: generating", flush=True)
    s = W.elast48()
    tuning = tune.load(tune.cache_key([s], "fp32", 4)) or {}
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning)
    dv = torch.from_numpy(s.values).cuda()
    B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    print(f"elasticity 48^3: fp32 factor + refinement, cut-offs {tuning}", flush=True)
    F = lib.factorize(sym, dv, "fp32")
    F.sync()
    X = torch.zeros_like(B0)
    info = F.solve_refined(dv, B0, X, tol=1e-12, maxit=200)
    F.close()
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
    print(f"elasticity 48^3 fp32 + refinement: {info}, host eta={eta:.3e}", flush=True)
    assert info["converged"] and info["status"] == lib.OK
    assert eta <= BERR_FP64
    print("elasticity 48^3: fp64 factor + solve", flush=True)
    F = lib.factorize(sym, dv, "fp64")
    F.sync()
    Bt = B0.clone()
    F.solve(Bt)
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Bt.cpu().numpy().T, s.B)
    print(f"elasticity 48^3 fp64: host eta={eta:.3e}", flush=True)
    assert eta <= BERR_FP64
    Lg = F.export()
    F.close()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    root = int(np.nonzero(S.level == 10)[0][0])
    Ls, first = S.factor_subtree(s.values, root)
    sl = slice(int(S.lptr[first]), int(S.lptr[root + 1]))
    relF = factor_error(Lg, Ls, S, first, root)
    print(f"elasticity 48^3 fp64: subtree of supernode {root}, relF={relF:.2e}", flush=True)
    assert relF <= REL_F_FP64
    tb = tune.load(tune.cache_key([s], "bf16upd", 4)) or {}
    print(f"elasticity 48^3: bf16-update factor + refinement, cut-offs {tb}", flush=True)
    symb = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tb)
    F = lib.factorize(symb, dv, "bf16upd")
    F.sync()
    Lb = F.export()
    X = torch.zeros_like(B0)
    info = F.solve_refined(dv, B0, X, tol=1e-12, maxit=200)
    F.close()
    relB = oracle.rel_frobenius(Lb[sl], Ls[sl], S.lower_mask()[sl])
    print(f"elasticity 48^3 bf16upd: {info}, subtree relF vs oracle {relB:.2e}", flush=True)
    assert info["status"] in (lib.OK, lib.NO_CONVERGENCE)
    assert np.isfinite(info["berr"]) and info["berr"] < 1.0
    if info["status"] == lib.OK:
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
        print(f"elasticity 48^3 bf16upd: host eta={eta:.3e}", flush=True)
        assert info["converged"] and eta <= BERR_FP64
    assert relF < relB <= 0.1  # the BF16 path really ran, at BF16's accuracy


@pytest.mark.timeout(300)
def test_batch512_full_size(torch_dev, lib):
    """The 512-system batch at full size (n from ~1k to 40k, 16 RHS each)
    with the cut-offs the benchmark takes for it, all systems in one
    schedule: in FP64, the largest 2D and 3D members and the first and last
    match the oracle's factor, and every member's plain solve has a host
    backward error below 1e-12; in FP32, the batched FP64 refinement brings
    every member to 1e-12."""
    from paper_2202_09288_amd import tune
    torch = torch_dev
    print("batch of 512: generating", flush=True)
    systems = W.batch512()
    tuning = tune.load(tune.cache_key(systems, "fp32", 16)) or {}
    syms = [lib.Symbolic(x.colptr, x.rowidx, x.perm, 0.05, tuning) for x in systems]
    dvs = [torch.from_numpy(x.values).cuda() for x in systems]
    Bs0 = [torch.from_numpy(np.ascontiguousarray(x.B.T)).cuda() for x in systems]
    specs = W.batch_specs(len(systems), 0)
    big3 = max((i for i, (k, _) in enumerate(specs) if k == "3d"), key=lambda i: specs[i][1])
    big2 = max((i for i, (k, _) in enumerate(specs) if k == "2d"), key=lambda i: specs[i][1])

    def worst_eta(Xs):
        return max(oracle.backward_error(x.n, x.colptr, x.rowidx, x.values, b.cpu().numpy().T, x.B)
                   for x, b in zip(systems, Xs))

    print(f"batch of 512: fp64 factor + solve, cut-offs {tuning}", flush=True)
    batch = lib.Batch(syms, "fp64")
    batch.factorize(dvs)
    batch.sync()
    Bs = [b.clone() for b in Bs0]
    batch.solve(Bs)
    for i in sorted({0, big2, big3, len(systems) - 1}):
        x = systems[i]
        S = oracle.Symbolic(x.colptr, x.rowidx, x.perm, 0.05)
        relF = oracle.rel_frobenius(batch.factor(i).export(), S.factor(x.values), S.lower_mask())
        print(f"batch of 512, fp64 member {x.name}: relF={relF:.2e}", flush=True)
        assert relF <= REL_F_FP64
    eta = worst_eta(Bs)
    print(f"batch of 512 fp64: worst host eta={eta:.3e}", flush=True)
    assert eta <= BERR_FP64
    batch.close()
    print("batch of 512: fp32 factor + batched refinement", flush=True)
    batch = lib.Batch(syms, "fp32")
    batch.factorize(dvs)
    batch.sync()
    Xs = [torch.zeros_like(b) for b in Bs0]
    out = batch.solve_refined(Bs0, Xs, tol=1e-12, maxit=100)
    assert out["status"] == lib.OK and all(r["converged"] for r in out["systems"])
    eta = worst_eta(Xs)
    print(f"batch of 512 fp32 + refinement: max iterations "
          f"{max(r['iterations'] for r in out['systems'])}, worst host eta={eta:.3e}", flush=True)
    assert eta <= BERR_FP64
    batch.close()


@pytest.mark.timeout(300)
def test_serving_full_size_mix(torch_dev, lib):
    """Serving at the full sizes of its mix (batch-mix systems up to 40k
    unknowns and 50^3 7-point grids, 8 RHS each, 30% re-solves of resident
    factors), four requests overlapping on the device: every request ends
    ok, and its solution, checked on the host against the values it was
    factored with, has a backward error below 1e-12.  Seed 6 is taken
    because its first 32 requests hold three 50^3 factor requests."""
    from paper_2202_09288_amd import serving as SV
    print("serving full-size mix: generating", flush=True)
    reqs = SV.make_requests(32, 200.0, 6)
    big = [r.rid for r in reqs if r.kind == "factor" and r.system.n == 50 ** 3]
    assert len(big) >= 3, big
    srv = SV.Server(slots=4, keep_solutions=True)
    print("serving full-size mix: running", flush=True)
    out = srv.run(reqs, time_scale=1.0)
    srv.close()
    systems = {r.rid: r.system for r in reqs if r.kind == "factor"}
    scales = {r.rid: r.values_scale for r in reqs if r.kind == "factor"}
    worst = 0.0
    for r in out:
        assert r.status == "ok" and r.berr <= 1e-12, (r.rid, r.kind, r.status, r.berr)
        key = r.rid if r.kind == "factor" else r.target
        s, sc = systems[key], scales[key]
        Bh = SV.Server.rhs(r, s).T if r.kind == "resolve" else s.B[:, :r.nrhs]
        worst = max(worst, oracle.backward_error(s.n, s.colptr, s.rowidx, s.values * sc, r.X, Bh))
    print(f"serving full-size mix: {len(out)} requests, worst host eta={worst:.3e}", flush=True)
    assert len(out) == len(reqs)
    assert worst <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dims", [(40, 37), (12, 11, 10), (16, 15, 14)])
def test_factor_componentwise_backward_error(torch_dev, lib, dims, precision):
    """The computed factor of either precision, independently of the oracle's
    numbers: Cholesky's componentwise backward error bound (Demmel; Higham,
    Accuracy and Stability, Thm. 10.3) with k the most nonzeros in a row of
    L, plus the rounding of A to the working precision:
    |P^T A P - L L^T| <= gamma_{k+2} (|L| |L^T| + |P^T A P|),
    gamma_j = j u / (1 - j u), u = 2^-53 or 2^-24 (measured worst entry:
    about 0.02 of the bound)."""
    torch = torch_dev
    s = grid(dims, seed=3)
    print(f"componentwise bound {dims} {precision}", flush=True)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    F = lib.factorize(sym, torch.from_numpy(s.values).cuda(), precision)
    F.sync()
    L = np.tril(S.to_dense_L(F.export()))
    F.close()
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values).toarray()
    Ah = A[np.ix_(S.perm, S.perm)]
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    k = int((L != 0).sum(axis=1).max()) + 2
    gamma = k * u / (1 - k * u)
    E = np.abs(Ah - L @ L.T)
    bound = gamma * (np.abs(L) @ np.abs(L).T + np.abs(Ah))
    assert np.all(E <= bound), float((E / np.where(bound > 0, bound, np.inf)).max())


# ---- full-size 60^3: every panel against the oracle ------------------------

@pytest.mark.timeout(600)
def test_grid3d_60_every_panel(torch_dev, lib):
    """The 60^3 7-point workload in the benchmark's launch configuration,
    every panel (the 5,340-wide root and its 84-step chain included) compared
    with the oracle's factor, per supernode and as a whole.  The oracle runs
    in its deterministic multi-threaded mode (bit-identical to the
    sequential one) on the host's cores."""
    import os
    torch = torch_dev
    s = W.grid3d_cond()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    print(f"60^3 every panel: oracle on {threads} threads", flush=True)
    Lref = S.factor(s.values, threads=threads)
    from paper_2202_09288_amd import tune
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning=tune.load(tune.cache_key([s], "fp64", 1)) or {})
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv)
    F.set_graph(True)
    F.refactorize(dv)  # the replayed graph, as the benchmark runs it
    F.sync()
    Lg = F.export()
    err = factor_error(Lg, Lref, S)
    print(f"60^3 every panel: {S.nsuper} supernodes, max(relF, worst supernode) = {err:.3e}", flush=True)
    assert err <= REL_F_FP64


# ---- device-side waits that give up -----------------------------------------

def test_wait_limit_reports_device_error(torch_dev, lib):
    """With the poll limit at 0 every wait of one workgroup on another gives
    up at once (the kernels still run to their end, on garbage): the
    factorization's hand-over waits and the persistent solve sweeps' waits
    both report SPC_DEVICE_ERROR, never SPC_OK or SPC_NOT_SPD; a
    factorization with the default limit clears it again."""
    torch = torch_dev
    s = W.laplacian((24, 24, 24), "7pt", 88, 5, unit=False, shift=1e-2, nrhs=1)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    assert sym.info["max_width"] >= 2 * 64  # blocks 1.. are handed over
    assert sym.info["solve_persistent_levels"] > 0
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv)
    F.sync()
    # factorization waits
    F.set_wait_limit(0)
    F.refactorize(dv)
    with pytest.raises(lib.SpcError) as e:
        F.sync()
    assert e.value.status == lib.DEVICE_ERROR
    # back to the default: the factor is good again
    F.set_wait_limit(1 << 20)
    F.refactorize(dv)
    F.sync()
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    F.solve(B.clone())
    F.sync()
    # solve waits only (the factor is good)
    F.set_wait_limit(0)
    X = B.clone()
    F.solve(X)
    with pytest.raises(lib.SpcError) as e:
        F.sync()
    assert e.value.status == lib.DEVICE_ERROR
    Xr = torch.zeros_like(B)
    with pytest.raises(lib.SpcError) as e:
        F.solve_refined(dv, B, Xr)
    assert e.value.status == lib.DEVICE_ERROR


# ---- NaN in the refinement norms ----------------------------------------------

def test_refined_nan_rhs_is_not_converged(torch_dev, lib):
    """A NaN in b reaches the residual and the solution; the refinement's
    column maxima carry it (as +Inf), so the result is SPC_NO_CONVERGENCE,
    never a converged status with a NaN solution: single factor and batch."""
    torch = torch_dev
    s = grid((20, 19, 18), nrhs=2)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, "fp32")
    F.sync()
    Bh = np.ascontiguousarray(s.B.T).copy()
    Bh[1, 7] = np.nan
    B = torch.from_numpy(Bh).cuda()
    X = torch.zeros_like(B)
    res = F.solve_refined(dv, B, X, maxit=5)
    print(f"single: {res}", flush=True)
    assert res["status"] == lib.NO_CONVERGENCE and not res["converged"]
    systems = small_batch(3, seed=4)
    syms = [lib.Symbolic(x.colptr, x.rowidx, x.perm, 0.05) for x in systems]
    batch = lib.Batch(syms, "fp32")
    dvs = [torch.from_numpy(x.values).cuda() for x in systems]
    batch.factorize(dvs)
    batch.sync()
    Bs = []
    for i, x in enumerate(systems):
        b = np.ascontiguousarray(x.B.T).copy()
        if i == 1:
            b[0, 3] = np.nan
        Bs.append(torch.from_numpy(b).cuda())
    Xs = [torch.zeros_like(b) for b in Bs]
    out = batch.solve_refined(Bs, Xs, maxit=5)
    print(f"batch: {out}", flush=True)
    assert out["status"] == lib.NO_CONVERGENCE
    assert not out["systems"][1]["converged"]
    assert out["systems"][0]["converged"] and out["systems"][2]["converged"]


# ---- BF16 Schur updates (SPC_FP32_BF16UPD) + FP64 refinement ----------------

def test_bf16upd_factor_error_vs_oracle(torch_dev, lib):
    """The BF16-update factor against the FP64 oracle on a grid whose big
    supernodes go through the BF16 tile kernels (64- and 128-tiles).  Parity
    unpinned: no closed form bounds it; BF16 rounds each operand to 8
    significant bits (unit roundoff 2^-9), so relF of a few 1e-3 is what the
    operands' rounding alone gives, and a wrong MFMA operand layout would
    give relF of order 1.  Refined in FP64 it meets the 1e-12 bar."""
    torch = torch_dev
    s = grid((30, 30, 30), nrhs=3)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lref = S.factor(s.values)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, tuning={"small_w": -1, "tiny_w": -1, "big_min": 64,
                                                                 "big_min_k": 32})
    dv = torch.from_numpy(s.values).cuda()
    res = {}
    for prec in ("fp32", "bf16upd"):
        F = lib.factorize(sym, dv, prec)
        F.sync()
        res[prec] = oracle.rel_frobenius(F.export(), Lref, S.lower_mask())
        B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
        X = torch.zeros_like(B)
        info = F.solve_refined(dv, B, X, tol=1e-12, maxit=50)
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
        print(f"30^3 {prec}: relF vs oracle {res[prec]:.3e}, refinement {info}, host eta {eta:.3e}", flush=True)
        assert info["converged"] and eta <= BERR_FP64
    assert res["bf16upd"] <= 2e-2
    assert res["bf16upd"] > res["fp32"]  # the BF16 path really ran


def test_bf16upd_refined_elasticity_kappa1e6(torch_dev, lib):
    """A kappa = 1e6 elasticity case (3x3 blocks of random orientation):
    the BF16-update factor (pivots below 2^-8 of their diagonal entry raised
    to it) refined in FP64 (classical steps, then CG) to a backward error of
    1e-12 on 4 right-hand sides.  Its distance from the oracle's factor is
    reported (parity unpinned)."""
    torch = torch_dev
    s = W.elasticity27((14, 13, 12), 88, 1, kappa=1e6, nrhs=4, power_iters=30)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, "bf16upd")
    F.sync()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    relF = oracle.rel_frobenius(F.export(), S.factor(s.values), S.lower_mask())
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    X = torch.zeros_like(B)
    info = F.solve_refined(dv, B, X, tol=1e-12, maxit=200)
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
    print(f"elasticity kappa 1e6 n={s.n} bf16upd: relF vs oracle {relF:.3e}, {F.pivot_floors()} pivots raised "
          f"to their floor, {info}, host eta {eta:.3e}", flush=True)
    assert info["converged"] and info["status"] == lib.OK
    assert eta <= BERR_FP64


# ---- the persistent launch over the small subtrees ---------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_persistent_small_subtrees_batch(torch_dev, lib, precision):
    """A batch whose small subtrees (of every system, all their levels) run
    as one persistent launch with device-side dependency counters: every
    system's factor against the oracle, and the solves."""
    torch = torch_dev
    systems = small_batch(16, seed=3)
    syms = [lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"persist": 1}) for s in systems]
    batch = lib.Batch(syms, precision)
    dvs = [torch.from_numpy(s.values).cuda() for s in systems]
    batch.set_profiling(True)
    batch.factorize(dvs)
    batch.sync()
    ks = batch.kernel_stats()
    print(f"persistent launch: {ks['small_trees']}", flush=True)
    assert ks["small_trees"]["launches"] == 1
    Bs = [torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda() for s in systems]
    batch.solve(Bs)
    for i, s in enumerate(systems):
        S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        Lref = S.factor(s.values)
        Lg = batch.factor(i).export()
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Bs[i].cpu().numpy().T, s.B)
        if precision == "fp64":
            assert factor_error(Lg, Lref, S) <= REL_F_FP64 and eta <= BERR_FP64
        else:
            assert oracle.rel_frobenius(Lg, Lref, S.lower_mask()) <= 1e-4 and eta <= 1e-5


def test_persistent_small_subtrees_not_spd(torch_dev, lib):
    """A failing pivot inside the persistent launch is reported at the
    oracle's column, and every later supernode still runs to its end."""
    s = grid((13, 12, 11), seed=6)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    iperm = np.argsort(S.perm)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, {"persist": 1})
    for r in (5, s.n // 3):
        v = s.values.copy()
        v[s.colptr[r]] = -v[s.colptr[r]]
        with pytest.raises(oracle.NotSPD) as eo:
            S.factor(v)
        F = lib.factorize(sym, torch_dev.from_numpy(v).cuda())
        with pytest.raises(lib.NotSPD) as eg:
            F.sync()
        assert eg.value.column == eo.value.column == iperm[r]


def test_serving_pooled_refactorization(torch_dev, lib):
    """Serving in FP64 with a budget that holds a few factors: factor
    requests of a known pattern refactorize an idle slot of that pattern
    (spc_refactorize, replayed from the slot's graph), and every factor
    served, pooled or new, matches the oracle's factor of the values it was
    given; re-solves pick resident factors and never miss."""
    from paper_2202_09288_amd import serving as SV
    reqs = SV.make_requests(40, 2000.0, 5, max_side={"2d": 40, "3d": 11})
    srv = SV.Server(slots=2, precision="fp64", export_factors=True, keep_solutions=True)
    fps = {r.key: srv.footprint(srv.symbolic(r.system), r.nrhs) for r in reqs if r.kind == "factor"}
    srv.budget = int(3.5 * max(fps.values()))
    out = srv.run(reqs)
    srv.close()
    summ = SV.summarize(out, 1.0)
    print(f"pooled serving: {summ}", flush=True)
    assert summ["ok"] == len(out) and summ["misses"] == 0
    assert summ["pooled_factor_requests"] > 0
    refs = {}
    for r in out:
        if r.kind != "factor":
            continue
        s = r.system
        if r.key not in refs:
            refs[r.key] = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        S = refs[r.key]
        err = factor_error(r.L, S.factor(s.values * r.values_scale), S)
        assert err <= REL_F_FP64, (r.rid, r.pooled, err)
    assert srv.peak <= srv.budget


def test_graph_capture_beside_other_threads(torch_dev, lib):
    """One thread captures factorization graphs (a new factor with graph
    replay on, each first refactorization captures) while two others
    factorize, synchronize, solve and export on streams of their own: no
    call fails (host copies never go through the legacy stream, which the
    runtime refuses while another thread captures), and every factor matches
    the oracle's."""
    import threading
    torch = torch_dev
    systems = [grid((23, 21), seed=40 + i, nrhs=2) for i in range(3)]
    refs = []
    for s in systems:
        S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
        refs.append((S, S.factor(s.values)))
    errors, worst = [], [0.0]

    def work(i, capture):
        try:
            s = systems[i]
            S, Lref = refs[i]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
                dv = torch.from_numpy(s.values).cuda()
                for _ in range(12):
                    F = lib.factorize(sym, dv, stream=st)
                    if capture:
                        F.set_graph(True)
                        F.refactorize(dv, stream=st)  # captures, then replays
                    F.sync()
                    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
                    F.solve(B, stream=st)
                    st.synchronize()
                    worst[0] = max(worst[0], factor_error(F.export(), Lref, S))
                    F.close()
        except Exception as e:  # recorded, checked below
            errors.append(f"thread {i}: {e}")

    threads = [threading.Thread(target=work, args=(i, i == 0)) for i in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    print(f"capture beside other threads: errors {errors}, worst factor error {worst[0]:.2e}", flush=True)
    assert not errors
    assert worst[0] <= REL_F_FP64


@pytest.mark.parametrize("case", ["grid7", "elasticity27"])
def test_device_backward_error_matches_host(torch_dev, lib, case):
    """The backward error the refinement computes on the device (FP64
    residual, matrix and vector infinity norms: the short-row and the
    long-row lane groups) equals the oracle's host definition of the same
    solution, per right-hand side maximum, to a relative 1e-6."""
    torch = torch_dev
    s = grid((14, 13, 12), seed=21, nrhs=3) if case == "grid7" else \
        W.elasticity27((7, 6, 5), 21, 0, kappa=1e4, nrhs=3, power_iters=5)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, "fp32")
    F.sync()
    B = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    X = torch.zeros_like(B)
    info = F.solve_refined(dv, B, X, tol=0.0, maxit=0)  # the plain FP32 solve, measured in FP64
    eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
    print(f"{case}: device berr {info['berr']:.6e}, host eta {eta:.6e}", flush=True)
    assert eta > 1e-12  # an FP32 solve: far from the FP64 level, so the two norms are tested
    assert abs(info["berr"] - eta) <= 1e-6 * eta


# ---- orderings computed without coordinates ---------------------------------

@pytest.mark.parametrize("method", ["nd", "md"])
def test_graph_orderings_factor_and_solve(torch_dev, lib, method):
    """The factor under an order spc_order computes (graph nested dissection,
    minimum degree) matches the oracle's factor under that order, and the
    solution, which no order changes, matches the oracle's solution under the
    coordinate nested dissection of the workload (within kappa u)."""
    torch = torch_dev
    s = grid((22, 21, 20), seed=12, nrhs=2) if method == "nd" else grid((60, 61), seed=12, nrhs=2)
    perm = lib.order(s.colptr, s.rowidx, method)
    relF, eta, F, S = run_case(torch, lib, s.colptr, s.rowidx, s.values, perm, s.B)
    print(f"{method}: relF={relF:.2e} eta={eta:.2e}", flush=True)
    assert relF <= REL_F_FP64 and eta <= BERR_FP64
    Bt = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    F.solve(Bt)
    X = Bt.cpu().numpy().T
    Sc = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Xc = Sc.solve(Sc.factor(s.values), s.B)
    assert np.max(np.abs(X - Xc)) <= 1e-9 * np.max(np.abs(Xc))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_few_rhs_instantiations(torch_dev, lib, precision):
    """Right-hand-side counts that take the 4- and 8-column forms of the
    backward sweep (and the 16-column one beyond), in the level launches and
    the persistent top sweep: each column's solution meets the bar of its
    precision and equals the one-column solve's."""
    torch = torch_dev
    s = grid((26, 25, 24), seed=14, nrhs=11)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    assert sym.info["solve_persistent_levels"] > 0
    F = lib.factorize(sym, torch.from_numpy(s.values).cuda(), precision)
    F.sync()
    bar = BERR_FP64 if precision == "fp64" else 1e-5
    B0 = np.ascontiguousarray(s.B.T)
    one = np.zeros_like(B0)
    for q in range(B0.shape[0]):
        x = torch.from_numpy(B0[q].copy()).cuda()
        F.solve(x)
        one[q] = x.cpu().numpy()
    for nrhs in (2, 3, 4, 5, 8, 11):
        X = torch.from_numpy(B0[:nrhs].copy()).cuda()
        F.solve(X)
        Xh = X.cpu().numpy()
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, Xh.T, s.B[:, :nrhs])
        diff = np.max(np.abs(Xh - one[:nrhs])) / np.max(np.abs(one[:nrhs]))
        print(f"{precision} nrhs={nrhs}: eta={eta:.2e}, against one at a time {diff:.2e}", flush=True)
        assert eta <= bar
        assert diff <= (1e-12 if precision == "fp64" else 1e-4)


def handover_cases():
    """A grid whose top supernodes span many column blocks, and one dense
    supernode of 10 blocks with a ragged last one."""
    g = grid((40, 38, 36), seed=21, nrhs=16)
    n = 611
    rng = np.random.default_rng(6)
    Xd = rng.standard_normal((n, n))
    A = Xd @ Xd.T + n * np.eye(n)
    r, c = np.tril_indices(n)
    colptr, rowidx, values = W.lower_csc(n, r, c, A[r, c])
    return [("grid-40x38x36", g.colptr, g.rowidx, g.values, g.perm, g.B),
            ("dense-611", colptr, rowidx, values, np.arange(n, dtype=np.int32), rng.standard_normal((n, 16)))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_block_handover(torch_dev, lib, precision):
    """Solves whose every level is persistent (blocks of a supernode hand
    over through the polled buffers) meet the precision's bar for 1, 3, 4, 8
    and 16 right-hand sides (every instantiation), twice in a row (the
    buffers are set again per solve), and agree with the level launches,
    which hand nothing over."""
    torch = torch_dev
    bar = BERR_FP64 if precision == "fp64" else 1e-5
    for name, colptr, rowidx, values, perm, B in handover_cases():
        n = len(colptr) - 1
        levels = lib.Symbolic(colptr, rowidx, perm, 0.05, {"solve_persist_max": -1})
        every = lib.Symbolic(colptr, rowidx, perm, 0.05, {"solve_persist_max": 1 << 30})
        assert levels.info["solve_handovers"] == 0 and every.info["solve_handovers"] > 0
        dv = torch.from_numpy(values).cuda()
        Fl = lib.factorize(levels, dv, precision)
        Fe = lib.factorize(every, dv, precision)
        Fl.sync()
        Fe.sync()
        for q in (1, 3, 4, 8, 16):
            B0 = np.ascontiguousarray(B[:, :q].T)
            Xl = torch.from_numpy(B0.copy()).cuda()
            Fl.solve(Xl)
            ref = Xl.cpu().numpy()
            for rep in range(2):
                Xe = torch.from_numpy(B0.copy()).cuda()
                Fe.solve(Xe)
                Xh = Xe.cpu().numpy()
                eta = oracle.backward_error(n, colptr, rowidx, values, Xh.T, B[:, :q])
                diff = np.max(np.abs(Xh - ref)) / np.max(np.abs(ref))
                print(f"block hand-over {name} {precision} nrhs={q} rep={rep}: eta={eta:.2e}, "
                      f"against the level launches {diff:.2e}", flush=True)
                assert eta <= bar
                assert diff <= (1e-10 if precision == "fp64" else 1e-3)


def test_refined_starts_with_cg_after_a_switch(torch_dev, lib):
    """After a refined solve that switched to CG (kappa = 1e8 elasticity in
    FP32), the next one with the same factorization starts with CG: it meets
    1e-12 in no more steps; a new factorization starts over and meets it
    again."""
    torch = torch_dev
    s = W.elasticity27((7, 6, 5), 88, 1, kappa=1e8, nrhs=4, power_iters=50)
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, "fp32")
    F.sync()
    B0 = torch.from_numpy(np.ascontiguousarray(s.B.T)).cuda()
    steps = []
    for rep in range(3):
        if rep == 2:
            F.refactorize(dv)
            F.sync()
        X = torch.zeros_like(B0)
        info = F.solve_refined(dv, B0, X, tol=1e-12, maxit=200)
        eta = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X.cpu().numpy().T, s.B)
        print(f"refined solve {rep}: {info}, eta={eta:.2e}", flush=True)
        assert info["converged"] and eta <= 1e-12
        steps.append(info["iterations"])
    assert steps[1] <= steps[0]


def test_hbm_budget_factor_and_batch(torch_dev, lib):
    """The analysis's device budget: a factorization at exactly its footprint
    runs and matches the oracle, one byte less is refused with
    SPC_OUT_OF_MEMORY; a batch is held to its members' smallest budget over
    the merged footprint."""
    torch = torch_dev
    s = grid((9, 7, 11), nrhs=2)
    need = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05).info["factor_bytes_fp64"]
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, hbm_budget=need)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, "fp64")
    F.sync()
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    Lref = S.factor(s.values)
    assert factor_error(F.export(), Lref, S) <= REL_F_FP64
    tight = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, hbm_budget=need - 1)
    with pytest.raises(lib.SpcError) as e:
        lib.factorize(tight, dv, "fp64")
    assert e.value.status == lib.OUT_OF_MEMORY
    # FP32 needs less than the FP64 footprint
    F32 = lib.factorize(tight, dv, "fp32")
    F32.sync()
    # two members that each fit alone, merged over the smaller budget
    with pytest.raises(lib.SpcError) as e:
        lib.Batch([sym, lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)], "fp64")
    assert e.value.status == lib.OUT_OF_MEMORY
    roomy = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, hbm_budget=3 * need)
    batch = lib.Batch([roomy, roomy], "fp64")
    batch.factorize([dv, dv])
    batch.sync()
    for i in range(2):
        assert factor_error(batch.factor(i).export(), Lref, S) <= REL_F_FP64
