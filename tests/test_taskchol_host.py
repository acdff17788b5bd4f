"""The host task-parallel baseline (the paper's Sec. 3-4 method) on the CPU:
every strategy reaches the oracle's factor (relF within the FP64 bar, per
supernode), Algorithm 1 (Opt-D) and the hybrid rule on hand-worked values,
and a failing pivot is reported at the oracle's column."""
import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import spchol  # noqa: F401  (conftest builds the libraries)
from paper_2202_09288_amd import taskchol as T
from paper_2202_09288_amd import workloads as W


def test_opt_d_hand_values():
    """Algorithm 1 by hand.  C = [0,0,0,0,1,1,2,2,5,10], n = 100: goal =
    max(1.1 * 10, 100 / 14) = 11; from D = 11 the histogram adds the outer
    tasks with 10 updates (tasks 20), then 5 (tasks 25); the loop runs on
    while D > 0.3 * 10 and stops at D = 3.  With n = 1400 the goal is 100
    tasks, never reached (31 at most), so D runs down to 0."""
    C = [0, 0, 0, 0, 1, 1, 2, 2, 5, 10]
    assert T.opt_d(100, C) == 3
    assert T.opt_d(1400, C) == 0
    # no updates anywhere: maxChildren = 0, D starts at 1 and the goal of
    # 1.1 n_super tasks forces it to 0
    assert T.opt_d(50, [0, 0, 0]) == 0
    # the goal rule: 3000 supernodes with one update each and one with 100;
    # a goal of 1.1 * 3001 tasks needs more than the big task alone, D = 1
    C = [1] * 3000 + [100]
    assert T.opt_d(3001, C) == 1
    # the n_super / 1000 rule: 10,000 supernodes, one with 1000 updates, nine
    # with 200, the rest none; the goal (11,000 tasks) is met at D = 1000
    # and D <= 0.3 * 1000 at D = 300, but only one outer task would be split
    # there, fewer than 10,000 / 1000, so D comes down to 200
    C = [1000] + [200] * 9 + [0] * 9990
    assert T.opt_d(10000, C) == 200


def test_hybrid_rule_hand_values():
    """Sec. 4.4: mt-BLAS above 50 columns per supernode, or above 20 with a
    density below 1e-4; Opt-D-Cost otherwise."""
    assert T.hybrid_choice(60.0, 1.0) == "mt_blas"
    assert T.hybrid_choice(30.0, 5e-5) == "mt_blas"
    assert T.hybrid_choice(30.0, 2e-4) == "opt_d_cost"
    assert T.hybrid_choice(50.0, 1e-3) == "opt_d_cost"
    assert T.hybrid_choice(10.0, 1e-6) == "opt_d_cost"


def plan_of(s):
    sym = spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    return T.TaskPlan.from_symbolic(sym, s.colptr, s.rowidx), sym


@pytest.mark.parametrize("dims", [(23, 21), (11, 10, 9), (16, 15, 14)])
@pytest.mark.parametrize("strategy", list(T.STRATEGIES))
def test_strategies_match_oracle(dims, strategy):
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 77, 3, unit=False, shift=1e-2, nrhs=1)
    plan, sym = plan_of(s)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    assert np.array_equal(sym.export("lptr"), S.lptr)
    Lref = S.factor(s.values)
    for threads in (1, 4):
        Lx, info = plan.factor(s.values, strategy, threads=threads)
        mask = S.lower_mask()
        glob = oracle.rel_frobenius(Lx, Lref, mask)
        per = oracle.supernode_rel_errors(Lx, Lref, S.lptr, mask).max()
        assert max(glob, per) <= 1e-12, (strategy, threads, glob, per)


def test_nested_creates_one_inner_task_per_update():
    s = W.laplacian((12, 11, 10), "7pt", 77, 1, unit=False, shift=1e-2, nrhs=1)
    plan, _ = plan_of(s)
    st = plan.stats()
    C = plan.update_counts()
    assert st["updates"] == int(C.sum()) and st["max_updates"] == int(C.max())
    assert st["opt_d"] == T.opt_d(s.n, C)
    assert st["tasks_nested"] == st["nsuper"] + st["updates"]
    _, info = plan.factor(s.values, "nested", threads=2)
    assert info["inner_tasks"] == st["updates"]
    _, info = plan.factor(s.values, "opt_d", threads=2)
    assert info["inner_tasks"] == st["tasks_opt_d"] - st["nsuper"]
    _, info = plan.factor(s.values, "opt_d_cost", threads=2)
    assert info["inner_tasks"] == st["tasks_opt_d_cost"] - st["nsuper"]
    _, info = plan.factor(s.values, "nonested", threads=2)
    assert info["inner_tasks"] == 0


@pytest.mark.parametrize("strategy", ["nonested", "nested", "mt_blas"])
def test_not_spd_column(strategy):
    s = W.laplacian((9, 8, 7), "7pt", 77, 2, unit=False, shift=1e-2, nrhs=1)
    plan, _ = plan_of(s)
    S = oracle.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    v = s.values.copy()
    r = s.n // 2
    v[s.colptr[r]] = -v[s.colptr[r]]
    with pytest.raises(oracle.NotSPD) as eo:
        S.factor(v)
    with pytest.raises(T.NotSPD) as et:
        plan.factor(v, strategy, threads=3)
    assert et.value.column == eo.value.column


def test_library_exports_every_declared_function():
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(root, "include", "taskchol.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(tch_[a-z_0-9]+)\s*\(", txt)))
    assert names and set(names) == set(T.EXPORTS)
    for nm in names:
        assert hasattr(T._lib, nm), nm
