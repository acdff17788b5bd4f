"""spc_solve_noalloc (the solve whose work lives in the library's fixed
scratch array) against spc_solve, through the C ABI: the same solution to the
solve bar (normwise backward error <= 1e-12 in FP64, host residual) on two
calls in a row, the second on a smaller input, and in chunks when the
right-hand sides do not all fit the array at once."""
import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import workloads as W

pytestmark = pytest.mark.gpu

BERR_FP64 = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def lib(torch_dev):
    from paper_2202_09288_amd import spchol
    return spchol


def both_solves(torch, lib, s, precision, nrhs):
    sym = lib.Symbolic(s.colptr, s.rowidx, s.perm, 0.05)
    dv = torch.from_numpy(s.values).cuda()
    F = lib.factorize(sym, dv, precision)
    F.sync()
    Bh = np.ascontiguousarray(s.B.T[:nrhs])
    X1 = torch.from_numpy(Bh.copy()).cuda()
    F.solve(X1)
    X2 = torch.from_numpy(Bh.copy()).cuda()
    F.solve_noalloc(X2)
    F.sync()
    x1 = X1.cpu().numpy().T
    x2 = X2.cpu().numpy().T
    B = Bh.T
    e1 = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, x1, B)
    e2 = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, x2, B)
    d = float(np.max(np.abs(x1 - x2)) / max(np.max(np.abs(x1)), 1e-300))
    print(f"n={s.n} nrhs={nrhs} {precision}: eta solve {e1:.2e}, eta noalloc {e2:.2e}, max rel diff {d:.2e}",
          flush=True)
    return e1, e2, d


def test_noalloc_matches_solve_two_calls(torch_dev, lib):
    """Two calls in a row, the second on a smaller system with fewer
    right-hand sides: the scratch keeps the first call's contents, and the
    second must not depend on them."""
    big = W.laplacian((30, 30, 30), "7pt", 88, 1, unit=False, shift=1e-2, nrhs=20)
    small = W.laplacian((40, 37), "5pt", 88, 2, unit=False, shift=1e-2, nrhs=3)
    for s, nrhs in ((big, 20), (small, 3)):
        e1, e2, d = both_solves(torch_dev, lib, s, "fp64", nrhs)
        assert e1 <= BERR_FP64 and e2 <= BERR_FP64
        assert d <= 1e-10


def test_noalloc_in_chunks_full_size(torch_dev, lib):
    """At 60^3 in FP64 one right-hand side needs 5.2 MB of work, so 13 of
    them go through the 64 MiB array in two chunks."""
    s = W.grid3d_cond(nrhs=13)
    e1, e2, d = both_solves(torch_dev, lib, s, "fp64", 13)
    assert e1 <= BERR_FP64 and e2 <= BERR_FP64
    assert d <= 1e-8


def test_noalloc_fp32(torch_dev, lib):
    s = W.laplacian((25, 24, 23), "7pt", 88, 3, unit=False, shift=1e-2, nrhs=5)
    e1, e2, d = both_solves(torch_dev, lib, s, "fp32", 5)
    assert e2 <= 1e-5 and d <= 1e-4
