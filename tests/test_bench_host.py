"""Host checks of bench.py's own pieces (no device): its backward error,
computed with scipy so that the timed paths never call the oracle, equals the
oracle's normwise backward error, and is zero for the exact solution."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2202_09288_amd import workloads as W

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("dims,nrhs", [((9, 7, 11), 3), ((37, 23), 1), ((6, 6, 6), 16)])
def test_bench_backward_error_matches_oracle(dims, nrhs):
    s = W.laplacian(dims, "5pt" if len(dims) == 2 else "7pt", 88, 1, unit=False, shift=1e-2, nrhs=nrhs)
    X = np.random.default_rng(5).standard_normal(s.B.shape)
    a = oracle.backward_error(s.n, s.colptr, s.rowidx, s.values, X, s.B)
    b = bench.host_backward_error(s.n, s.colptr, s.rowidx, s.values, X, s.B)
    assert a > 0 and abs(a - b) <= 1e-14 * a


def test_bench_backward_error_exact_solution():
    s = W.laplacian((8, 8), "5pt", 88, 0, unit=False, shift=1e-2, nrhs=2)
    A = oracle.full_csr(s.n, s.colptr, s.rowidx, s.values).toarray()
    X = np.linalg.solve(A, s.B.reshape(s.n, -1))
    assert bench.host_backward_error(s.n, s.colptr, s.rowidx, s.values, X, s.B) < 1e-15
