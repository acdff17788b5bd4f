"""Host checks of the seeded workloads and the serving request mix."""
import numpy as np

from paper_2202_09288_amd import workloads as W


def test_splitmix64_reference_values():
    # SplitMix64 from state 0: published first outputs of the generator
    out = W.splitmix64(0, 3)
    assert [hex(int(x)) for x in out] == ["0xe220a8397b1dcdaf", "0x6e789e6aa1b965f4", "0x6c45d188009454f"]


def test_uniform_range_and_determinism():
    a = W.uniform(W.stream_key(1, 0, W.P_RHS), 1000)
    b = W.uniform(W.stream_key(1, 0, W.P_RHS), 1000)
    c = W.uniform(W.stream_key(1, 1, W.P_RHS), 1000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() < 1.0


def test_nd_perm_is_permutation_and_separator_last():
    for dims in [(5,), (7, 4), (6, 5, 3)]:
        p = W.nd_perm(dims)
        assert np.array_equal(np.sort(p), np.arange(int(np.prod(dims))))
    # 2D: the first separator (the middle column of the longest axis) comes last
    p = W.nd_perm((9, 4))
    last = p[-4:]
    assert sorted(last.tolist()) == sorted([4 + 9 * y for y in range(4)])


def test_grid3d_60_sizes():
    s = W.grid3d_cond(k=6)
    assert s.n == 216 and s.nnz == 216 + 3 * 6 * 6 * 5
    A = np.zeros((s.n, s.n))
    c = np.repeat(np.arange(s.n), np.diff(s.colptr))
    A[s.rowidx, c] = s.values
    A = A + np.tril(A, -1).T
    off = np.abs(A).sum(1) - np.abs(np.diag(A))
    assert np.allclose(np.diag(A) - off, 1e-6, rtol=0, atol=1e-9)
    offd = -A[np.tril_indices(s.n, -1)]
    offd = offd[offd != 0]
    assert offd.min() >= 1e-2 and offd.max() < 1e2


def test_batch_mix_sizes():
    specs = W.batch_specs(512, 0)
    sides2 = [sd for k, sd in specs if k == "2d"]
    sides3 = [sd for k, sd in specs if k == "3d"]
    assert min(sides2) >= 32 and max(sides2) <= 200 and min(sides3) >= 10 and max(sides3) <= 34
    assert 200 < len(sides2) < 312
    ns = [sd * sd if k == "2d" else sd ** 3 for k, sd in specs]
    assert min(ns) >= 1000 and max(ns) <= 40000


def test_serving_mix():
    reqs = W.serving_requests(2000, 10.0, 0)
    kinds = [r["kind"] for r in reqs]
    frac_resolve = kinds.count("resolve") / len(kinds)
    assert 0.25 < frac_resolve < 0.35
    big = sum(1 for r in reqs if r["kind"] == "factor" and r["sys"] == ("3d", 50))
    assert 0.02 < big / kinds.count("factor") < 0.08
    t = np.array([r["t"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 10.0) < 1.0


def test_serving_requests_target_earlier_factors():
    from paper_2202_09288_amd import serving as SV
    reqs = SV.make_requests(60, 5.0, 1, system_fn=lambda k, s: W.laplacian(
        (s, s) if k == "2d" else (s, s, s), "5pt" if k == "2d" else "7pt", 5, 0, unit=False, shift=1e-2, nrhs=8),
        max_side={"2d": 12, "3d": 5})
    seen = set()
    for r in reqs:
        if r.kind == "factor":
            seen.add(r.rid)
        else:
            assert r.target in seen
