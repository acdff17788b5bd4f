"""The autotuner's host side: cache keys and the cache file (no GPU)."""
import json

from paper_2202_09288_amd import spchol, tune
from paper_2202_09288_amd import workloads as W


def test_cache_roundtrip(tmp_path):
    s = W.laplacian((6, 5), "5pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    key = tune.cache_key([s], "fp64", 1)
    assert key == f"fp64:systems=1:n={s.n}:nnz={int(s.colptr[-1])}:nrhs=1"
    path = str(tmp_path / "t.json")
    assert tune.load(key, path) is None
    tune.save(key, {"tuning": {"tiny_w": -1}, "factor_ms": 1.0}, path)
    tune.save("other", {"tuning": {}}, path)
    assert tune.load(key, path) == {"tiny_w": -1}
    assert set(json.load(open(path))) == {key, "other"}


def test_committed_cache_entries_are_valid_options():
    """Every setting in the shipped cache is accepted by spc_analyze."""
    data = json.load(open(tune.CACHE))
    s = W.laplacian((9, 8, 7), "7pt", 88, 0, unit=False, shift=1e-2, nrhs=1)
    for key, entry in data.items():
        assert set(entry["tuning"]) <= set(spchol.TUNING_FIELDS), key
        spchol.Symbolic(s.colptr, s.rowidx, s.perm, 0.05, entry["tuning"])
        # every trial passed or was rejected by the backward-error bar
        assert all("berr" in t for t in entry["trials"])


def test_candidate_groups_start_at_defaults():
    defaults = {"tiny_w": 8, "tiny_m": 64, "small_w": 32, "small_m": 128, "big_min": 256, "big_min_k": 128,
                "solve_persist_max": 1024, "handover": 1, "delay": 1, "persist": -1, "group": 1, "bulk128": -1, "lookahead": -1}
    for _, fields, cands in tune.GROUPS:
        assert tuple(defaults[f] for f in fields) == cands[0]


def test_second_pass_finds_settings_that_pay_together(monkeypatch):
    """Coordinate descent with a second pass: a cost where the deeper bulk
    update pays only once the hand-over rule has changed, which the first
    pass (bulk depth before hand-over) cannot see; no setting is timed
    twice, and a rejected trial (backward error above the bar) never wins."""
    import torch

    def cost(t):
        c = 10.0
        if t.get("handover") == 2:
            c -= 1.0
            if t.get("delay") == 2:
                c -= 3.0
        return c

    def fake_measure(systems, nrhs, tuning, precision, reps, torch_mod):
        if tuning.get("group") == -1:
            return 0.5, 0.0, 1.0  # fastest, but its backward error is rejected
        return cost(tuning), 0.0, 1e-16

    monkeypatch.setattr(tune, "measure", fake_measure)
    monkeypatch.setattr(torch.cuda, "set_device", lambda *_: None)
    res = tune.tune([None], 1, "fp64", log=lambda *_: None)
    assert res["tuning"] == {"handover": 2, "delay": 2}
    assert res["factor_ms"] == 6.0
    keys = [json.dumps(t["tuning"], sort_keys=True) for t in res["trials"]]
    assert len(keys) == len(set(keys))
    assert any(not t["ok"] for t in res["trials"])
