"""The autotuner's analytic stage: the FORS-fusion search of the paper's
Section III-B reproduces its Table 4, and the gfx950 grouping model only
proposes compiled variants that fit the LDS of a compute unit."""
import json
import os

import pytest

from paper_2512_23969_amd import autotune as at

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))


@pytest.mark.parametrize("alpha", [0.51, 0.6, 0.6875])
@pytest.mark.parametrize("name,shape", [("128f", (33, 6, 16)), ("192f", (33, 8, 24))])
def test_fusion_search_reproduces_table4(name, shape, alpha):
    k, log_t, n = shape
    best, cand = at.fors_fusion_search(k, log_t, n, smem_bytes=48 * 1024, max_threads=1024, alpha=alpha)
    want = GOLD["tree_tuning"][name]  # Table 4 prints F, U_S and U_T
    assert best["fusion"] == want["F"]
    assert best["smem_use"] == pytest.approx(want["U_S"])
    assert best["thread_use"] == pytest.approx(want["U_T"])
    # every feasible layout respects the block's limits
    for c in cand:
        assert c["thread_use"] >= alpha and c["smem_use"] <= 1 and c["threads"] <= 1024
        assert not (c["thread_use"] == 1 and c["smem_use"] == 1)


def test_fusion_search_alpha_sensitivity():
    # alpha above 0.6875 excludes the 128f optimum of Table 4
    best, _ = at.fors_fusion_search(33, 6, 16, 48 * 1024, 1024, 0.7)
    assert best["fusion"] != 3


def test_fusion_search_barrier_count():
    # 128f with 11 trees of 64 leaves per block (704 threads) fused 3 times:
    # ceil(33 / 11) / 3 = 1 round of 6 level barriers
    best, _ = at.fors_fusion_search(33, 6, 16, 48 * 1024, 1024, 0.6)
    assert (best["trees"], best["fusion"], best["barriers"]) == (11, 3, 6.0)


@pytest.mark.parametrize("param", [1, 2, 3])
def test_gfx950_groups(param):
    groups = at.gfx950_groups(param)
    assert groups and all(g["fg"] in at.COMPILED_GROUPS[param] for g in groups)
    assert all(g["lds_bytes"] <= 160 * 1024 for g in groups)
    bars = [g["barriers_per_msg"] for g in groups]
    assert bars == sorted(bars)


def test_cache_key_buckets():
    assert at.cache_key("gfx950", 1, 4096) == "gfx950/1/4096"
    assert at.cache_key("gfx950", 2, 3000) == "gfx950/2/4096"
    assert at.cache_key("gfx950", 3, 1) == "gfx950/3/1"


def _table(tmp_path, monkeypatch):
    monkeypatch.setattr(at, "_arch", lambda: "gfx950")
    best = {"mode": "graph-plain", "ms": 13.9, "fors_trees_per_group": 16,
            "by_mode": {"plain": {"mode": "plain", "ms": 14.0, "fors_trees_per_group": 16},
                        "fused": {"mode": "fused", "ms": 14.1, "fors_trees_per_group": 8, "fused_schedule": 2},
                        "graph": {"mode": "graph", "ms": 14.05, "fors_trees_per_group": 8},
                        "graph-plain": {"mode": "graph-plain", "ms": 13.9, "fors_trees_per_group": 16}}}
    f = tmp_path / "tuning.json"
    f.write_text(json.dumps({"gfx950/1/4096": {"best": best}}))
    return str(f)


def test_resolve_mode(tmp_path, monkeypatch):
    """The benchmark's modes: a named mode takes that mode's tuned knobs,
    "auto" the fastest mode, "graph-any" the faster hipGraph pipeline; an
    untuned (set, batch) falls back to the defaults."""
    path = _table(tmp_path, monkeypatch)
    mode, k = at.resolve_mode(1, 4096, "fused", path)
    assert mode == "fused" and k["fors_trees_per_group"] == 8 and k["fused_schedule"] == 2
    assert at.resolve_mode(1, 4096, "auto", path)[0] == "graph-plain"
    mode, k = at.resolve_mode(1, 3000, "graph-any", path)  # the 4096 bucket
    assert mode == "graph-plain" and k["ms"] == 13.9
    assert at.resolve_mode(2, 4096, "auto", path) == ("plain", None)
    assert at.resolve_mode(2, 4096, "graph-any", path) == ("graph", None)


def test_apply_sets_every_knob(tmp_path, monkeypatch):
    """apply() passes every slh_tuning knob, tuned or default, to the context."""
    path = _table(tmp_path, monkeypatch)
    got = {}

    class Ctx:
        def set_tuning(self, param, **knobs):
            got.update(knobs, param=param)

    _, k = at.resolve_mode(1, 4096, "fused", path)
    assert at.apply(Ctx(), 1, k) == "fused"
    assert set(got) == set(at.KNOB_DEFAULTS) | {"param"}
    assert got["fors_trees_per_group"] == 8 and got["fused_schedule"] == 2 and got["keep_chains"] == 1
    from paper_2512_23969_amd import slh
    assert set(at.KNOB_DEFAULTS) == set(slh.TUNING_FIELDS)
