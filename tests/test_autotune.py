"""The autotuner's analytic stage: the paper's Algorithm 1 reproduces its
Table 4, and the gfx950 grouping model only proposes compiled variants that
fit the LDS of a compute unit."""
import json
import os

import pytest

from paper_2512_23969_amd import autotune as at

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))


@pytest.mark.parametrize("alpha", [0.51, 0.6, 0.6875])
@pytest.mark.parametrize("name,shape", [("128f", (33, 6, 16)), ("192f", (33, 8, 24))])
def test_algorithm1_reproduces_table4(name, shape, alpha):
    k, log_t, n = shape
    best, cand = at.tree_tuning(k, log_t, n, s_max=48 * 1024, t_max=1024, alpha=alpha)
    want = GOLD["tree_tuning"][name]
    assert best["F"] == want["F"]
    assert best["U_S"] == pytest.approx(want["U_S"])
    assert best["U_T"] == pytest.approx(want["U_T"])
    # every candidate respects the constraints of the algorithm
    for c in cand:
        assert c["U_T"] >= alpha and not (c["U_T"] == 1 and c["U_S"] == 1) and c["U_S"] <= 1


def test_algorithm1_alpha_sensitivity():
    # alpha above 0.6875 excludes the 128f optimum of Table 4
    best, _ = at.tree_tuning(33, 6, 16, 48 * 1024, 1024, 0.7)
    assert best["F"] != 3


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
