"""The weighting-parameter heuristic of Sec. 3.7 (NEXT row f3): the selection
rule on synthetic counts and on the oracle's iteration counts."""
import json
import os

import pytest

from paper_2006_08821_amd.emu import choose_alpha

HERE = os.path.dirname(os.path.abspath(__file__))


def test_rule_takes_the_alpha_before_the_jump():
    a = [1, 10, 100, 1000]
    assert choose_alpha(a, [20, 25, 30, 400], [True] * 4) == (100, 2)
    assert choose_alpha(a, [20, 70, 90, 100], [True] * 4) == (1, 0)        # 70 > 3 x 20
    assert choose_alpha(a, [20, 25, 30, 35], [True] * 4) == (1000, 3)      # no jump: the largest
    assert choose_alpha(a, [20, 25, 30, 35], [True, True, False, True]) == (10, 1)  # failure counts as a jump
    assert choose_alpha(a, [20, 50, 90, 100], [True] * 4, spike=2.0) == (1, 0)
    with pytest.raises(ValueError):
        choose_alpha([], [], [])


def test_rule_on_oracle_counts():
    # oracle EMU counts on the 2x2x8 box beam (tests/golden/make_alpha_trend.py):
    # nearly flat up to alpha_hat = 10, then a jump of more than 10x
    g = json.load(open(os.path.join(HERE, "golden", "alpha_trend_box2x2x8.json")))
    assert g["iters"][0] <= g["iters"][1] < g["iters"][2]
    assert choose_alpha(g["alpha_hats"], g["iters"], g["converged"]) == (10.0, 1)
