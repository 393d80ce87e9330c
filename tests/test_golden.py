"""Stored oracle values (tests/golden/, written by make_golden.py from oracle/ + the input
generator only) still match the oracle, and satisfy the eq. (1) / eq. (9) relation: the
truncated energy lies within the rigorous bound of the direct 250k-pair sum."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ball_pair_seed1.json")


def test_golden_ball_pair_regression(orc, synth):
    g = json.load(open(GOLD))
    w = synth.ball_pair(seed=1)
    assert np.allclose(w["R"], g["R"], rtol=0, atol=1e-13)
    QA = orc.moments(w["xyzA"], w["qA"], w["cA"], 12)
    QB = orc.moments(w["xyzB"], w["qB"], w["cB"], 12)
    for L in (0, 2, 5, 10, 12):
        assert orc.energy(QA, QB, w["R"], L) == pytest.approx(g["tcm"][str(L)], rel=1e-13)
    c = g["coulomb"]
    for L, U in g["tcm"].items():
        assert abs(U - c) <= g["bound"][L]
    assert abs(g["tcm"]["10"] - c) / abs(c) < 1e-8
