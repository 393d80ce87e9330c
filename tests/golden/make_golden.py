"""Write the stored oracle values under tests/golden/.  Calls only oracle/ and the seeded
input generator; nothing here comes from the HIP path.

ball_pair_seed1.json: two balls of 500 charges (radius 10 A, q ~ U[-1, 1]) with centres
60 A apart along a random unit vector (seed 1); the oracle's eq. (9) energy for L = 0..12
about the ball centres, the eq. (1) direct sum over the 250k pairs, the radii and the
rigorous truncation bound for each L.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_0704_1672_amd import synth  # noqa: E402


def ball_pair_seed1():
    w = synth.ball_pair(seed=1)
    QA = oracle.moments(w["xyzA"], w["qA"], w["cA"], 12)
    QB = oracle.moments(w["xyzB"], w["qB"], w["cB"], 12)
    aA, aB = oracle.radius(w["xyzA"], w["cA"]), oracle.radius(w["xyzB"], w["cB"])
    R = float(np.linalg.norm(w["R"]))
    out = dict(
        description="two 500-charge balls, radius 10, q~U[-1,1], centres 60 apart (seed 1)",
        citation="eq. (1) direct sum; eq. (8) moments; eq. (9) square truncation l1,l2<=L",
        R=list(map(float, w["R"])), radiusA=aA, radiusB=aB,
        coulomb=oracle.coulomb(w["xyzA"], w["qA"], w["xyzB"], w["qB"]),
        tcm={str(L): oracle.energy(QA, QB, w["R"], L) for L in range(13)},
        bound={str(L): oracle.trunc_bound(np.abs(w["qA"]).sum(), np.abs(w["qB"]).sum(), aA, aB, R, L)
               for L in range(13)},
    )
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "ball_pair_seed1.json"), "w") as f:
        json.dump(ball_pair_seed1(), f, indent=1)
    print("written")
