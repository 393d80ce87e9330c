"""Adaptive truncation (tcm_batch_energy_adaptive): per pair, the smallest order whose
rigorous truncation bound meets the tolerance.  Checked against the direct Coulomb sum of
eq. (1) (the error is within the tolerance), against the oracle's bound (the order is the
smallest that meets it), against the fixed-order batch path at the chosen order (bit for
bit) and on the error cases."""
import numpy as np
import pytest

from paper_0704_1672_amd import tcm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tcm.Context(0)
    yield c.h
    c.close()


@pytest.mark.parametrize("tol_rel", [1e-2, 1e-4, 1e-7])
def test_adaptive_meets_tolerance_with_smallest_order(ctx, orc, synth, tol_rel):
    w = synth.ball_pair(seed=1)
    xA, qA, xB, qB, cA, cB = w["xyzA"], w["qA"], w["xyzB"], w["qB"], w["cA"], w["cB"]
    mA = tcm.tcm_mol_upload(ctx, xA, qA, centre=cA, precision=tcm.TCM_F64)
    mB = tcm.tcm_mol_upload(ctx, xB - cB, qB, centre=np.zeros(3), precision=tcm.TCM_F64)
    try:
        aA, aB = orc.radius(xA, cA), orc.radius(xB, cB)
        SA, SB = np.sum(np.abs(qA)), np.sum(np.abs(qB))
        u = (cB - cA) / np.linalg.norm(cB - cA)
        dists = np.array([1.3, 1.8, 2.5, 4.0, 8.0]) * (aA + aB)
        R = dists[:, None] * u[None, :]
        Lmax = 24
        # the tolerance relative to the charge scale S_A S_B / R at the closest distance
        tol = tol_rel * SA * SB / dists[0]
        U, Lu, bnd, st, rc = tcm.tcm_batch_energy_adaptive(ctx, tcm.make_requests(mA, mB, R, Lmax), tol)
        assert rc == 0 and np.all(st == 0)
        for k in range(len(dists)):
            L = int(Lu[k])
            want_b = orc.trunc_bound(SA, SB, aA, aB, dists[k], L)
            assert abs(bnd[k] - want_b) <= 1e-12 * want_b
            if L < Lmax:
                assert bnd[k] <= tol
            if L > 0:
                assert orc.trunc_bound(SA, SB, aA, aB, dists[k], L - 1) > tol
            # the truncation error against eq. (1) is within the bound
            Uc = orc.coulomb(xA, qA, xB - cB + R[k] + cA, qB)
            assert abs(U[k] - Uc) <= bnd[k] * (1 + 1e-9) + 1e-12 * SA * SB / dists[k]
            # the same contraction as the fixed-order path at that order
            Uf, stf, _ = tcm.tcm_batch_energy(ctx, tcm.make_requests(mA, mB, R[k], L, flags=tcm.TCM_REUSE))
            assert stf[0] == 0 and Uf[0] == U[k]
        assert np.all(np.diff(Lu) <= 0)            # farther pairs need no higher order
    finally:
        tcm.tcm_mol_release(ctx, mA)
        tcm.tcm_mol_release(ctx, mB)


def test_adaptive_errors_and_limits(ctx, synth):
    xa, qa, _ = synth.chain(17, 1, 800)
    mA = tcm.tcm_mol_upload(ctx, xa, qa)
    try:
        R = np.array([[2.0, 0, 0], [400.0, 0, 0], [0, 0, 0]])
        req = tcm.make_requests(mA, mA, R, 6)
        U, Lu, b, st, rc = tcm.tcm_batch_energy_adaptive(ctx, req, 1e-30)
        assert st[0] == tcm.TCM_EDOMAIN and Lu[0] == -1 and np.isnan(U[0])
        assert st[1] == 0 and Lu[1] == 6 and b[1] > 1e-30          # tolerance out of reach: L = max
        assert st[2] == tcm.TCM_EINVAL
        U, Lu, b, st, rc = tcm.tcm_batch_energy_adaptive(ctx, req[1:2], 1e30)
        assert st[0] == 0 and Lu[0] == 0
        with pytest.raises(tcm.TCMError):
            tcm.tcm_batch_energy_adaptive(ctx, req, 0.0)
        U, Lu, b, st, rc = tcm.tcm_batch_energy_adaptive(ctx, tcm.make_requests([987654], mA, R[1], 6), 1.0)
        assert st[0] == tcm.TCM_ENOTFOUND
    finally:
        tcm.tcm_mol_release(ctx, mA)
