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


def _adaptive_requests(synth, a, b, n, seed):
    rng = np.random.default_rng(seed)
    R = rng.normal(size=(n, 3))
    R *= (rng.uniform(12.0, 40.0, n) / np.linalg.norm(R, axis=1))[:, None]
    flags = np.where(rng.random(n) < 0.3, tcm.TCM_TRIANGULAR, 0)
    return tcm.make_requests(a, b, R, 16, synth.quaternions(seed, 0, n), flags=flags)


@pytest.mark.parametrize("use_graph", [True, False])
def test_adaptive_plan_equals_adaptive_call(ctx, synth, use_graph):
    """An adaptive plan, run and replayed (graph, direct, phased, timed), gives the one-shot
    adaptive call's energies, orders, bounds and statuses bit for bit."""
    xa, qa = synth.ball(101, 0, 400, 4.0)
    xb, qb = synth.ball(102, 0, 300, 3.5)
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    b = tcm.tcm_mol_upload(ctx, xb, qb, precision=tcm.TCM_F64)
    pl = None
    try:
        n = 300
        req = _adaptive_requests(synth, a, b, n, 103)
        tol = 1e-6 * np.sum(np.abs(qa)) * np.sum(np.abs(qb)) / 20.0
        U1, L1, b1, st1, rc = tcm.tcm_batch_energy_adaptive(ctx, req, tol)
        assert rc == tcm.TCM_OK and np.all(st1 == 0)
        assert L1.min() < L1.max() <= 16                      # the orders differ from pair to pair
        pl = tcm.tcm_plan_create_adaptive(ctx, req, tol, use_graph=use_graph)
        runs = [lambda: tcm.tcm_plan_run(ctx, pl), lambda: tcm.tcm_plan_run(ctx, pl),
                lambda: tcm.tcm_plan_run_phased(ctx, pl), lambda: tcm.tcm_plan_run_timed(ctx, pl)]
        for run in runs:
            run()
            U, st = tcm.tcm_plan_results(ctx, pl, n)
            Lc, bc = tcm.tcm_plan_orders(ctx, pl, n)
            assert np.array_equal(U, U1) and np.array_equal(st, st1)
            assert np.array_equal(Lc, L1) and np.array_equal(bc, b1)
    finally:
        if pl is not None:
            tcm.tcm_plan_destroy(pl)
        tcm.tcm_mol_release(ctx, a)
        tcm.tcm_mol_release(ctx, b)


def test_adaptive_plan_replay_chooses_again(ctx, synth):
    """A replay chooses every pair's order again from the requested one: after the atoms of B
    (device memory the plan reads) move apart by 30%, the bounds grow and orders rise, and the
    replay equals a fresh adaptive call on the moved atoms bit for bit."""
    import torch
    xa, qa = synth.ball(111, 0, 400, 4.0)
    xb, qb = synth.ball(112, 0, 300, 3.5)
    t = torch.tensor(np.vstack([xb.T, qb[None, :]]), dtype=torch.float64, device="cuda").contiguous()
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    b = tcm.tcm_mol_register_device(ctx, t[0], t[1], t[2], t[3], len(qb), precision=tcm.TCM_F64)
    pl = None
    try:
        n = 200
        req = _adaptive_requests(synth, a, b, n, 113)
        tol = 1e-6 * np.sum(np.abs(qa)) * np.sum(np.abs(qb)) / 20.0
        pl = tcm.tcm_plan_create_adaptive(ctx, req, tol)
        tcm.tcm_plan_run(ctx, pl)
        L0, _ = tcm.tcm_plan_orders(ctx, pl, n)
        torch.cuda.synchronize()
        t[0:3] *= 1.3
        torch.cuda.synchronize()
        tcm.tcm_plan_run(ctx, pl)
        U, st = tcm.tcm_plan_results(ctx, pl, n)
        Lc, bc = tcm.tcm_plan_orders(ctx, pl, n)
        U1, L1, b1, st1, rc = tcm.tcm_batch_energy_adaptive(ctx, req, tol)
        assert rc == tcm.TCM_OK and np.all(st1 == 0)
        assert np.any(L1 > L0)                                # some orders had to rise
        assert np.array_equal(Lc, L1) and np.array_equal(bc, b1)
        assert np.array_equal(U, U1) and np.array_equal(st, st1)
    finally:
        if pl is not None:
            tcm.tcm_plan_destroy(pl)
        tcm.tcm_mol_release(ctx, a)
        tcm.tcm_mol_release(ctx, b)
        torch.cuda.synchronize()


def test_plan_orders_rejects_fixed_plans(ctx, synth):
    xa, qa = synth.ball(121, 0, 100, 3.0)
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    pl = None
    try:
        pl = tcm.tcm_plan_create(ctx, tcm.make_requests(a, a, [20.0, 0.0, 0.0], 8))
        with pytest.raises(tcm.TCMError):
            tcm.tcm_plan_orders(ctx, pl, 1)
        with pytest.raises(tcm.TCMError):
            tcm.tcm_plan_create_adaptive(ctx, tcm.make_requests(a, a, [20.0, 0.0, 0.0], 8), 0.0)
    finally:
        if pl is not None:
            tcm.tcm_plan_destroy(pl)
        tcm.tcm_mol_release(ctx, a)
