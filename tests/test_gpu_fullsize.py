"""Parity at the full workload sizes, in the launch configuration the benchmark uses, on
sampled outputs the oracle computes one by one, plus properties that hold at any size.

chain pair       two 100k-bead chains, L in {8, 16, 24}, 16 separations 2..10 x Rg
                 (the close ones violate eq. 2 and must return TCM_EDOMAIN), FP64 and FP32C
orientation scan two 50k-charge balls, 4096 poses of B in one graph launch, L = 16 (FP32C
                 moments, FP64 rotation and contraction); sampled poses vs the oracle
                 recomputing B's moments from rotated atoms
uneven batch     1024 chain pairs (77M atoms), L in {8, 12, 16, 20}, autotuned tiles, graph
                 replay; sampled pairs vs the oracle; one pair alone vs in the batch, bitwise
"""
import numpy as np
import pytest

from paper_0704_1672_amd import tcm

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10      # |dU| / sum|terms|; FP64 results must also be within 1e-6 of U itself
TOL_F32 = 1e-5       # |dU| / sum|terms| for FP32-compensated moments


@pytest.fixture(scope="module")
def ctx():
    c = tcm.Context(0)
    yield c.h
    c.close()


def test_chain_pair_all_orders_and_separations(ctx, orc, synth):
    w = synth.chain_pair(seed=2, n=100_000)
    xA, qA, xB, qB = w["xyzA"], w["qA"], w["xyzB_body"], w["qB"]
    cA, cB = orc.centroid(xA), orc.centroid(xB)
    aA, aB = orc.radius(xA, cA), orc.radius(xB, cB)
    QA, QB = orc.moments(xA, qA, cA, 24), orc.moments(xB, qB, cB, 24)
    # B sits at xyzB_body + sep: the vector between the two centres is sep + cB - cA
    Rs = [np.asarray(sep) + (cB - cA) for sep in w["seps"]]
    want = {(L, k): orc.energy(QA, QB, Rs[k], L, full=True) for L in w["Ls"] for k in range(len(Rs))}
    n_out = 0
    for prec, tol in ((tcm.TCM_F64, TOL_F64), (tcm.TCM_F32C, TOL_F32)):
        mA = tcm.tcm_mol_upload(ctx, xA, qA, precision=prec)
        mB = tcm.tcm_mol_upload(ctx, xB, qB, precision=prec)
        try:
            for L in w["Ls"]:
                req = tcm.make_requests(mA, mB, np.array(Rs), L)
                U, st, _ = tcm.tcm_batch_energy(ctx, req)
                for k, R in enumerate(Rs):
                    if not np.linalg.norm(R) > aA + aB:     # eq. 2 violated
                        assert st[k] == tcm.TCM_EDOMAIN and np.isnan(U[k])
                        n_out += 1
                        continue
                    assert st[k] == tcm.TCM_OK
                    d = want[(L, k)]
                    assert abs(U[k] - d["U"]) <= tol * d["abs_sum"], (prec, L, k, U[k], d["U"])
                    if prec == tcm.TCM_F64:
                        assert abs(U[k] - d["U"]) <= 1e-6 * abs(d["U"]), (L, k, U[k], d["U"])
        finally:
            tcm.tcm_mol_release(ctx, mA)
            tcm.tcm_mol_release(ctx, mB)
    assert n_out > 0            # the closest separations fall inside a_A + a_B


def test_orientation_scan_4096_poses(ctx, orc, synth):
    w = synth.orientation_scan(seed=3)
    L = w["L"]
    mA = tcm.tcm_mol_upload(ctx, w["xyzA"], w["qA"], centre=w["cA"], precision=tcm.TCM_F32C)
    mB = tcm.tcm_mol_upload(ctx, w["xyzB"], w["qB"], centre=w["cB"], precision=tcm.TCM_F32C)
    try:
        req = tcm.make_requests(mA, mB, w["R"], L, w["quats"])
        plan = tcm.tcm_plan_create(ctx, req, use_graph=True)
        try:
            tcm.tcm_plan_run(ctx, plan)
            U, st = tcm.tcm_plan_results(ctx, plan, len(req))
            assert np.all(st == 0) and np.all(np.isfinite(U))
            tcm.tcm_plan_run(ctx, plan)
            U2, _ = tcm.tcm_plan_results(ctx, plan, len(req))
            assert np.array_equal(U, U2)
        finally:
            tcm.tcm_plan_destroy(plan)
        QA = orc.moments(w["xyzA"], w["qA"], w["cA"], L)
        for p in np.linspace(0, len(req) - 1, 10).astype(int):
            xBr = orc.pose(w["xyzB"], w["cB"], w["quats"][p], w["cB"])
            d = orc.energy(QA, orc.moments(xBr, w["qB"], w["cB"], L), w["R"][p], L, full=True)
            assert abs(U[p] - d["U"]) <= TOL_F32 * d["abs_sum"], (p, U[p], d["U"])
    finally:
        tcm.tcm_mol_release(ctx, mA)
        tcm.tcm_mol_release(ctx, mB)


def test_uneven_batch_full_size(ctx, orc, synth):
    import torch
    w = synth.uneven_batch(seed=4, npairs=1024)
    ntot = int(w["offsets"][-1])
    soa = torch.empty((4, ntot), dtype=torch.float64, device="cuda")
    soa[0:3] = torch.from_numpy(np.ascontiguousarray(w["xyz"].T)).cuda()
    soa[3] = torch.from_numpy(w["q"]).cuda()
    torch.cuda.synchronize()
    base, row = soa.data_ptr(), ntot * 8
    ids = []
    for f in range(2048):
        off = int(w["offsets"][f]) * 8
        ids.append(tcm.tcm_mol_register_device(ctx, base + off, base + row + off, base + 2 * row + off,
                                               base + 3 * row + off, int(w["counts"][f])))
    try:
        req = tcm.make_requests(ids[0::2], ids[1::2], w["R"], w["L"], w["quats"])
        assert tcm.tcm_autotune_batch(ctx, req) > 0      # the benchmark's launch configuration
        plan = tcm.tcm_plan_create(ctx, req, use_graph=True)
        try:
            tcm.tcm_plan_run(ctx, plan)
            U, st = tcm.tcm_plan_results(ctx, plan, 1024)
        finally:
            tcm.tcm_plan_destroy(plan)
        assert np.all(st == 0) and np.all(np.isfinite(U))
        # one pair alone (its own launch) equals its value in the full batch, bit for bit
        p0 = int(np.argmax(w["counts"][0::2]))
        Ualone, st0, _ = tcm.tcm_batch_energy(ctx, req[p0:p0 + 1])
        assert st0[0] == 0 and Ualone[0] == U[p0]
        # sampled pairs vs the oracle (smallest pairs of each order)
        for L in (8, 12, 16, 20):
            cand = np.nonzero(w["L"] == L)[0]
            p = cand[np.argmin(w["counts"][2 * cand] + w["counts"][2 * cand + 1])]
            a, b = 2 * p, 2 * p + 1
            xa = w["xyz"][w["offsets"][a]:w["offsets"][a + 1]]
            qa = w["q"][w["offsets"][a]:w["offsets"][a + 1]]
            xb = w["xyz"][w["offsets"][b]:w["offsets"][b + 1]]
            qb = w["q"][w["offsets"][b]:w["offsets"][b + 1]]
            cA, cB = orc.centroid(xa), orc.centroid(xb)
            d = orc.energy(orc.moments(xa, qa, cA, L), orc.moments(orc.pose(xb, cB, w["quats"][p], cB), qb, cB, L),
                           w["R"][p], L, full=True)
            assert abs(U[p] - d["U"]) <= TOL_F32 * d["abs_sum"], (L, p, U[p], d["U"])
    finally:
        for i in ids:
            tcm.tcm_mol_release(ctx, i)
        del soa
        torch.cuda.empty_cache()


def test_very_large_molecule_capped_statistics_items(ctx, orc, synth):
    """17M charges: more chunks than the planner's statistics-item cap, so each item covers a
    run of chunks.  Centre (centroid), radius and the FP64 moments at L = 4 against the oracle
    and the direct definitions."""
    n = 17_000_000
    x, q = synth.ball(91, 1, n, 5000.0)
    mid = tcm.tcm_mol_upload(ctx, x, q, precision=tcm.TCM_F64)
    try:
        Q, radius, centre = tcm.tcm_mol_moments(ctx, mid, 4)
        c = orc.centroid(x)
        assert np.allclose(centre, c, rtol=0, atol=1e-9 * 5000.0), (centre, c)
        assert abs(radius - orc.radius(x, centre)) <= 1e-12 * radius
        Qo = orc.complex_to_packed(orc.moments(x, q, centre, 4))
        _, qa = orc.moments(x, q, centre, 4, with_abs=True)
        scale = np.max(qa)
        assert np.max(np.abs(Q - Qo)) <= 1e-10 * scale, np.max(np.abs(Q - Qo)) / scale
    finally:
        tcm.tcm_mol_release(ctx, mid)
