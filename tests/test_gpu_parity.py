"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances
  FP64 moment pass:  |dQ_h| <= 1e-12 * A_h, A_h = sum_i |q_i| |C_lm(r_i)| (oracle's absolute sums)
  FP32C moment pass: |dQ_h| <= (8 (l+1) + 2 kper + 64) 2^-24 A_h  -- input rounding of the scaled
                     coordinates and charges (~(l+1) u), the recurrence (~(l+1) u), the plain
                     per-thread run over kper atoms (kper u), the compensated merges (~u)
  pair energy (FP64): |dU| <= 1e-12 * sum |terms| (oracle's abs_sum); with a pose 1e-11
  end to end at FP64: relative 1e-6 (the stated target; observed ~1e-13)
"""
import math

import numpy as np
import pytest

from paper_0704_1672_amd import tcm

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    c = tcm.Context(0)
    yield c.h
    c.close()


def packed_abs(orc, Qabs, L):
    out = np.zeros((L + 1) ** 2)
    for l in range(L + 1):
        out[l * l] = Qabs[l * l + l]
        for m in range(1, l + 1):
            out[l * l + 2 * m - 1] = out[l * l + 2 * m] = Qabs[l * l + l + m]
    return out


def l_of_packed(L):
    return np.concatenate([[l] * (2 * l + 1) for l in range(L + 1)])


def oracle_packed(orc, xyz, q, c, L):
    Q, A = orc.moments(xyz, q, c, L, with_abs=True)
    return orc.complex_to_packed(Q, L), packed_abs(orc, A, L)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 8, 10, 13, 16, 21, 24, 27, 32])
def test_moments_f64_and_f32c_match_oracle(ctx, orc, synth, L):
    n = 5000                                   # 5 tiles of 1024 atoms, ragged last tile
    c0 = np.array([3.0, -2.0, 1.5])
    xyz, q = synth.ball(11, L, n, 10.0, c0)
    ref, A = oracle_packed(orc, xyz, q, c0, L)
    ls = l_of_packed(L)
    for prec in (tcm.TCM_F64, tcm.TCM_F32C):
        tcm.tcm_tune_set(ctx, prec, L, n, 4)
        Q, rad, cen = tcm.tcm_moments(ctx, xyz, q, L, prec, centre=c0)
        err = np.abs(Q - ref)
        if prec == tcm.TCM_F64:
            tol = 1e-12 * A + 1e-300
        else:
            tol = (8 * (ls + 1) + 2 * 4 + 64) * U32 * A + 1e-300
        bad = np.nonzero(err > tol)[0]
        assert len(bad) == 0, (prec, L, bad[:5], err[bad[:5]], tol[bad[:5]])
        assert rad == pytest.approx(orc.radius(xyz, c0), rel=1e-14)
        assert np.all(cen == c0)


@pytest.mark.parametrize("prec", [tcm.TCM_F64, tcm.TCM_F32C])
def test_moments_default_centroid_and_tiling(ctx, orc, synth, prec):
    """Centroid centre (device reduction) and the default tile choice on a zero-net-charge
    chain of 60k beads (several statistics chunks and tiles)."""
    xyz, q, _ = synth.chain(7, 1, 60_000)
    xyz = xyz + np.array([100.0, -50.0, 20.0])
    L = 12
    Q, rad, cen = tcm.tcm_moments(ctx, xyz, q, L, prec)
    c_ref = orc.centroid(xyz)
    assert np.max(np.abs(cen - c_ref)) < 1e-11
    ref, A = oracle_packed(orc, xyz, q, c_ref, L)
    ls = l_of_packed(L)
    kper = tcm.tcm_tune_get(ctx, prec, L, len(q))
    # the centre differs from the oracle's by rounding (~1e-13 A); its effect on Q_l is
    # bounded by l |dc| / a relative to A
    dc = np.max(np.abs(cen - c_ref)) * (ls + 1) / rad
    tol = (1e-12 + dc) * A if prec == tcm.TCM_F64 else ((8 * (ls + 1) + 2 * kper + 64) * U32 + dc) * A
    err = np.abs(Q - ref)
    assert np.all(err <= tol + 1e-300), (np.max(err / (tol + 1e-300)))
    assert rad == pytest.approx(orc.radius(xyz, cen), rel=1e-13)


def test_moments_edge_cases(ctx, orc):
    for prec in (tcm.TCM_F64, tcm.TCM_F32C):
        # empty molecule: zero moments, radius 0, given centre
        Q, rad, cen = tcm.tcm_moments(ctx, np.zeros((0, 3)), np.zeros(0), 6, prec, centre=[1, 2, 3])
        assert np.all(Q == 0) and rad == 0 and np.all(cen == [1, 2, 3])
        # empty molecule without centre: origin
        Q, rad, cen = tcm.tcm_moments(ctx, np.zeros((0, 3)), np.zeros(0), 2, prec)
        assert np.all(Q == 0) and np.all(cen == 0)
        # single atom at the centre: Q_00 = q only
        Q, rad, cen = tcm.tcm_moments(ctx, [[1.0, 2.0, 3.0]], [0.7], 10, prec)
        assert Q[0] == pytest.approx(0.7, rel=1e-7) and np.all(Q[1:] == 0) and rad == 0
        # single atom off the centre, along z: Q_l0 = q h^l
        Q, rad, cen = tcm.tcm_moments(ctx, [[0.0, 0.0, 2.0]], [0.5], 8, prec, centre=[0, 0, 0])
        for l in range(9):
            assert Q[l * l] == pytest.approx(0.5 * 2.0 ** l, rel=1e-12 if prec == 0 else 1e-6)
        # L = 0 is the total charge
        Q, _, _ = tcm.tcm_moments(ctx, np.random.default_rng(1).normal(size=(100, 3)), np.ones(100), 0, prec)
        assert Q[0] == pytest.approx(100.0, rel=1e-12)


def test_moments_rejects_bad_arguments(ctx):
    with pytest.raises(tcm.TCMError) as e:
        tcm.tcm_moments(ctx, [[0, 0, 1.0]], [1.0], 33, tcm.TCM_F64)
    assert e.value.code == tcm.TCM_EINVAL
    with pytest.raises(tcm.TCMError):
        tcm.tcm_moments(ctx, [[0, 0, np.nan]], [1.0], 3, tcm.TCM_F64)
    with pytest.raises(tcm.TCMError):
        tcm.tcm_moments(ctx, [[0, 0, 1.0]], [1.0], 3, 7)


def _two_balls(synth, seed, nA=300, nB=250, t=0.5):
    u = synth.unit_vectors(seed, 0, 1)[0]
    aA, aB = 3.0, 4.0
    R = (aA + aB) / t * u
    xA, qA = synth.ball(seed, 1, nA, aA)
    xB, qB = synth.ball(seed, 2, nB, aB, R)
    return xA, qA, np.zeros(3), xB, qB, R


@pytest.mark.parametrize("L", [0, 1, 2, 5, 10, 16, 24, 32])
def test_pair_energy_matches_oracle(ctx, orc, synth, L):
    xA, qA, cA, xB, qB, cB = _two_balls(synth, 20 + L, t=0.45)
    QA = orc.moments(xA, qA, cA, L)
    QB = orc.moments(xB, qB, cB, L)
    d = orc.energy(QA, QB, cB - cA, L, full=True)
    aA, aB = orc.radius(xA, cA), orc.radius(xB, cB)
    U = tcm.tcm_pair_energy(ctx, orc.complex_to_packed(QA), aA, orc.complex_to_packed(QB), aB, cB - cA, L)
    assert abs(U - d["U"]) <= 1e-12 * d["abs_sum"], (L, U, d["U"], d["abs_sum"])


def test_pair_energy_along_axis(ctx, orc, synth):
    xA, qA, cA, xB, qB, cB = _two_balls(synth, 5, t=0.4)
    R = np.linalg.norm(cB - cA)
    for sgn in (1, -1):
        Rv = np.array([0.0, 0.0, sgn * R])
        QA, QB = orc.moments(xA, qA, cA, 12), orc.moments(xB - cB, qB, np.zeros(3), 12)
        d = orc.energy(QA, QB, Rv, 12, full=True)
        U = tcm.tcm_pair_energy(ctx, orc.complex_to_packed(QA), 3.0, orc.complex_to_packed(QB), 4.0, Rv, 12)
        assert abs(U - d["U"]) <= 1e-12 * d["abs_sum"]


@pytest.mark.parametrize("L", [1, 4, 10, 16, 24, 32])
def test_pair_energy_pose_matches_recomputed_moments(ctx, orc, synth, L):
    """Rotation of B's moments (a3) vs the oracle recomputing eq. (8) from rotated atoms."""
    xA, qA, cA, xB, qB, cB = _two_balls(synth, 40 + L, t=0.45)
    quats = synth.quaternions(40 + L, 9, 3)
    QA = orc.moments(xA, qA, cA, L)
    QB = orc.moments(xB, qB, cB, L)
    pA, pB = orc.complex_to_packed(QA), orc.complex_to_packed(QB)
    for qv in list(quats) + [np.array([1.0, 0, 0, 0]), np.array([0.0, 0, 0, 1.0]), np.array([0.0, 1.0, 0, 0])]:
        xBr = orc.pose(xB, cB, qv, cB)
        d = orc.energy(QA, orc.moments(xBr, qB, cB, L), cB - cA, L, full=True)
        U = tcm.tcm_pair_energy(ctx, pA, 3.0, pB, 4.0, cB - cA, L, quat_b=qv)
        assert abs(U - d["U"]) <= 1e-11 * d["abs_sum"], (L, qv, U, d["U"])


@pytest.mark.parametrize("L", [8, 16])
def test_pair_energy_degenerate_euler_poses(ctx, orc, synth, L):
    """R along +-z (the frame rotation is the identity, so B's rotation is its pose exactly)
    with poses whose Euler decomposition is degenerate: half turns about axes in the xy-plane
    (w = z = 0) and rotations about z (x = y = 0), against the oracle's rotated atoms."""
    xA, qA, cA, xB, qB, cB = _two_balls(synth, 60 + L, t=0.45)
    R = np.linalg.norm(cB - cA)
    QA = orc.moments(xA, qA, cA, L)
    pA = orc.complex_to_packed(QA)
    pB = orc.complex_to_packed(orc.moments(xB, qB, cB, L))
    poses = [[0.0, 1.0, 0, 0], [0.0, 0, 1.0, 0], [0.0, 0.6, 0.8, 0], [0.0, -0.8, 0.6, 0],
             [1.0, 0, 0, 0], [0.0, 0, 0, 1.0], [0.8, 0, 0, -0.6]]
    for sgn in (1, -1):
        Rv = np.array([0.0, 0.0, sgn * R])
        for qv in map(np.array, poses):
            xBr = orc.pose(xB, cB, qv, cB)
            d = orc.energy(QA, orc.moments(xBr, qB, cB, L), Rv, L, full=True)
            U = tcm.tcm_pair_energy(ctx, pA, 3.0, pB, 4.0, Rv, L, quat_b=qv)
            assert abs(U - d["U"]) <= 1e-11 * d["abs_sum"], (L, sgn, qv, U, d["U"])


def test_domain_and_flags(ctx, orc, synth):
    xA, qA, cA, xB, qB, cB = _two_balls(synth, 3, t=0.5)
    L = 6
    pA = orc.complex_to_packed(orc.moments(xA, qA, cA, L))
    pB = orc.complex_to_packed(orc.moments(xB, qB, cB, L))
    R = cB - cA
    Rn = np.linalg.norm(R)
    with pytest.raises(tcm.TCMError) as e:
        tcm.tcm_pair_energy(ctx, pA, Rn / 2, pB, Rn / 2 + 1e-9, R, L)
    assert e.value.code == tcm.TCM_EDOMAIN
    with pytest.raises(tcm.TCMError) as e:                 # equality is outside the domain (strict)
        tcm.tcm_pair_energy(ctx, pA, Rn / 2, pB, Rn / 2, R, L)
    assert e.value.code == tcm.TCM_EDOMAIN
    U = tcm.tcm_pair_energy(ctx, pA, Rn, pB, Rn, R, L, flags=tcm.TCM_UNCHECKED)
    assert U == pytest.approx(orc.energy(orc.packed_to_complex(pA), orc.packed_to_complex(pB), R, L), rel=1e-12)
    for bad in (dict(R=[0.0, 0.0, 0.0]), dict(quat_b=[0, 0, 0, 0])):
        with pytest.raises(tcm.TCMError):
            tcm.tcm_pair_energy(ctx, pA, 1, pB, 1, bad.get("R", R), L, quat_b=bad.get("quat_b"))
    big = np.zeros(34 * 34)
    with pytest.raises(tcm.TCMError) as e:
        tcm.tcm_pair_energy(ctx, big, 1, big, 1, R, 33)
    assert e.value.code == tcm.TCM_EINVAL


def test_ball_pair_end_to_end_fp64(ctx, orc, synth):
    """Two 500-charge balls 60 A apart, L = 10: GPU moments and contraction vs the oracle's
    eq. (9) energy (stated bound 1e-6 relative; FP64 reaches ~1e-13), and the oracle's own
    truncation error vs the 250k-pair direct sum."""
    w = synth.ball_pair(seed=1)
    L = w["L"]
    QA, aA, _ = tcm.tcm_moments(ctx, w["xyzA"], w["qA"], L, tcm.TCM_F64, centre=w["cA"])
    QB, aB, _ = tcm.tcm_moments(ctx, w["xyzB"], w["qB"], L, tcm.TCM_F64, centre=w["cB"])
    U = tcm.tcm_pair_energy(ctx, QA, aA, QB, aB, w["R"], L)
    Uo = orc.pair_energy_from_atoms(w["xyzA"], w["qA"], w["cA"], w["xyzB"], w["qB"], w["cB"], L)
    assert abs(U - Uo) / abs(Uo) < 1e-12
    Uc = orc.coulomb(w["xyzA"], w["qA"], w["xyzB"], w["qB"])
    assert abs(U - Uc) <= orc.trunc_bound(np.abs(w["qA"]).sum(), np.abs(w["qB"]).sum(), aA, aB,
                                          np.linalg.norm(w["R"]), L)


def _upload_set(ctx, synth):
    mols = []
    specs = [("ball", 900, tcm.TCM_F64), ("chain", 20_000, tcm.TCM_F32C), ("ball", 3000, tcm.TCM_F32C),
             ("chain", 7_000, tcm.TCM_F64), ("ball", 1, tcm.TCM_F32C), ("chain", 41_000, tcm.TCM_F32C)]
    for i, (kind, n, prec) in enumerate(specs):
        if kind == "ball":
            xyz, q = synth.ball(60 + i, 0, n, 5.0 + i)
        else:
            xyz, q, _ = synth.chain(60 + i, 0, n)
        mid = tcm.tcm_mol_upload(ctx, xyz, q, precision=prec)
        mols.append(dict(id=mid, xyz=xyz, q=q, prec=prec))
    return mols


def test_batch_matches_single_pair_path_and_oracle(ctx, orc, synth):
    mols = _upload_set(ctx, synth)
    rng = np.random.default_rng(5)
    pairs = [(0, 1), (2, 3), (1, 5), (4, 0), (5, 2), (3, 3), (0, 2)]
    Ls = [4, 8, 12, 16, 10, 6, 20]
    quats = synth.quaternions(77, 0, len(pairs))
    try:
        ext = {}
        for i, m in enumerate(mols):
            c = orc.centroid(m["xyz"])
            ext[i] = orc.radius(m["xyz"], c)
        Rs = []
        for (a, b) in pairs:
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            Rs.append(1.3 * (ext[a] + ext[b] + 1.0) * u)
        req = tcm.make_requests([mols[a]["id"] for a, _ in pairs], [mols[b]["id"] for _, b in pairs], Rs, Ls, quats)
        U, st, rc = tcm.tcm_batch_energy(ctx, req)
        assert rc == tcm.TCM_OK and np.all(st == 0)
        for k, (a, b) in enumerate(pairs):
            L = Ls[k]
            QA, aA, cA = tcm.tcm_mol_moments(ctx, mols[a]["id"], L, flags=tcm.TCM_REUSE)
            QB, aB, cB = tcm.tcm_mol_moments(ctx, mols[b]["id"], L, flags=tcm.TCM_REUSE)
            Us = tcm.tcm_pair_energy(ctx, QA, aA, QB, aB, Rs[k], L, quat_b=quats[k])
            assert Us == U[k]                  # same kernels, same inputs: bit for bit
            xA, qA = mols[a]["xyz"], mols[a]["q"]
            xB, qB = mols[b]["xyz"], mols[b]["q"]
            xBr = orc.pose(xB, cB, quats[k], cB)
            d = orc.energy(orc.moments(xA, qA, cA, L), orc.moments(xBr, qB, cB, L), Rs[k], L, full=True)
            tol = 1e-11 if (mols[a]["prec"] == 0 and mols[b]["prec"] == 0) else 3e-5
            assert abs(U[k] - d["U"]) <= tol * d["abs_sum"], (k, U[k], d["U"], d["abs_sum"])
    finally:
        for m in mols:
            tcm.tcm_mol_release(ctx, m["id"])


def test_alone_vs_mix_bitwise(ctx, synth):
    mols = _upload_set(ctx, synth)
    try:
        ids = [m["id"] for m in mols]
        target = tcm.make_requests(ids[1], ids[5], [900.0, 200.0, -300.0], 16, [0.8, 0.2, -0.3, 0.4])
        Ualone, st, _ = tcm.tcm_batch_energy(ctx, target)
        others = tcm.make_requests([ids[0], ids[2], ids[3], ids[4]], [ids[2], ids[3], ids[0], ids[1]],
                                   [[500.0, 0, 0]] * 4, [8, 12, 20, 24])
        mix = np.concatenate([others[:2], target, others[2:]])
        Umix, st2, _ = tcm.tcm_batch_energy(ctx, mix)
        assert st[0] == 0 and st2[2] == 0
        assert Umix[2] == Ualone[0]
    finally:
        for m in mols:
            tcm.tcm_mol_release(ctx, m["id"])


def test_batch_item_errors_do_not_fail_others(ctx, synth):
    mols = _upload_set(ctx, synth)
    try:
        ids = [m["id"] for m in mols]
        req = tcm.make_requests([ids[0], ids[0], 999_999, ids[2]], [ids[2], ids[2], ids[1], ids[3]],
                                [[1000.0, 0, 0], [1e-3, 0, 0], [1000.0, 0, 0], [1000.0, 0, 0]], [6, 6, 6, 40])
        U, st, rc = tcm.tcm_batch_energy(ctx, req)
        assert list(st) == [tcm.TCM_OK, tcm.TCM_EDOMAIN, tcm.TCM_ENOTFOUND, tcm.TCM_EINVAL]
        assert np.isfinite(U[0]) and np.all(np.isnan(U[1:]))
        assert rc == tcm.TCM_EDOMAIN
    finally:
        for m in mols:
            tcm.tcm_mol_release(ctx, m["id"])


def test_plan_graph_replay_matches_batch(ctx, synth):
    import torch
    mols = _upload_set(ctx, synth)
    try:
        ids = [m["id"] for m in mols]
        req = tcm.make_requests([ids[0], ids[1], ids[2]], [ids[3], ids[5], ids[4]],
                                [[800.0, 10, 0], [0, 1500.0, 0], [0, 0, 300.0]], [10, 16, 24],
                                synth.quaternions(3, 3, 3))
        Ub, stb, _ = tcm.tcm_batch_energy(ctx, req)
        for use_graph in (True, False):
            plan = tcm.tcm_plan_create(ctx, req, use_graph=use_graph)
            try:
                for rep in range(3):
                    tcm.tcm_plan_run(ctx, plan)
                    U, st = tcm.tcm_plan_results(ctx, plan, len(req))
                    assert np.all(st == 0) and np.array_equal(U, Ub), (use_graph, rep)
                    x = torch.randn(1000, device="cuda")   # unrelated eager work between replays
                    torch.cuda.synchronize()
                    del x
                tcm.tcm_plan_run_phased(ctx, plan)
                U, st = tcm.tcm_plan_results(ctx, plan, len(req))
                assert np.array_equal(U, Ub)
                info = tcm.tcm_plan_info(plan)
                assert info["pairs"] == 3 and info["atoms"] > 0
            finally:
                tcm.tcm_plan_destroy(plan)
    finally:
        for m in mols:
            tcm.tcm_mol_release(ctx, m["id"])


def test_register_device_matches_upload(ctx, synth):
    import torch
    xyz, q, _ = synth.chain(8, 0, 30_000)
    for prec in (tcm.TCM_F64, tcm.TCM_F32C):
        m1 = tcm.tcm_mol_upload(ctx, xyz, q, precision=prec)
        t = torch.tensor(np.vstack([xyz.T, q[None, :]]), dtype=torch.float64, device="cuda").contiguous()
        m2 = tcm.tcm_mol_register_device(ctx, t[0], t[1], t[2], t[3], len(q), precision=prec)
        try:
            Q1, r1, c1 = tcm.tcm_mol_moments(ctx, m1, 14)
            Q2, r2, c2 = tcm.tcm_mol_moments(ctx, m2, 14)
            assert np.array_equal(Q1, Q2) and r1 == r2 and np.array_equal(c1, c2)
        finally:
            tcm.tcm_mol_release(ctx, m1)
            tcm.tcm_mol_release(ctx, m2)
        torch.cuda.synchronize()


def test_contraction_kernels_give_the_same_bits(ctx, synth):
    """A pair's energy does not depend on the contraction kernel its launch takes: alone at
    order L (largest order <= 16: the 17-order register kernel), beside a pair of order 20 (the
    25-order register kernel) and beside a pair of order 28 (the LDS-staged kernel) it is the
    same to the bit, square and triangular.  The moments are computed once at order 28 and
    reused, so every call contracts the same tables."""
    xa, qa = synth.ball(71, 0, 400, 4.0)
    xb, qb = synth.ball(72, 0, 500, 5.0)
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    b = tcm.tcm_mol_upload(ctx, xb, qb, precision=tcm.TCM_F64)
    try:
        rng = np.random.default_rng(73)
        n = 70                                            # two groups of 64, the second ragged
        R = rng.normal(size=(n, 3))
        R *= (rng.uniform(14.0, 30.0, n) / np.linalg.norm(R, axis=1))[:, None]
        quats = synth.quaternions(74, 0, n + 1)
        _, st, rc = tcm.tcm_batch_energy(ctx, tcm.make_requests(a, b, [20.0, 0.0, 0.0], 28))
        assert rc == tcm.TCM_OK
        reuse = tcm.TCM_REUSE
        for flags in (0, tcm.TCM_TRIANGULAR):
            for L in (6, 12):
                alone = np.empty(n)
                for k in range(n):
                    U, st, rc = tcm.tcm_batch_energy(
                        ctx, tcm.make_requests(a, b, R[k], L, quats[k], flags=flags | reuse))
                    assert rc == tcm.TCM_OK
                    alone[k] = U[0]
                for Lf in (20, 28):                      # a last pair raises the launch's largest order
                    req = tcm.make_requests(a, b, np.vstack([R, [[0.0, 0.0, 25.0]]]), [L] * n + [Lf],
                                            quats, flags=flags | reuse)
                    U, st, rc = tcm.tcm_batch_energy(ctx, req)
                    assert rc == tcm.TCM_OK
                    assert np.array_equal(U[:n], alone), (flags, L, Lf)
    finally:
        tcm.tcm_mol_release(ctx, a)
        tcm.tcm_mol_release(ctx, b)


def test_large_batch_planned_on_threads_equals_small_batches(ctx, synth):
    """From 8192 pairs on the plan's pair records and rotation frames are filled on several
    host threads: 9000 posed pairs (mixed orders, some triangular) in one batch must equal, to the
    bit, the same pairs in two batches of 4500 planned on one thread."""
    xa, qa = synth.ball(81, 0, 300, 4.0)
    xb, qb = synth.ball(82, 0, 350, 4.5)
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    b = tcm.tcm_mol_upload(ctx, xb, qb, precision=tcm.TCM_F64)
    try:
        rng = np.random.default_rng(83)
        n = 9000
        R = rng.normal(size=(n, 3))
        R *= (rng.uniform(12.0, 40.0, n) / np.linalg.norm(R, axis=1))[:, None]
        L = rng.integers(2, 15, n)
        flags = np.where(rng.random(n) < 0.3, tcm.TCM_TRIANGULAR, 0) | tcm.TCM_REUSE
        quats = synth.quaternions(84, 0, n)
        _, _, rc = tcm.tcm_batch_energy(ctx, tcm.make_requests(a, b, [20.0, 0.0, 0.0], 14))
        assert rc == tcm.TCM_OK
        U, st, rc = tcm.tcm_batch_energy(ctx, tcm.make_requests(a, b, R, L, quats, flags=flags))
        assert rc == tcm.TCM_OK and np.all(st == 0)
        parts = []
        for s0 in (0, n // 2):
            sl = slice(s0, s0 + n // 2)
            Up, stp, rcp = tcm.tcm_batch_energy(ctx, tcm.make_requests(a, b, R[sl], L[sl], quats[sl], flags=flags[sl]))
            assert rcp == tcm.TCM_OK
            parts.append(Up)
        assert np.array_equal(U, np.concatenate(parts))
    finally:
        tcm.tcm_mol_release(ctx, a)
        tcm.tcm_mol_release(ctx, b)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129])
def test_group_edge_counts_match_single_pair_path(ctx, synth, n):
    """The pair kernels take 64 pairs per wavefront: batches that end one short of, at and one
    past a group of 64 (mixed orders, some triangular) give each pair the energy of the
    single-pair path on the same moments, to the bit."""
    xa, qa = synth.ball(91, 0, 300, 4.0)
    xb, qb = synth.ball(92, 0, 250, 3.5)
    a = tcm.tcm_mol_upload(ctx, xa, qa, precision=tcm.TCM_F64)
    b = tcm.tcm_mol_upload(ctx, xb, qb, precision=tcm.TCM_F64)
    try:
        Lmax = 14
        _, _, rc = tcm.tcm_batch_energy(ctx, tcm.make_requests(a, b, [20.0, 0.0, 0.0], Lmax))
        assert rc == tcm.TCM_OK                                  # both tables resident at Lmax
        QA, aA, _ = tcm.tcm_mol_moments(ctx, a, Lmax, flags=tcm.TCM_REUSE)
        QB, aB, _ = tcm.tcm_mol_moments(ctx, b, Lmax, flags=tcm.TCM_REUSE)
        rng = np.random.default_rng(93 + n)
        R = rng.normal(size=(n, 3))
        R *= (rng.uniform(12.0, 40.0, n) / np.linalg.norm(R, axis=1))[:, None]
        L = rng.integers(1, Lmax + 1, n)
        tri = rng.random(n) < 0.3
        quats = synth.quaternions(94, n, n)
        U, st, rc = tcm.tcm_batch_energy(ctx, tcm.make_requests(
            a, b, R, L, quats, flags=np.where(tri, tcm.TCM_TRIANGULAR, 0) | tcm.TCM_REUSE))
        assert rc == tcm.TCM_OK and np.all(st == 0)
        for k in range(n):
            h = (int(L[k]) + 1) ** 2
            Us = tcm.tcm_pair_energy(ctx, QA[:h], aA, QB[:h], aB, R[k], int(L[k]), quat_b=quats[k],
                                     flags=tcm.TCM_TRIANGULAR if tri[k] else 0)
            assert Us == U[k], (n, k, int(L[k]), bool(tri[k]), Us, U[k])
    finally:
        tcm.tcm_mol_release(ctx, a)
        tcm.tcm_mol_release(ctx, b)
