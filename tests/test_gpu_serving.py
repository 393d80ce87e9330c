"""The serving loop (continuous batching) through the C ABI: results equal the batch path's
bit for bit, a request's result is the same alone and in a mix, admission under a small HBM
budget evicts idle fragments and keeps serving, resident moments are reused across poses."""
import time

import numpy as np
import pytest

from paper_0704_1672_amd import tcm

pytestmark = pytest.mark.gpu


def frags(synth, n=8, seed=31):
    import torch
    sizes = [3000, 12000, 800, 25000, 5000, 40000, 1500, 9000][:n]
    out = []
    for i, s in enumerate(sizes):
        xyz, q, _ = synth.chain(seed, i, s)
        t = torch.tensor(np.vstack([xyz.T, q[None, :]]), dtype=torch.float64, device="cuda").contiguous()
        c = xyz.mean(0)
        a = float(np.sqrt(((xyz - c) ** 2).sum(1)).max())
        out.append(dict(xyz=xyz, q=q, t=t, n=s, ext=a, ptr=[t[k].data_ptr() for k in range(4)]))
    torch.cuda.synchronize()
    return out


def run_all(ctx, reqs, timeout=60.0):
    tickets = []
    for r in reqs:
        rc, tk = tcm.tcm_submit(ctx, r)
        assert rc == tcm.TCM_OK
        tickets.append(tk)
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for tk in tickets:
            if tk in res:
                continue
            rc, U, st, lat = tcm.tcm_poll(ctx, tk)
            if rc == tcm.TCM_OK:
                res[tk] = (U, st, lat)
        assert time.time() - t0 < timeout, "serving did not complete"
        time.sleep(0.001)
    return [res[tk] for tk in tickets]


def request(F, a, b, L, quat=(1.0, 0, 0, 0), d=1.6, with_atoms=True):
    u = np.array([0.3, -0.5, 0.8])
    u /= np.linalg.norm(u)
    R = d * (F[a]["ext"] + F[b]["ext"] + 1.0) * u
    return tcm.make_request(a, b, R, L, quat, atoms_a=F[a]["ptr"] if with_atoms else None, n_a=F[a]["n"],
                            atoms_b=F[b]["ptr"] if with_atoms else None, n_b=F[b]["n"])


def test_served_results_equal_batch_path(synth):
    F = frags(synth)
    pairs = [(0, 1, 8), (2, 3, 12), (1, 4, 16), (5, 6, 20), (7, 0, 24), (3, 5, 10), (0, 1, 8), (4, 2, 14)]
    quats = synth.quaternions(9, 9, len(pairs))
    with tcm.Context(0) as c:
        ids = [tcm.tcm_mol_register_device(c.h, *f["ptr"], f["n"]) for f in F]
        reqs = [request(F, a, b, L, quats[i]) for i, (a, b, L) in enumerate(pairs)]
        breq = tcm.make_requests([ids[a] for a, _, _ in pairs], [ids[b] for _, b, _ in pairs],
                                 [list(r.R) for r in reqs], [L for _, _, L in pairs], quats)
        Ub, stb, _ = tcm.tcm_batch_energy(c.h, breq)
        tcm.tcm_server_start(c.h, max_inflight_batches=2, max_batch_pairs=3, queue_capacity=64)
        out = run_all(c.h, reqs)
        stats = tcm.tcm_server_stats(c.h)
        tcm.tcm_server_stop(c.h)
    assert all(st == 0 for _, st, _ in out)
    assert np.array_equal(np.array([U for U, _, _ in out]), Ub)
    assert stats["completed"] == len(pairs) and stats["launches"] >= 3
    assert stats["cache_hits"] > 0


def test_alone_vs_mix(synth):
    F = frags(synth)
    target = request(F, 3, 5, 16, (0.6, 0.0, 0.8, 0.0))
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=3, max_batch_pairs=4, queue_capacity=64)
        (Ualone, st, _), = run_all(c.h, [target])
        tcm.tcm_server_stop(c.h)
        tcm.tcm_server_start(c.h, max_inflight_batches=3, max_batch_pairs=4, queue_capacity=64)
        rng = np.random.default_rng(4)
        mix = [request(F, int(a), int(b), int(L)) for a, b, L in
               zip(rng.integers(0, 8, 15), rng.integers(0, 8, 15), rng.integers(8, 25, 15))]
        mix.insert(7, target)
        out = run_all(c.h, mix)
        tcm.tcm_server_stop(c.h)
    assert st == 0 and out[7][1] == 0
    assert out[7][0] == Ualone


def test_admission_under_small_budget(synth, orc):
    F = frags(synth)
    total_atoms = 32 * sum(f["n"] for f in F)
    largest_pair = 32 * (F[5]["n"] + F[3]["n"])
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=2, max_batch_pairs=2, queue_capacity=64)
        run_all(c.h, [request(F, 2, 6, 8, with_atoms=True)])            # arena and workspaces
        used, _ = tcm.tcm_mem_info(c.h)
        # room for the largest pair plus a little, well below all fragments together
        budget = used + largest_pair + (total_atoms - largest_pair) // 4
        tcm.tcm_set_budget(c.h, budget)
        pairs = [(i % 8, (i * 3 + 1) % 8, 8 + (i % 3) * 4) for i in range(16)]
        out = run_all(c.h, [request(F, a, b, L) for a, b, L in pairs])
        stats = tcm.tcm_server_stats(c.h)
        used_after, _ = tcm.tcm_mem_info(c.h)
        tcm.tcm_server_stop(c.h)
    assert used_after <= budget
    assert all(st == 0 for _, st, _ in out), [st for _, st, _ in out]
    assert stats["evictions"] > 0
    # spot-check one result against the oracle
    a, b, L = pairs[5]
    r = request(F, a, b, L)
    cA, cB = orc.centroid(F[a]["xyz"]), orc.centroid(F[b]["xyz"])
    d = orc.energy(orc.moments(F[a]["xyz"], F[a]["q"], cA, L), orc.moments(F[b]["xyz"], F[b]["q"], cB, L),
                   np.array(list(r.R)), L, full=True)
    assert abs(out[5][0] - d["U"]) <= 1e-5 * d["abs_sum"]


def test_request_larger_than_budget_fails_alone(synth):
    F = frags(synth)
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=1, max_batch_pairs=4, queue_capacity=16)
        run_all(c.h, [request(F, 2, 6, 8)])
        used, _ = tcm.tcm_mem_info(c.h)
        tcm.tcm_set_budget(c.h, used + 4 * 2**20)
        import torch
        xyz, q, _ = synth.chain(1, 1, 300_000)                 # 9.6 MB of atoms: cannot fit
        t = torch.tensor(np.vstack([xyz.T, q[None, :]]), dtype=torch.float64, device="cuda").contiguous()
        torch.cuda.synchronize()
        huge = tcm.make_request(100, 0, [5000.0, 0, 0], 8, atoms_a=[t[k].data_ptr() for k in range(4)],
                                n_a=len(q), atoms_b=F[0]["ptr"], n_b=F[0]["n"])
        out = run_all(c.h, [huge, request(F, 0, 2, 8)])
        tcm.tcm_server_stop(c.h)
    assert out[0][1] == tcm.TCM_ENOMEM and np.isnan(out[0][0])
    assert out[1][1] == tcm.TCM_OK


def test_reuse_across_poses_hits_cache(synth, orc):
    F = frags(synth)
    quats = synth.quaternions(12, 1, 6)
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=2, max_batch_pairs=8, queue_capacity=64)
        first = run_all(c.h, [request(F, 1, 3, 12)])
        again = run_all(c.h, [request(F, 1, 3, 12, quats[i], with_atoms=False) for i in range(6)])
        stats = tcm.tcm_server_stats(c.h)
        tcm.tcm_server_stop(c.h)
    assert first[0][1] == 0 and all(st == 0 for _, st, _ in again)
    assert stats["cache_hits"] >= 12 and stats["cache_misses"] == 2
    cA, cB = orc.centroid(F[1]["xyz"]), orc.centroid(F[3]["xyz"])
    QA = orc.moments(F[1]["xyz"], F[1]["q"], cA, 12)
    r = request(F, 1, 3, 12, quats[2], with_atoms=False)
    xBr = orc.pose(F[3]["xyz"], cB, quats[2], cB)
    d = orc.energy(QA, orc.moments(xBr, F[3]["q"], cB, 12), np.array(list(r.R)), 12, full=True)
    assert abs(again[2][0] - d["U"]) <= 1e-5 * d["abs_sum"]


def test_serving_errors(synth):
    F = frags(synth)
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=1, max_batch_pairs=4, queue_capacity=2)
        unknown = request(F, 0, 1, 8, with_atoms=False)          # never seen, no atoms
        clash = tcm.make_request(0, 1, [1e-3, 0, 0], 8, atoms_a=F[0]["ptr"], n_a=F[0]["n"],
                                 atoms_b=F[1]["ptr"], n_b=F[1]["n"])
        out = run_all(c.h, [unknown, clash])
        assert out[0][1] == tcm.TCM_ENOTFOUND
        assert out[1][1] == tcm.TCM_EDOMAIN
        bad = request(F, 0, 1, 40)
        assert tcm.tcm_submit(c.h, bad)[0] == tcm.TCM_EINVAL
        rc, U, st, lat = tcm.tcm_poll(c.h, 10**9)
        assert rc == tcm.TCM_ENOTFOUND
        tcm.tcm_server_stop(c.h)


def test_reuse_after_atom_eviction(synth, orc):
    """A fragment whose atoms were evicted keeps its moment table: a request at an order it
    holds is served from it (same result as before the eviction, a cache hit); a higher order
    without atoms is ENOTFOUND and counted as an evicted miss; with atoms it is computed again."""
    F = frags(synth)
    quats = synth.quaternions(14, 2, 3)
    with tcm.Context(0) as c:
        tcm.tcm_server_start(c.h, max_inflight_batches=1, max_batch_pairs=4, queue_capacity=64)
        first = run_all(c.h, [request(F, 1, 3, 12)])
        used, _ = tcm.tcm_mem_info(c.h)
        # room for fragments 7 and 0 only once the atoms of 1 and 3 are gone
        gone = 32 * (F[1]["n"] + F[3]["n"])
        # (64 KiB of slack for the launch's workspace growth, far less than either fragment's atoms)
        tcm.tcm_set_budget(c.h, used - gone + 32 * (F[7]["n"] + F[0]["n"]) + (1 << 16))
        other = run_all(c.h, [request(F, 7, 0, 8)])
        s1 = tcm.tcm_server_stats(c.h)
        again = run_all(c.h, [request(F, 1, 3, 12, with_atoms=False)] +
                        [request(F, 1, 3, 10, quats[i], with_atoms=False) for i in range(3)])
        higher = run_all(c.h, [request(F, 1, 3, 16, with_atoms=False)])
        s2 = tcm.tcm_server_stats(c.h)
        tcm.tcm_set_budget(c.h, 0)
        refetched = run_all(c.h, [request(F, 1, 3, 16, quats[0])])
        s3 = tcm.tcm_server_stats(c.h)
        tcm.tcm_server_stop(c.h)
    assert first[0][1] == 0 and other[0][1] == 0
    assert s1["evictions"] >= 2 and s1["dropped"] == 0
    assert all(st == 0 for _, st, _ in again)
    assert again[0][0] == first[0][0]                       # the kept table, the same kernels
    assert s2["cache_hits"] - s1["cache_hits"] == 8         # both sides of the four reuse requests
    assert higher[0][1] == tcm.TCM_ENOTFOUND and np.isnan(higher[0][0])
    assert s2["evicted_misses"] == 1 and s1["evicted_misses"] == 0
    assert refetched[0][1] == 0 and s3["evicted_misses"] == 1
    cA, cB = orc.centroid(F[1]["xyz"]), orc.centroid(F[3]["xyz"])
    for L, q, U in [(10, quats[1], again[2][0]), (16, quats[0], refetched[0][0])]:
        r = request(F, 1, 3, L, q, with_atoms=False)
        xBr = orc.pose(F[3]["xyz"], cB, q, cB)
        d = orc.energy(orc.moments(F[1]["xyz"], F[1]["q"], cA, L), orc.moments(xBr, F[3]["q"], cB, L),
                       np.array(list(r.R)), L, full=True)
        assert abs(U - d["U"]) <= 1e-5 * d["abs_sum"], (L, U, d["U"])
