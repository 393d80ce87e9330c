"""Benchmark of the two-centre multipole (TCM) hot path on one MI355X.

Workload (one "step"): the uneven batch -- 1024 pairs of excluded-volume random-walk chains,
fragment sizes log-uniform in [1e3, 2e5] atoms (~77M atoms in total), order L per pair
uniform in {8, 12, 16, 20}, separation 1.5 (a_A + a_B) along a random direction, a random
pose of B; FP32-compensated moment pass, FP64 rotation and contraction.  The atoms are
resident in HBM (FP64 structure of arrays) before timing starts; one step runs the whole
batch -- centroid/scale statistics, the moment pass of all 2048 fragments, the fixed-order
finalisation and the 1024 posed pair contractions -- timed both as a replay of the captured
HIP graph and as direct launches on two streams, the faster of the two giving `value`.

Prints one JSON line (pair energies per second) with the moment pass's roofline position,
the relative error against the FP64 oracle on a sample of pairs, and the oracle's own
single-core throughput on that sample, followed by the serving, scan, all-pairs, forces,
adaptive-truncation and single-pair sections.  The oracle is called only in the CPU leg --
the baseline timing and the error statements -- which --no-cpu skips entirely.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0
# HBM traffic of the moment pass comes from rocprofv3 counter runs, summarised in this file
# together with the SHA-256 of every source the tile kernels are built from; it is reported
# only while those sources are unchanged
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_uneven_batch_1024.md")
TILE_SOURCES = ["paper_0704_1672_amd/csrc/tcm_device.h", "paper_0704_1672_amd/csrc/tcm_internal.h"] + \
               [f"paper_0704_1672_amd/csrc/tcm_tiles_f32_{k}.hip" for k in "abcd"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_tile_traffic():
    """Bytes per step of the tile launches from the committed counter summary, or None when
    it is missing or the tile kernel sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    for path in TILE_SOURCES:
        digest = hashlib.sha256(open(os.path.join(ROOT, path), "rb").read()).hexdigest()
        if f"{digest}  {path}" not in text:
            return None
    m = re.search(r"tile_traffic_bytes_per_step:\s*([0-9]+)", text)
    return int(m.group(1)) if m else None


def serving_section(tcm, synth, torch, nreq=10000, pool=48, oracle_seconds=8.0, fractions=(0.25, 0.5, 0.75, 0.9, 1.1),
                    inflight=3, batch=64, check=True):
    """Serving workload: a pool of chain fragments (log-uniform 1e3..1e6 atoms) resident in HBM,
    a trace of nreq pair requests with L ~ U{8..24}; 70% name two new fragments (new keys, atoms
    referenced in place), 30% reuse the fragments of an earlier request with a new pose and
    distance.  Saturation throughput from a closed burst; then Poisson arrivals at fractions of
    it, with p50/p99 of (completion - submission); the plain synchronous single-pair path
    (tcm_batch_energy on one request at a time) is timed on the same trace and its FIFO
    latencies computed for the same arrival times."""
    w = synth.serving_trace(seed=5, pool=pool, nreq=nreq, nmin=1_000, nmax=1_000_000, Lmin=8, Lmax=24,
                            reuse=0.3, qps=1.0, nthreads=min(16, os.cpu_count() or 1))
    ntot = int(w["offsets"][-1])
    dev = torch.device("cuda:0")
    soa = torch.empty((4, ntot), dtype=torch.float64, device=dev)
    soa[0:3] = torch.from_numpy(np.ascontiguousarray(w["xyz"].T)).to(dev)
    soa[3] = torch.from_numpy(w["q"]).to(dev)
    torch.cuda.synchronize()
    base, row = soa.data_ptr(), ntot * 8

    def ptrs(f):
        off = int(w["offsets"][f]) * 8
        return [base + k * row + off for k in range(4)]

    # request records: (key_a, frag_a, key_b, frag_b, new)
    recs = []
    news = []
    for i in range(nreq):
        if w["reuse"][i] and news:
            j = news[int(w["a"][i]) % len(news)]
            recs.append((recs[j][0], recs[j][1], recs[j][2], recs[j][3], False))
        else:
            recs.append((2 * i, int(w["a"][i]), 2 * i + 1, int(w["b"][i]), True))
            news.append(i)
    ext = w["extent"]
    dirs = w["R"] / np.linalg.norm(w["R"], axis=1)[:, None]

    def make(i, borrow=True):
        ka, fa, kb, fb, new = recs[i]
        R = 1.5 * (ext[fa] + ext[fb]) * dirs[i]
        return tcm.make_request(ka, kb, R, int(w["L"][i]), w["quats"][i],
                                atoms_a=ptrs(fa) if new else None, n_a=int(w["counts"][fa]),
                                atoms_b=ptrs(fb) if new else None, n_b=int(w["counts"][fb]),
                                flags=tcm.TCM_BORROW_ATOMS if borrow else 0)

    reqs = [make(i) for i in range(nreq)]

    def run(ctx, arrivals, rq=None):
        rq = reqs if rq is None else rq
        tcm.tcm_server_start(ctx.h, max_inflight_batches=inflight, max_batch_pairs=batch, queue_capacity=nreq + 16)
        tickets = [None] * nreq
        lat = np.zeros(nreq)
        U = np.zeros(nreq)
        st = np.zeros(nreq, dtype=np.int32)
        done = 0
        t0 = time.perf_counter()
        i = 0
        pending = []
        while done < nreq:
            now = time.perf_counter() - t0
            while i < nreq and (arrivals is None or arrivals[i] <= now):
                rc, tk = tcm.tcm_submit(ctx.h, rq[i])
                assert rc == 0
                tickets[i] = tk
                pending.append(i)
                i += 1
            keep = []
            for k in pending:
                rc, u, s_, l_ = tcm.tcm_poll(ctx.h, tickets[k])
                if rc == 0:
                    U[k], st[k], lat[k] = u, s_, l_
                    done += 1
                else:
                    keep.append(k)
            pending = keep
        elapsed = time.perf_counter() - t0
        stats = tcm.tcm_server_stats(ctx.h)
        tcm.tcm_server_stop(ctx.h)
        return U, st, lat, elapsed, stats

    ctx = tcm.Context(0)
    tcm.tcm_set_budget(ctx.h, 64 << 30)                       # a realistic, non-binding HBM budget
    run(ctx, None)                                            # warm-up (allocations, code load)
    U, st, lat, elapsed, stats = run(ctx, None)
    sat = nreq / elapsed
    out = {"workload": f"serving trace: {nreq} requests, pool of {pool} chain fragments ({ntot} atoms), "
                       "log-uniform 1e3..1e6 atoms, L ~ U{8..24}, 30% reuse of resident fragments, "
                       "R0 = 1.5(a_A+a_B), random poses; inputs resident in HBM (borrowed); 64 GiB budget",
           "server": {"max_inflight_batches": inflight, "max_batch_pairs": batch},
           "saturation_pairs_per_s": sat, "burst_stats": stats, "statuses_ok": int(np.sum(st == 0))}
    rng = np.random.default_rng(55)
    gaps = rng.exponential(1.0, nreq)
    loads = {}
    for f in fractions:
        arr = np.cumsum(gaps) / (f * sat)
        Uf, stf, latf, el, sts = run(ctx, arr)
        loads[str(f)] = {"qps": f * sat, "pairs_per_s": nreq / el, "p50_ms": 1e3 * float(np.percentile(latf, 50)),
                         "p99_ms": 1e3 * float(np.percentile(latf, 99)), "launches": sts["launches"],
                         "cache_hits": sts["cache_hits"], "cache_misses": sts["cache_misses"]}
    out["open_loop"] = loads
    # alone vs in the mix: every served result equals the burst's bit for bit
    out["alone_vs_mix_bitwise_equal"] = bool(np.array_equal(Uf, U))
    # a binding HBM budget: the atoms copied into server memory (not borrowed), 512 MiB for
    # atoms, moment tables and launch workspaces, so fragments are evicted least recently used
    # first; a request whose resident fragment was evicted reports TCM_ENOTFOUND
    budget = 512 << 20
    ctxb = tcm.Context(0)
    tcm.tcm_set_budget(ctxb.h, budget)
    reqs_c = [make(i, borrow=False) for i in range(nreq)]
    run(ctxb, None, reqs_c)                                   # warm-up, as for the unbounded run
    Ub, stb, latb, elb, stsb = run(ctxb, None, reqs_c)
    ok = stb == 0
    out["binding_budget"] = {
        "budget_bytes": budget, "atoms": "copied into server memory",
        "saturation_pairs_per_s": nreq / elb, "server_stats": stsb,
        "statuses": {str(int(v)): int(np.sum(stb == v)) for v in np.unique(stb)},
        "ok_results_equal_unbounded_bitwise": bool(np.array_equal(Ub[ok], U[ok]))}
    ctxb.close()
    # plain single-pair GPU path on the same trace
    ids = {}
    for f in range(pool):
        ids[f] = tcm.tcm_mol_register_device(ctx.h, *ptrs(f), int(w["counts"][f]))
    service = np.zeros(nreq)
    Up = np.zeros(nreq)
    for i in range(nreq):
        ka, fa, kb, fb, new = recs[i]
        r = reqs[i]
        rq = tcm.make_requests(ids[fa], ids[fb], list(r.R), int(r.L), list(r.quat_b),
                               flags=0 if new else tcm.TCM_REUSE)
        t1 = time.perf_counter()
        u, s_, _ = tcm.tcm_batch_energy(ctx.h, rq)
        service[i] = time.perf_counter() - t1
        Up[i] = u[0]
    out["plain_single_pair"] = {"pairs_per_s": nreq / service.sum(), "mean_service_ms": 1e3 * service.mean()}
    for f in fractions:
        arr = np.cumsum(gaps) / (f * sat)
        fin = np.zeros(nreq)
        tprev = 0.0
        for i in range(nreq):
            tprev = max(arr[i], tprev) + service[i]
            fin[i] = tprev
        l = fin - arr
        out["plain_single_pair"][str(f)] = {"p50_ms": 1e3 * float(np.percentile(l, 50)),
                                            "p99_ms": 1e3 * float(np.percentile(l, 99))}
    out["served_vs_plain_max_rel_diff"] = float(np.max(np.abs(U - Up) / np.maximum(np.abs(Up), 1e-300)))
    # relative error vs the FP64 oracle on a sample (smallest requests first, bounded time):
    # part of the CPU leg, skipped with --no-cpu
    out["rel_err"] = None
    if check:
        import oracle
        order = np.argsort([w["counts"][r[1]] + w["counts"][r[3]] for r in recs])
        rel, t_cpu, k = [], 0.0, 0
        for i in order:
            if t_cpu > oracle_seconds:
                break
            ka, fa, kb, fb, new = recs[i]
            xa = w["xyz"][w["offsets"][fa]:w["offsets"][fa + 1]]
            qa = w["q"][w["offsets"][fa]:w["offsets"][fa + 1]]
            xb = w["xyz"][w["offsets"][fb]:w["offsets"][fb + 1]]
            qb = w["q"][w["offsets"][fb]:w["offsets"][fb + 1]]
            L = int(w["L"][i])
            ts = time.perf_counter()
            cA, cB = oracle.centroid(xa), oracle.centroid(xb)
            d = oracle.energy(oracle.moments(xa, qa, cA, L),
                              oracle.moments(oracle.pose(xb, cB, w["quats"][i], cB), qb, cB, L),
                              np.array(list(reqs[i].R)), L, full=True)
            t_cpu += time.perf_counter() - ts
            k += 1
            rel.append((abs(U[i] - d["U"]) / abs(d["U"]), abs(U[i] - d["U"]) / d["abs_sum"]))
        rel = np.array(rel)
        out["rel_err"] = {"sample_requests": k, "max_rel": float(rel[:, 0].max()), "median_rel": float(np.median(rel[:, 0])),
                          "max_err_over_abs_terms": float(rel[:, 1].max())}
    ctx.close()
    del soa
    torch.cuda.empty_cache()
    return out


def scan_section(tcm, synth, torch, npos=1 << 20, L=16, oracle_samples=8, check=True):
    """Translation scan (the paper's section IV scan shape, in all directions): B at npos
    positions around A, B keeping one pose, L = 16, two 20k-bead chains; positions, energies and
    statuses in device memory.  Throughput of tcm_scan_translations against the pair path
    (tcm_batch_energy with resident moments) on the first 16384 positions, and the error
    against the FP64 oracle on a sample."""
    import ctypes as C
    xa, qa, _ = synth.chain(21, 1, 20_000)
    xb, qb, _ = synth.chain(21, 2, 20_000)
    ctx = tcm.Context(0)
    mA = tcm.tcm_mol_upload(ctx.h, xa, qa, precision=tcm.TCM_F32C)
    mB = tcm.tcm_mol_upload(ctx.h, xb, qb, precision=tcm.TCM_F32C)
    cA, cB = synth.centroid(xa), synth.centroid(xb)
    rho = synth.max_extent(xa, cA) + synth.max_extent(xb, cB)
    rng = np.random.default_rng(77)
    d = rng.normal(size=(npos, 3))
    R = d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(1.1, 3.0, npos)[:, None] * rho
    quat = np.array([0.7, 0.1, -0.5, 0.5])
    quat /= np.linalg.norm(quat)
    dR = torch.tensor(R, dtype=torch.float64, device="cuda")
    dU = torch.empty(npos, dtype=torch.float64, device="cuda")
    dS = torch.empty(npos, dtype=torch.int32, device="cuda")
    q = np.ascontiguousarray(quat)
    torch.cuda.synchronize()                  # R is on the device before the context's stream reads it

    def scan(flags):
        rc = tcm.lib().tcm_scan_translations(ctx.h, mA, mB, L, q.ctypes.data_as(tcm._dp), flags | tcm.TCM_DEVICE_IO,
                                             C.cast(dR.data_ptr(), tcm._dp), npos, C.cast(dU.data_ptr(), tcm._dp),
                                             C.cast(dS.data_ptr(), tcm._ip32))
        assert rc == tcm.TCM_OK, rc

    scan(0)                                   # moments at L, then the scan
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        scan(tcm.TCM_REUSE)
    torch.cuda.synchronize()
    t_scan = (time.perf_counter() - t0) / reps
    U = dU.cpu().numpy()
    st = dS.cpu().numpy()
    npair = 16384
    req = tcm.make_requests(mA, mB, R[:npair], L, quat, flags=tcm.TCM_REUSE)
    tcm.tcm_batch_energy(ctx.h, req)
    t0 = time.perf_counter()
    Ub, stb, _ = tcm.tcm_batch_energy(ctx.h, req)
    t_pair = time.perf_counter() - t0
    errs = []
    if check:                                 # the CPU leg (skipped with --no-cpu)
        import oracle
        QA = oracle.moments(xa, qa, cA, L)
        QB = oracle.moments(oracle.pose(xb, cB, quat, cB), qb, cB, L)
        for k in np.linspace(0, npos - 1, oracle_samples).astype(int):
            e = oracle.energy(QA, QB, R[k], L, full=True)
            errs.append(abs(U[k] - e["U"]) / e["abs_sum"])
    out = {"workload": f"two 20k-bead chains, L = {L}, {npos} positions at 1.1-3.0 (a_A + a_B) in random "
                       "directions, one pose of B; FP32-compensated moments once, FP64 pair tensor and "
                       "evaluation; positions and results in device memory",
           "positions_per_s": npos / t_scan, "ms_per_scan": 1e3 * t_scan, "statuses_ok": int(np.sum(st == 0)),
           "pair_path_positions_per_s": npair / t_pair,
           "speedup_vs_pair_path": (npos / t_scan) / (npair / t_pair),
           "scan_vs_pair_path_max_abs_diff": float(np.max(np.abs(U[:npair] - Ub))),
           "max_err_over_abs_terms_vs_oracle": float(max(errs)) if errs else None,
           "oracle_samples": len(errs)}
    tcm.tcm_mol_release(ctx.h, mA)
    tcm.tcm_mol_release(ctx.h, mB)
    ctx.close()
    return out


def all_pairs_section(tcm, synth, K=256, L=8, reps=5):
    """Every pair of K chain fragments in place (log-uniform 2k..20k beads on a cubic grid
    wide enough that no two overlap): moments once per fragment, then K(K-1)/2 contractions.
    Timed as a first call in a fresh context (moments + centres + contractions, with the
    context's workspaces allocated), as calls reusing the resident moments, and as calls
    recomputing the moments with warm workspaces."""
    counts = np.floor(np.exp(np.random.default_rng(41).uniform(np.log(2e3), np.log(2e4), K))).astype(np.int64)
    xyz, q, off, _ = synth.chains(41, 1, counts, nthreads=min(16, os.cpu_count() or 1))
    side = int(np.ceil(K ** (1 / 3)))
    ctx = tcm.Context(0)
    ids = []
    for k in range(K):
        x = xyz[off[k]:off[k + 1]]
        g = np.array([k % side, (k // side) % side, k // (side * side)], dtype=float) * 600.0
        ids.append(tcm.tcm_mol_upload(ctx.h, x - x.mean(axis=0) + g, q[off[k]:off[k + 1]], precision=tcm.TCM_F32C))
    t0 = time.perf_counter()
    U, st = tcm.tcm_all_pairs(ctx.h, ids, L)
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(reps):
        U2, _ = tcm.tcm_all_pairs(ctx.h, ids, L, flags=tcm.TCM_REUSE)
    t_reuse = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        U3, _ = tcm.tcm_all_pairs(ctx.h, ids, L)          # moments recomputed, workspaces warm
    t_recompute = (time.perf_counter() - t0) / reps
    npairs = len(U)
    out = {"workload": f"{K} chain fragments in place ({int(counts.sum())} atoms, log-uniform 2e3..2e4 beads, "
                       f"600 A grid), L = {L}, FP32-compensated moments, FP64 contractions, host I/O",
           "pairs": npairs, "statuses_ok": int(np.sum(st == 0)),
           "first_call_ms": 1e3 * t_first, "pairs_per_s_first_call": npairs / t_first,
           "first_call_note": "a fresh context: includes allocating and growing its workspaces",
           "recompute_call_ms": 1e3 * t_recompute, "pairs_per_s_recompute": npairs / t_recompute,
           "reuse_call_ms": 1e3 * t_reuse, "pairs_per_s_reuse": npairs / t_reuse,
           "reuse_equal_bitwise": bool(np.array_equal(U, U2)),
           "recompute_equal_bitwise": bool(np.array_equal(U, U3)),
           "system_energy": float(np.sum(U[st == 0]))}
    for i in ids:
        tcm.tcm_mol_release(ctx.h, i)
    ctx.close()
    return out


def forces_section(tcm, synth, torch, L=16, npose=4096, reps=10):
    """Forces: (1) per-atom forces on two 100k-bead chains at L = 16 (B posed), device I/O,
    resident FP32C moments; (2) force and torque on the centres for 4096 poses of the pair
    (tcm_batch_forces) against the energy-only batch on the same requests."""
    import ctypes as C
    w = synth.chain_pair(seed=2, n=100_000)
    xA, qA, xB, qB = w["xyzA"], w["qA"], w["xyzB_body"], w["qB"]
    ctx = tcm.Context(0)
    mA = tcm.tcm_mol_upload(ctx.h, xA, qA, precision=tcm.TCM_F32C)
    mB = tcm.tcm_mol_upload(ctx.h, xB, qB, precision=tcm.TCM_F32C)
    cA, cB = xA.mean(axis=0), xB.mean(axis=0)
    R = np.ascontiguousarray(np.asarray(w["seps"][-1]) + (cB - cA))
    quat = np.ascontiguousarray(synth.quaternions(15, 0, 1)[0])
    FA = torch.empty((len(qA), 3), dtype=torch.float64, device="cuda")
    FB = torch.empty((len(qB), 3), dtype=torch.float64, device="cuda")
    out = np.empty(10)

    def call(flags):
        rc = tcm.lib().tcm_pair_forces(ctx.h, mA, mB, R.ctypes.data_as(tcm._dp), quat.ctypes.data_as(tcm._dp), L,
                                       flags | tcm.TCM_DEVICE_IO, out.ctypes.data_as(tcm._dp),
                                       C.cast(FA.data_ptr(), tcm._dp), C.cast(FB.data_ptr(), tcm._dp))
        assert rc == tcm.TCM_OK, rc

    call(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        call(tcm.TCM_REUSE)
    torch.cuda.synchronize()
    t_atoms = (time.perf_counter() - t0) / reps
    rng = np.random.default_rng(61)
    d = rng.normal(size=(npose, 3))
    Rs = d / np.linalg.norm(d, axis=1)[:, None] * np.linalg.norm(R)
    req = tcm.make_requests(mA, mB, Rs, L, synth.quaternions(16, 0, npose), flags=tcm.TCM_REUSE)
    def med(f, k=5):                          # median of k timed calls after one untimed
        f()
        ts = []
        for _ in range(k):
            t0 = time.perf_counter()
            r = f()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), r

    t_ft, (o, st, _) = med(lambda: tcm.tcm_batch_forces(ctx.h, req))
    t_e, (U, _, _) = med(lambda: tcm.tcm_batch_energy(ctx.h, req))
    res = {"workload": f"two 100k-bead chains, L = {L}, FP32-compensated resident moments, FP64 derivatives",
           "per_atom": {"atoms": len(qA) + len(qB), "ms_per_call": 1e3 * t_atoms,
                        "atoms_per_s": (len(qA) + len(qB)) / t_atoms,
                        "note": "tcm_pair_forces with device I/O: pair kernel (U, F_B, torques, per-atom tables) + "
                                "two per-atom launches, one synchronisation"},
           "batch": {"pairs": npose, "statuses_ok": int(np.sum(st == 0)), "ms": 1e3 * t_ft,
                     "pairs_per_s": npose / t_ft, "energy_only_ms": 1e3 * t_e, "timing": "median of 5 calls",
                     "max_rel_diff_U_vs_energy_path": float(np.max(np.abs(o[:, 0] - U) / np.abs(U)))}}
    tcm.tcm_mol_release(ctx.h, mA)
    tcm.tcm_mol_release(ctx.h, mB)
    del FA, FB
    ctx.close()
    return res


def adaptive_section(tcm, synth, L=24, npose=4096, fracs=(1e-3, 1e-5)):
    """Adaptive truncation: two 50k-charge balls, 4096 random poses at 3..6 radii of gyration,
    maximum order 24, resident moments; each tolerance is a fraction of S_A S_B / median |R|
    (S = sum |q|, the scale of the rigorous bound).  Times the adaptive call against the fixed
    order-24 batch on the same requests (median of 5 calls each) and reports the orders chosen
    and the largest |U_adaptive - U_24| over the sum of the two bounds (at most 1 up to the
    moment pass's rounding, since each bound covers its own truncation)."""
    w = synth.orientation_scan(seed=3, n=50_000, nposes=npose, L=L)
    ctx = tcm.Context(0)
    mA = tcm.tcm_mol_upload(ctx.h, w["xyzA"], w["qA"], precision=tcm.TCM_F32C)
    mB = tcm.tcm_mol_upload(ctx.h, w["xyzB"], w["qB"], precision=tcm.TCM_F32C)
    req = tcm.make_requests(mA, mB, w["R"], L, w["quats"], flags=tcm.TCM_REUSE)
    tcm.tcm_batch_energy(ctx.h, tcm.make_requests(mA, mB, w["R"][:1], L, w["quats"][:1]))   # resident moments

    def med(f, k=5):
        f()
        ts = []
        for _ in range(k):
            t0 = time.perf_counter()
            r = f()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), r

    t_fix, (U24, st24, _) = med(lambda: tcm.tcm_batch_energy(ctx.h, req))
    _, _, b24, _, _ = tcm.tcm_batch_energy_adaptive(ctx.h, req, 1e-300)     # the bound at order 24
    scale = float(np.sum(np.abs(w["qA"])) * np.sum(np.abs(w["qB"])) / np.median(np.linalg.norm(w["R"], axis=1)))
    runs = {}
    for f in fracs:
        tol = f * scale
        t_ad, (U, Lu, b, st, rc) = med(lambda: tcm.tcm_batch_energy_adaptive(ctx.h, req, tol))
        ok = (st == 0) & (st24 == 0)
        met = ok & (b <= tol)
        reqL = req.copy()
        reqL["L"] = np.maximum(Lu, 0)
        t_at, _ = med(lambda: tcm.tcm_batch_energy(ctx.h, reqL))     # the same orders, given
        runs[f"{f:g}"] = {"tol": tol, "ms": 1e3 * t_ad, "pairs_per_s": npose / t_ad,
                          "speedup_vs_fixed_L": t_fix / t_ad, "statuses_ok": int(np.sum(st == 0)),
                          "batch_at_chosen_orders_ms": 1e3 * t_at,
                          "L_used": {"min": int(Lu[ok].min()), "median": float(np.median(Lu[ok])),
                                     "mean": float(Lu[ok].mean()), "max": int(Lu[ok].max())},
                          "pairs_meeting_tol": int(np.sum(met)),
                          "max_diff_over_bounds": float(np.max(np.abs(U[ok] - U24[ok]) / (b[ok] + b24[ok])))}
    res = {"workload": f"two 50k-charge balls (q ~ U[-1, 1]), {npose} poses at 3..6 Rg, maximum L = {L}, "
                       "FP32-compensated resident moments; tol = fraction x S_A S_B / median |R|",
           "fixed_L": {"L": L, "ms": 1e3 * t_fix, "pairs_per_s": npose / t_fix}, "adaptive": runs,
           "timing": "median of 5 calls"}
    tcm.tcm_mol_release(ctx.h, mA)
    tcm.tcm_mol_release(ctx.h, mB)
    ctx.close()
    return res


def single_pair_section(tcm, synth, reps=1000, check=True):
    """One pair at a time (two balls of 500 charges, q ~ U[-1, 1], radius 10, centres 60 apart,
    L = 10, FP64 moments): p50/p99 of tcm_batch_energy over `reps` synchronous calls, with the
    moments recomputed in every call and with resident moments, and the error of the result
    against the FP64 oracle and against the direct Coulomb sum of eq. (1) (the CPU leg, skipped
    with --no-cpu)."""
    w = synth.ball_pair(seed=1)
    L = int(w["L"])
    ctx = tcm.Context(0)
    mA = tcm.tcm_mol_upload(ctx.h, w["xyzA"], w["qA"], centre=w["cA"], precision=tcm.TCM_F64)
    mB = tcm.tcm_mol_upload(ctx.h, w["xyzB"], w["qB"], centre=w["cB"], precision=tcm.TCM_F64)
    out = {"workload": "two balls of 500 charges (q ~ U[-1, 1], radius 10), centres 60 apart, L = 10, "
                       "FP64 moments and contraction, one synchronous call per pair", "calls": reps}
    U = None
    for name, flags in (("moments_recomputed", 0), ("resident_moments", tcm.TCM_REUSE)):
        req = tcm.make_requests(mA, mB, w["R"], L, flags=flags)
        tcm.tcm_batch_energy(ctx.h, req)                      # warm-up
        ts = np.empty(reps)
        for i in range(reps):
            t0 = time.perf_counter()
            u, st, _ = tcm.tcm_batch_energy(ctx.h, req)
            ts[i] = time.perf_counter() - t0
        assert st[0] == 0
        U = float(u[0])
        out[name] = {"p50_ms": 1e3 * float(np.percentile(ts, 50)), "p99_ms": 1e3 * float(np.percentile(ts, 99)),
                     "pairs_per_s": reps / float(ts.sum())}
    out["U"] = U
    out["rel_err_vs_oracle"] = out["rel_truncation_vs_coulomb"] = None
    if check:
        import oracle
        d = oracle.energy(oracle.moments(w["xyzA"], w["qA"], w["cA"], L),
                          oracle.moments(w["xyzB"], w["qB"], w["cB"], L), w["R"], L, full=True)
        Uc = oracle.coulomb(w["xyzA"], w["qA"], w["xyzB"], w["qB"])
        out["rel_err_vs_oracle"] = abs(U - d["U"]) / abs(d["U"])
        out["rel_truncation_vs_coulomb"] = abs(U - Uc) / abs(Uc)
    tcm.tcm_mol_release(ctx.h, mA)
    tcm.tcm_mol_release(ctx.h, mB)
    ctx.close()
    return out


def large_molecule(tcm, torch, n, L=8, reps=8):
    """Phase times (HIP events) of the moment pass of one molecule of n atoms: the statistics
    and centre/scale, the tile launch, and the finalisation that merges the tiles' partials
    (the pair launch is a single pair with itself, unchecked)."""
    stride = n + 64
    buf = torch.rand(4 * stride, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ctx = tcm.Context(0)
    base = buf.data_ptr()
    mid = tcm.tcm_mol_register_device(ctx.h, *[base + 8 * stride * k for k in range(4)], n)
    pl = tcm.tcm_plan_create(ctx.h, tcm.make_requests(mid, mid, [1e9, 0.0, 0.0], L, flags=tcm.TCM_UNCHECKED),
                             use_graph=False)
    ms = np.array([tcm.tcm_plan_run_timed(ctx.h, pl) for _ in range(reps)])[2:]
    tcm.tcm_plan_destroy(pl)
    tcm.tcm_mol_release(ctx.h, mid)
    ctx.close()
    med = np.median(ms, axis=0)
    return {"workload": f"one molecule of {n} atoms (uniform random in device memory), L = {L}, FP32 moments",
            "phase_ms": {"stats": float(med[0]), "moment_tiles": float(med[1]), "moment_finalise": float(med[2]),
                         "pairs": float(med[3])}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--npairs", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="bound on the oracle sample time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-inflight", type=int, default=3, help="serving launches in flight at once")
    ap.add_argument("--serve-batch", type=int, default=64, help="requests admitted into one serving launch")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--no-all-pairs", action="store_true")
    ap.add_argument("--no-forces", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--large-molecule", type=int, default=0, metavar="N",
                    help="only time the moment pass of one molecule of N atoms (L = 8, uniform random "
                         "coordinates and charges in device memory) by phase, and exit")
    ap.add_argument("--alu-calibration", action="store_true",
                    help="only measure the sustained plain FP32 and FP64 FMA rates and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (reference "
                         "point for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    from paper_0704_1672_amd import synth, tcm
    if args.large_molecule > 0:
        print(json.dumps(large_molecule(tcm, torch, args.large_molecule)), flush=True)
        return
    if args.alu_calibration:
        ctx = tcm.Context(0)
        r = {"fp32_fma_tflops": tcm.tcm_alu_calibrate(ctx.h, tcm.TCM_F32C),
             "fp64_fma_tflops": tcm.tcm_alu_calibrate(ctx.h, tcm.TCM_F64)}
        ctx.close()
        print(json.dumps(r), flush=True)
        return

    t0 = time.time()
    w = synth.uneven_batch(seed=4, npairs=args.npairs, nthreads=min(16, os.cpu_count() or 1))
    ntot = int(w["offsets"][-1])
    log(f"bench: generated {2 * args.npairs} fragments, {ntot} atoms in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    soa = torch.empty((4, ntot), dtype=torch.float64, device=dev)
    soa[0:3] = torch.from_numpy(np.ascontiguousarray(w["xyz"].T)).to(dev)
    soa[3] = torch.from_numpy(w["q"]).to(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream(device=dev)
    ctx = tcm.Context(0)
    tcm.tcm_set_stream(ctx.h, stream)
    ids = []
    base = soa.data_ptr()
    row = ntot * 8
    for f in range(2 * args.npairs):
        off = int(w["offsets"][f]) * 8
        n = int(w["counts"][f])
        ids.append(tcm.tcm_mol_register_device(ctx.h, base + off, base + row + off, base + 2 * row + off,
                                               base + 3 * row + off, n, precision=tcm.TCM_F32C))
    # autotuned tile shapes: for each L group of this batch, the atoms per thread whose tile
    # launch is fastest on the batch itself (one value per group, kept for its size buckets)
    req = tcm.make_requests(ids[0::2], ids[1::2], w["R"], w["L"], w["quats"])
    t_tune = time.time()
    tcm.tcm_autotune_batch(ctx.h, req)
    tuned = {}
    for L in sorted(set(int(x) for x in w["L"])):
        sizes = np.concatenate([w["counts"][0::2][w["L"] == L], w["counts"][1::2][w["L"] == L]])
        for b in sorted(set(int(np.log2(n)) for n in sizes)):
            tuned[f"L{L}/2^{b}"] = tcm.tcm_tune_get(ctx.h, tcm.TCM_F32C, L, 1 << b)
    log(f"bench: batch autotune in {time.time() - t_tune:.2f}s: {tuned}")
    plan = tcm.tcm_plan_create(ctx.h, req, use_graph=True)           # serial order, one graph
    plan_s = tcm.tcm_plan_create(ctx.h, req, use_graph=False)        # tile launches on two streams
    info = tcm.tcm_plan_info(plan)
    log(f"bench: plan: {info}")

    def timed(p):
        for _ in range(args.warmup):
            tcm.tcm_plan_run(ctx.h, p)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            tcm.tcm_plan_run(ctx.h, p)
        stream.synchronize()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t1) / args.steps

    ms_graph = timed(plan)
    U, st = tcm.tcm_plan_results(ctx.h, plan, args.npairs)
    ms_streams = timed(plan_s)
    Us, sts = tcm.tcm_plan_results(ctx.h, plan_s, args.npairs)
    assert np.array_equal(U, Us) and np.array_equal(st, sts), "graph and stream runs differ"
    mode = "graph" if ms_graph <= ms_streams else "streams"
    ms_step = min(ms_graph, ms_streams)
    log(f"bench: {args.steps} steps: graph replay {ms_graph:.3f} ms/step, direct launches on two streams "
        f"{ms_streams:.3f} ms/step; statuses ok: {int(np.sum(st == 0))}")

    # per-kernel durations: HIP events on the launch stream around each phase
    phases = np.array([tcm.tcm_plan_run_timed(ctx.h, plan) for _ in range(max(3, args.steps))])
    ph = phases.mean(axis=0)
    U2, _ = tcm.tcm_plan_results(ctx.h, plan, args.npairs)
    assert np.array_equal(U, U2), "phased run differs from graph replay"
    moment_tflops = info["moment_flops"] / (ph[1] * 1e-3) / 1e12
    log(f"bench: phase ms stats={ph[0]:.3f} tiles={ph[1]:.3f} finalise={ph[2]:.3f} pairs={ph[3]:.3f}; "
        f"moment pass {moment_tflops:.1f} TFLOP/s")
    # the sustained plain-FMA rate of this device (outside the timed region): the ceiling the
    # tile kernels can reach without packed FP32
    fp32_ceiling = tcm.tcm_alu_calibrate(ctx.h, tcm.TCM_F32C)
    log(f"bench: plain FP32 FMA ceiling {fp32_ceiling:.1f} TFLOP/s")

    # oracle on a bounded sample of pairs: throughput baseline and relative error
    cpu = None
    err = None
    if not args.no_cpu:
        import oracle
        oracle.load()
        rel, rel_abs = [], []
        t_cpu = 0.0
        k = 0
        order = np.argsort(w["counts"][0::2] + w["counts"][1::2])  # smallest pairs first
        sample_atoms = 0
        for p in order:
            if t_cpu > args.cpu_seconds:
                break
            a, b = 2 * p, 2 * p + 1
            xa = w["xyz"][w["offsets"][a]:w["offsets"][a + 1]]
            qa = w["q"][w["offsets"][a]:w["offsets"][a + 1]]
            xb = w["xyz"][w["offsets"][b]:w["offsets"][b + 1]]
            qb = w["q"][w["offsets"][b]:w["offsets"][b + 1]]
            L = int(w["L"][p])
            ts = time.perf_counter()
            cA = oracle.centroid(xa)
            cB = oracle.centroid(xb)
            xbr = oracle.pose(xb, cB, w["quats"][p], cB)
            d = oracle.energy(oracle.moments(xa, qa, cA, L), oracle.moments(xbr, qb, cB, L), w["R"][p], L,
                              full=True)
            t_cpu += time.perf_counter() - ts
            k += 1
            sample_atoms += len(qa) + len(qb)
            rel.append(abs(U[p] - d["U"]) / abs(d["U"]))
            rel_abs.append(abs(U[p] - d["U"]) / d["abs_sum"])
        cpu = {"value": k / t_cpu, "unit": "pair energies/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} smallest pairs of the batch ({sample_atoms} atoms), single-threaded FP64 oracle "
                         f"(eq. 8 moments + eq. 9 contraction), {t_cpu:.1f}s"}
        err = {"max_rel": float(np.max(rel)), "median_rel": float(np.median(rel)),
               "max_err_over_abs_terms": float(np.max(rel_abs)), "sample_pairs": k,
               "definition": "|U_gpu - U_oracle| / |U_oracle| (FP64 oracle, same centres and poses)"}
        log(f"bench: oracle sample {k} pairs in {t_cpu:.1f}s; max rel err {err['max_rel']:.2e}")

    tcm.tcm_plan_destroy(plan)
    tcm.tcm_plan_destroy(plan_s)
    ctx.close()
    del soa
    torch.cuda.empty_cache()
    serving = None
    if not args.no_serve:
        t_s = time.time()
        serving = serving_section(tcm, synth, torch, nreq=args.serve_requests, inflight=args.serve_inflight,
                                  batch=args.serve_batch, check=not args.no_cpu)
        log(f"bench: serving section in {time.time() - t_s:.1f}s: "
            f"saturation {serving['saturation_pairs_per_s']:.0f} pairs/s, open loop {serving['open_loop']}")

    scan = None
    if not args.no_scan:
        t_s = time.time()
        scan = scan_section(tcm, synth, torch, check=not args.no_cpu)
        log(f"bench: scan section in {time.time() - t_s:.1f}s: {scan['positions_per_s']:.3e} positions/s, "
            f"{scan['speedup_vs_pair_path']:.0f}x the pair path, err {scan['max_err_over_abs_terms_vs_oracle']}")

    all_pairs = None
    if not args.no_all_pairs:
        t_s = time.time()
        all_pairs = all_pairs_section(tcm, synth)
        log(f"bench: all-pairs section in {time.time() - t_s:.1f}s: {all_pairs['pairs']} pairs, first call "
            f"{all_pairs['first_call_ms']:.1f} ms, recompute {all_pairs['recompute_call_ms']:.1f} ms, "
            f"reuse {all_pairs['reuse_call_ms']:.1f} ms "
            f"({all_pairs['pairs_per_s_reuse']:.3e} pairs/s)")

    forces = None
    if not args.no_forces:
        t_s = time.time()
        forces = forces_section(tcm, synth, torch)
        log(f"bench: forces section in {time.time() - t_s:.1f}s: per-atom {forces['per_atom']['ms_per_call']:.3f} ms "
            f"for {forces['per_atom']['atoms']} atoms; batch {forces['batch']['pairs']} pairs in "
            f"{forces['batch']['ms']:.2f} ms (energy only {forces['batch']['energy_only_ms']:.2f} ms)")

    adaptive = None
    if not args.no_adaptive:
        t_s = time.time()
        adaptive = adaptive_section(tcm, synth)
        log(f"bench: adaptive section in {time.time() - t_s:.1f}s: fixed L {adaptive['fixed_L']['ms']:.2f} ms; " +
            "; ".join(f"tol {k}: {v['ms']:.2f} ms (same orders given {v['batch_at_chosen_orders_ms']:.2f} ms), "
                      f"mean L {v['L_used']['mean']:.1f}, "
                      f"diff/bounds {v['max_diff_over_bounds']:.2e}" for k, v in adaptive["adaptive"].items()))

    single = None
    if not args.no_single:
        t_s = time.time()
        single = single_pair_section(tcm, synth, check=not args.no_cpu)
        log(f"bench: single-pair section in {time.time() - t_s:.1f}s: recomputed p50 "
            f"{single['moments_recomputed']['p50_ms']:.3f} ms p99 {single['moments_recomputed']['p99_ms']:.3f} ms; "
            f"resident p50 {single['resident_moments']['p50_ms']:.3f} ms p99 {single['resident_moments']['p99_ms']:.3f} ms; "
            f"rel err vs oracle {single['rel_err_vs_oracle']}")

    out = {
        "metric": "pair energies/s & p50/p99 latency at stated rel. err vs FP64 oracle",
        "value": args.npairs / (ms_step * 1e-3),
        "unit": "pair energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "uneven_batch", "npairs": args.npairs, "atoms": ntot,
                   "fragment_atoms": "log-uniform 1e3..2e5", "L": "uniform in {8,12,16,20}",
                   "geometry": "excluded-volume random-walk chains, q~N(0,0.3) zero net charge, "
                               "R0 = 1.5(a_A+a_B), random pose of B",
                   "precision": "moments FP32 compensated; rotation, geometric factors, contraction FP64",
                   "execution": ("one HIP graph replay per step (serial order: one statistics launch, "
                                 "centre/scale, one tile launch per L, moment finalisation, pair "
                                 "kernel)" if mode == "graph" else
                                 "direct launches per step: one statistics launch, centre/scale, the per-L "
                                 "tile launches on two streams balanced by work, moment finalisation, pair "
                                 "kernel"),
                   "ms_per_step_graph": ms_graph, "ms_per_step_streams": ms_streams,
                   "tile_autotune": tuned,
                   "parallelism": "single GPU", "seed": 4},
        "latency_ms": {"p50": ms_step, "p99": ms_step,
                       "note": "all pairs of a batch complete together at the end of the replay"},
        "rel_err": err,
        "phase_ms": {"stats": ph[0], "moment_tiles": ph[1], "moment_finalise": ph[2], "pairs": ph[3]},
        "roofline": {"bound": "alu", "achieved": moment_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": moment_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_tile_traffic(),
                     "kernel": "moment-pass tile kernels (FP32), 6(L+1)(L+2) flops per atom; achieved and "
                               "traffic are per step (one launch of tcm_tiles<float, L> per order L)",
                     "measured_plain_fp32_fma_tflops": fp32_ceiling},
        "cpu_baseline": cpu,
        "serving": serving,
        "scan": scan,
        "all_pairs": all_pairs,
        "forces": forces,
        "adaptive": adaptive,
        "single_pair": single,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
