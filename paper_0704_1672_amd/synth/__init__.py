"""Seeded synthetic inputs for the two-centre multipole workloads.

This module holds no arithmetic of the multipole method (no harmonics, moments or
energies): random numbers from synth.c and the geometry recipes that place charges.  It
imports nothing else from the package, so the FP64 oracle's tests and the HIP path's tests
can both use it without either importing the other.

Workload recipes (the paper's own workloads are random-charge spheres and the 1AVW
protein pair, whose structure and charges are not available; these stand in for them):
  ball_pair     two charge balls, q ~ U[-1, 1], centres a fixed distance apart
  chain_pair    two excluded-volume random-walk chains, q ~ N(0, 0.3) with zero net charge
  orientation_scan  two balls, many random poses of B (quaternion + distance)
  uneven_batch  many chain pairs of log-uniform sizes and mixed orders
  serving_trace a fragment pool plus a Poisson request trace
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int64)


def build(verbose=False):
    src = os.path.join(_HERE, "synth.c")
    out = os.path.join(_HERE, "libtcmsynth.so")
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall", "-o", out,
           src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libtcmsynth.so")
        if not os.path.exists(path):
            build()
        lib = C.CDLL(path)
        u64, i64 = C.c_uint64, C.c_int64
        lib.synth_uniform.argtypes = [u64, u64, i64, C.c_double, C.c_double, _dp]
        lib.synth_normal.argtypes = [u64, u64, i64, C.c_double, C.c_double, _dp]
        lib.synth_unit_vectors.argtypes = [u64, u64, i64, _dp]
        lib.synth_quaternions.argtypes = [u64, u64, i64, _dp]
        lib.synth_ball.argtypes = [u64, u64, i64, C.c_double, _dp, C.c_double, C.c_double, _dp, _dp]
        lib.synth_chain.argtypes = [u64, u64, i64, C.c_double, C.c_double, C.c_int, C.c_double,
                                    _dp, _dp]
        lib.synth_chain.restype = i64
        lib.synth_chains.argtypes = [u64, u64, i64, _ip, _ip, C.c_double, C.c_double, C.c_int,
                                     C.c_double, C.c_int, _dp, _dp, _ip]
        lib.synth_chains.restype = C.c_int
        _LIB = lib
    return _LIB


def _p(a):
    return a.ctypes.data_as(_dp)


# ---- primitive streams ------------------------------------------------------------
def uniform(seed, stream, n, lo=0.0, hi=1.0):
    out = np.empty(int(n))
    _lib().synth_uniform(seed, stream, int(n), lo, hi, _p(out))
    return out


def normal(seed, stream, n, mu=0.0, sigma=1.0):
    out = np.empty(int(n))
    _lib().synth_normal(seed, stream, int(n), mu, sigma, _p(out))
    return out


def unit_vectors(seed, stream, n):
    out = np.empty((int(n), 3))
    _lib().synth_unit_vectors(seed, stream, int(n), _p(out))
    return out


def quaternions(seed, stream, n):
    out = np.empty((int(n), 4))
    _lib().synth_quaternions(seed, stream, int(n), _p(out))
    return out


def ball(seed, stream, n, R, centre=(0.0, 0.0, 0.0), qlo=-1.0, qhi=1.0):
    xyz = np.empty((int(n), 3))
    q = np.empty(int(n))
    c = np.ascontiguousarray(centre, dtype=np.float64)
    _lib().synth_ball(seed, stream, int(n), R, _p(c), qlo, qhi, _p(xyz), _p(q))
    return xyz, q


def chain(seed, stream, n, step=1.5, excl=1.2, max_trials=100, sigma=0.3):
    xyz = np.empty((int(n), 3))
    q = np.empty(int(n))
    v = _lib().synth_chain(seed, stream, int(n), step, excl, max_trials, sigma, _p(xyz), _p(q))
    if v < 0:
        raise MemoryError("synth_chain: allocation failed")
    return xyz, q, int(v)


def chains(seed, stream0, counts, step=1.5, excl=1.2, max_trials=100, sigma=0.3, nthreads=None):
    """Many chains generated in parallel; returns (xyz[sum n,3], q[sum n], offsets, violations)."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    offsets = np.zeros(len(counts) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    xyz = np.empty((int(offsets[-1]), 3))
    q = np.empty(int(offsets[-1]))
    viol = np.zeros(len(counts), dtype=np.int64)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    rc = _lib().synth_chains(seed, stream0, len(counts), counts.ctypes.data_as(_ip),
                             offsets.ctypes.data_as(_ip), step, excl, max_trials, sigma,
                             int(nthreads), _p(xyz), _p(q), viol.ctypes.data_as(_ip))
    if rc != 0:
        raise MemoryError("synth_chains: allocation failed")
    return xyz, q, offsets, viol


# ---- geometry helpers used only to place molecules -----------------------------------
def centroid(xyz):
    return np.asarray(xyz, dtype=np.float64).mean(axis=0)


def max_extent(xyz, c):
    return float(np.sqrt(((np.asarray(xyz) - c) ** 2).sum(axis=1)).max()) if len(xyz) else 0.0


def radius_of_gyration(xyz):
    c = centroid(xyz)
    return float(np.sqrt(((np.asarray(xyz) - c) ** 2).sum(axis=1).mean()))


def log_uniform_counts(seed, stream, n, lo, hi):
    u = uniform(seed, stream, n)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


# ---- workload recipes ------------------------------------------------------------------
def ball_pair(seed=1, n=500, radius=10.0, distance=60.0, L=10):
    """Two balls of n charges (q ~ U[-1,1]) of the given radius; centres `distance` apart
    along a random unit vector.  The centres are the ball centres."""
    u = unit_vectors(seed, 0, 1)[0]
    cA = np.zeros(3)
    cB = distance * u
    xyzA, qA = ball(seed, 1, n, radius, cA)
    xyzB, qB = ball(seed, 2, n, radius, cB)
    return dict(xyzA=xyzA, qA=qA, cA=cA, xyzB=xyzB, qB=qB, cB=cB, L=L, R=cB - cA)


def chain_pair(seed=2, n=100_000, nsep=16, smin=2.0, smax=10.0, Ls=(8, 16, 24)):
    """Two chains of n beads (1.5 A steps, 1.2 A exclusion, q ~ N(0, 0.3), net charge
    zeroed).  Separations d_k = s_k * (Rg_A + Rg_B)/2, s_k = linspace(smin, smax, nsep),
    along one random direction; A is centred on its centroid at the origin."""
    xyzA, qA, vA = chain(seed, 1, n)
    xyzB, qB, vB = chain(seed, 2, n)
    xyzA = xyzA - centroid(xyzA)
    xyzB = xyzB - centroid(xyzB)
    rg = 0.5 * (radius_of_gyration(xyzA) + radius_of_gyration(xyzB))
    u = unit_vectors(seed, 3, 1)[0]
    s = np.linspace(smin, smax, nsep)
    return dict(xyzA=xyzA, qA=qA, xyzB_body=xyzB, qB=qB, rg=rg, s=s, dirs=u,
                seps=[si * rg * u for si in s], Ls=list(Ls), violations=(vA, vB))


def orientation_scan(seed=3, n=50_000, nposes=4096, L=16, density_ref=(500, 10.0)):
    """Two balls at the number density of `density_ref` (n0 charges in radius r0), q ~ U[-1,1];
    nposes random poses of B: uniform quaternion, distance U[3, 6] * Rg with Rg the ball's
    radius of gyration sqrt(3/5) * radius, random direction."""
    n0, r0 = density_ref
    radius = r0 * (n / n0) ** (1.0 / 3.0)
    xyzA, qA = ball(seed, 1, n, radius)
    xyzB, qB = ball(seed, 2, n, radius)
    rg = math.sqrt(3.0 / 5.0) * radius
    quats = quaternions(seed, 3, nposes)
    dist = uniform(seed, 4, nposes, 3.0 * rg, 6.0 * rg)
    dirs = unit_vectors(seed, 5, nposes)
    return dict(xyzA=xyzA, qA=qA, xyzB=xyzB, qB=qB, radius=radius, rg=rg, quats=quats,
                R=dist[:, None] * dirs, L=L, cA=np.zeros(3), cB=np.zeros(3))


def uneven_batch(seed=4, npairs=1024, nmin=1_000, nmax=200_000, Ls=(8, 12, 16, 20),
                 sep_factor=1.5, poses=True, nthreads=None):
    """npairs chain pairs; per fragment n ~ floor(exp U[ln nmin, ln nmax]); L per pair uniform
    in Ls; separation R0 = sep_factor * (a_A + a_B) along a random direction, a = max extent
    about the centroid (the paper's placement rule for its random-sphere tests); optional
    random orientation of B (uniform quaternion).  Fragment 2p is A of pair p, 2p+1 is B."""
    counts = log_uniform_counts(seed, 0, 2 * npairs, nmin, nmax)
    xyz, q, offsets, viol = chains(seed, 1000, counts, nthreads=nthreads)
    Lsel = np.asarray(Ls)[np.minimum((uniform(seed, 1, npairs) * len(Ls)).astype(int),
                                     len(Ls) - 1)]
    dirs = unit_vectors(seed, 2, npairs)
    quats = quaternions(seed, 3, npairs) if poses else np.tile([1.0, 0, 0, 0], (npairs, 1))
    ext = np.empty(2 * npairs)
    cen = np.empty((2 * npairs, 3))
    for f in range(2 * npairs):
        s = xyz[offsets[f]:offsets[f + 1]]
        cen[f] = centroid(s)
        ext[f] = max_extent(s, cen[f])
    R = np.array([sep_factor * (ext[2 * p] + ext[2 * p + 1]) * dirs[p] for p in range(npairs)])
    return dict(xyz=xyz, q=q, offsets=offsets, counts=counts, L=Lsel, R=R, quats=quats,
                extent=ext, violations=viol)


def serving_trace(seed=5, pool=64, nreq=10_000, nmin=1_000, nmax=1_000_000, Lmin=8, Lmax=24,
                  reuse=0.3, qps=1000.0, sep_factor=1.5, nthreads=None):
    """A pool of `pool` chain fragments (log-uniform nmin..nmax beads) and a Poisson trace of
    nreq pair requests at rate qps.  Each request draws L ~ U{Lmin..Lmax}; with probability
    `reuse` it reuses two resident fragments with a new pose, otherwise it names two pool
    fragments as newly arriving.  Returns the pool and per-request arrays."""
    counts = log_uniform_counts(seed, 0, pool, nmin, nmax)
    xyz, q, offsets, viol = chains(seed, 1000, counts, nthreads=nthreads)
    gaps = -np.log(1.0 - uniform(seed, 1, nreq)) / qps
    t = np.cumsum(gaps)
    pick = np.minimum((uniform(seed, 2, 2 * nreq) * pool).astype(np.int64), pool - 1)
    Lr = Lmin + np.minimum((uniform(seed, 3, nreq) * (Lmax - Lmin + 1)).astype(int), Lmax - Lmin)
    is_reuse = uniform(seed, 4, nreq) < reuse
    dirs = unit_vectors(seed, 5, nreq)
    quats = quaternions(seed, 6, nreq)
    ext = np.empty(pool)
    for f in range(pool):
        s = xyz[offsets[f]:offsets[f + 1]]
        ext[f] = max_extent(s, centroid(s))
    a, b = pick[0::2], pick[1::2]
    R = (sep_factor * (ext[a] + ext[b]))[:, None] * dirs
    return dict(xyz=xyz, q=q, offsets=offsets, counts=counts, t=t, a=a, b=b, L=Lr,
                reuse=is_reuse, R=R, quats=quats, extent=ext, violations=viol)
