"""ctypes binding of libtcm (include/tcm.h): the same entry points, argument marshalling only.

Every computation runs in the HIP kernels of libtcm.so; there is no CPU fallback.  Loading
fails loudly if the library has not been built (python -m paper_0704_1672_amd.build, or
__graft_entry__.build()).  PyTorch is used only to hand device memory and streams over:
functions taking device buffers accept torch CUDA tensors (or raw addresses).
"""
import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "tcm.h")

TCM_OK, TCM_EINVAL, TCM_EDOMAIN, TCM_ENOMEM, TCM_EDEVICE, TCM_EAGAIN, TCM_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
TCM_LMAX = 32
TCM_F64, TCM_F32C = 0, 1
TCM_UNCHECKED, TCM_REUSE, TCM_HOST_ATOMS, TCM_BORROW_ATOMS, TCM_DEVICE_IO, TCM_TRIANGULAR = 1, 2, 4, 8, 16, 32

_dp = C.POINTER(C.c_double)
_ip32 = C.POINTER(C.c_int32)
_ip64 = C.POINTER(C.c_int64)
_vp = C.c_void_p


class tcm_pair_req(C.Structure):
    _fields_ = [("a", C.c_int64), ("b", C.c_int64), ("R", C.c_double * 3), ("quat_b", C.c_double * 4),
                ("L", C.c_int32), ("flags", C.c_int32)]


class tcm_request(C.Structure):
    _fields_ = [("key_a", C.c_int64), ("key_b", C.c_int64), ("atoms_a", _vp * 4), ("n_a", C.c_int64),
                ("atoms_b", _vp * 4), ("n_b", C.c_int64), ("R", C.c_double * 3),
                ("quat_b", C.c_double * 4), ("L", C.c_int32), ("flags", C.c_int32),
                ("precision", C.c_int32), ("pad", C.c_int32)]


class tcm_server_cfg(C.Structure):
    _fields_ = [("max_inflight_batches", C.c_int32), ("max_batch_pairs", C.c_int32),
                ("queue_capacity", C.c_int32), ("pad", C.c_int32)]


PAIR_REQ_DTYPE = np.dtype([("a", np.int64), ("b", np.int64), ("R", np.float64, 3), ("quat_b", np.float64, 4),
                           ("L", np.int32), ("flags", np.int32)])
assert PAIR_REQ_DTYPE.itemsize == C.sizeof(tcm_pair_req)

_SIGS = {
    "tcm_strerror": (C.c_char_p, [C.c_int]),
    "tcm_create": (C.c_int, [C.POINTER(_vp), C.c_int, C.c_size_t, C.c_int]),
    "tcm_destroy": (None, [_vp]),
    "tcm_set_stream": (C.c_int, [_vp, _vp]),
    "tcm_get_stream": (_vp, [_vp]),
    "tcm_mem_info": (C.c_int, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "tcm_set_budget": (C.c_int, [_vp, C.c_size_t]),
    "tcm_moments": (C.c_int, [_vp, _dp, _dp, C.c_int64, _dp, C.c_int, C.c_int, _dp, _dp, _dp]),
    "tcm_moments_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int64, _dp, C.c_int, C.c_int, _vp, _vp]),
    "tcm_pair_energy": (C.c_int, [_vp, _dp, C.c_double, _dp, C.c_double, _dp, _dp, C.c_int, C.c_int, _dp]),
    "tcm_mol_upload": (C.c_int, [_vp, _dp, _dp, C.c_int64, _dp, C.c_int, _ip64]),
    "tcm_mol_register_device": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int64, _dp, C.c_int, _ip64]),
    "tcm_mol_release": (C.c_int, [_vp, C.c_int64]),
    "tcm_mol_moments": (C.c_int, [_vp, C.c_int64, C.c_int, C.c_int, _dp, _dp, _dp]),
    "tcm_batch_energy": (C.c_int, [_vp, _vp, C.c_int64, _dp, _ip32]),
    "tcm_plan_create": (C.c_int, [_vp, _vp, C.c_int64, C.c_int, C.POINTER(_vp)]),
    "tcm_plan_create_adaptive": (C.c_int, [_vp, _vp, C.c_int64, C.c_double, C.c_int, C.POINTER(_vp)]),
    "tcm_plan_orders": (C.c_int, [_vp, _vp, _ip32, _dp]),
    "tcm_plan_run": (C.c_int, [_vp, _vp]),
    "tcm_plan_run_phased": (C.c_int, [_vp, _vp]),
    "tcm_plan_run_timed": (C.c_int, [_vp, _vp, _dp]),
    "tcm_plan_results": (C.c_int, [_vp, _vp, _dp, _ip32]),
    "tcm_plan_device_outputs": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp)]),
    "tcm_plan_info": (C.c_int, [_vp, _ip64, _dp, _ip64, _ip64]),
    "tcm_plan_destroy": (None, [_vp]),
    "tcm_tune_get": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int64, _ip32]),
    "tcm_tune_set": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int64, C.c_int]),
    "tcm_set_fp32_run": (C.c_int, [_vp, C.c_int]),
    "tcm_autotune": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int64, _ip32, _dp]),
    "tcm_autotune_batch": (C.c_int, [_vp, _vp, C.c_int64, _dp]),
    "tcm_scan_translations": (C.c_int, [_vp, C.c_int64, C.c_int64, C.c_int, _dp, C.c_int, _dp, C.c_int64, _dp,
                                        _ip32]),
    "tcm_all_pairs": (C.c_int, [_vp, _ip64, C.c_int64, C.c_int, C.c_int, _dp, _ip32]),
    "tcm_pair_forces": (C.c_int, [_vp, C.c_int64, C.c_int64, _dp, _dp, C.c_int, C.c_int, _dp, _dp, _dp]),
    "tcm_batch_forces": (C.c_int, [_vp, _vp, C.c_int64, _dp, _ip32]),
    "tcm_batch_energy_adaptive": (C.c_int, [_vp, _vp, C.c_int64, C.c_double, _dp, _ip32, _dp, _ip32]),
    "tcm_alu_calibrate": (C.c_int, [_vp, C.c_int, _dp]),
    "tcm_tune_save": (C.c_int, [_vp, C.c_char_p]),
    "tcm_tune_load": (C.c_int, [_vp, C.c_char_p]),
    "tcm_server_start": (C.c_int, [_vp, C.POINTER(tcm_server_cfg)]),
    "tcm_submit": (C.c_int, [_vp, C.POINTER(tcm_request), C.POINTER(C.c_uint64)]),
    "tcm_poll": (C.c_int, [_vp, C.c_uint64, _dp, _ip32, _dp]),
    "tcm_server_stop": (C.c_int, [_vp]),
    "tcm_server_stats": (C.c_int, [_vp, _ip64, _ip64, _ip64, _ip64, _ip64, _ip64, _ip64, _ip64]),
}

_lib = None


def lib():
    """The loaded libtcm.so (raises if it was never built)."""
    global _lib
    if _lib is None:
        try:
            # one HIP runtime per process: importing torch first loads its runtime, which the
            # library then binds to (same soname) instead of loading a second copy
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtcm.so not found at {LIB_PATH}: build it first "
                               "(python -m paper_0704_1672_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols():
    """Names of every function declared in include/tcm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcm_[a-z_0-9]+)\s*\(", text)))


class TCMError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {lib().tcm_strerror(code).decode()} ({code})")


def _check(rc, what):
    if rc != TCM_OK:
        raise TCMError(rc, what)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _addr(t):
    """Device address of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def nh(L):
    return (L + 1) * (L + 1)


# ---- thin wrappers with the C names ------------------------------------------------
def tcm_strerror(code):
    return lib().tcm_strerror(code).decode()


def tcm_create(device=0, hbm_budget_bytes=0, flags=0):
    h = _vp()
    _check(lib().tcm_create(C.byref(h), device, hbm_budget_bytes, flags), "tcm_create")
    return h.value


def tcm_destroy(ctx):
    lib().tcm_destroy(ctx)


def tcm_set_stream(ctx, stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t address, or None."""
    s = getattr(stream, "cuda_stream", stream)
    _check(lib().tcm_set_stream(ctx, s), "tcm_set_stream")


def tcm_get_stream(ctx):
    return lib().tcm_get_stream(ctx)


def tcm_mem_info(ctx):
    u, b = C.c_size_t(), C.c_size_t()
    _check(lib().tcm_mem_info(ctx, C.byref(u), C.byref(b)), "tcm_mem_info")
    return u.value, b.value


def tcm_set_budget(ctx, budget):
    _check(lib().tcm_set_budget(ctx, int(budget)), "tcm_set_budget")


def tcm_moments(ctx, coords, charges, L, precision=TCM_F64, centre=None):
    """eq. (8): returns (Q packed (L+1)^2, radius, centre)."""
    x = _f64(coords, (-1, 3))
    q = _f64(charges, (-1,))
    c = _f64(centre, (3,)) if centre is not None else None
    Q = np.empty(nh(L))
    r = C.c_double()
    co = np.empty(3)
    _check(lib().tcm_moments(ctx, _p(x), _p(q), len(q), _p(c), L, precision, _p(Q), C.byref(r), _p(co)),
           "tcm_moments")
    return Q, r.value, co


def tcm_pair_energy(ctx, QA, aA, QB, aB, R, L, quat_b=None, flags=0):
    qa, qb = _f64(QA), _f64(QB)
    if len(qa) < nh(L) or len(qb) < nh(L):
        raise ValueError("moment tables shorter than (L+1)^2")
    Rv = _f64(R, (3,))
    qt = _f64(quat_b, (4,)) if quat_b is not None else None
    U = C.c_double()
    _check(lib().tcm_pair_energy(ctx, _p(qa), float(aA), _p(qb), float(aB), _p(Rv), _p(qt), L, flags, C.byref(U)),
           "tcm_pair_energy")
    return U.value


def tcm_mol_upload(ctx, coords, charges, centre=None, precision=TCM_F32C):
    x = _f64(coords, (-1, 3))
    q = _f64(charges, (-1,))
    c = _f64(centre, (3,)) if centre is not None else None
    mid = C.c_int64()
    _check(lib().tcm_mol_upload(ctx, _p(x), _p(q), len(q), _p(c), precision, C.byref(mid)), "tcm_mol_upload")
    return mid.value


def tcm_moments_noalloc(ctx, x, y, z, q, n, centre, L, precision, Q, meta):
    """eq. (8) without allocation: device atoms (x, y, z, q), device outputs Q ((L+1)^2) and
    meta (8: centre, radius, scale); queued on the context's stream."""
    c = _f64(centre, (3,)) if centre is not None else None
    _check(lib().tcm_moments_noalloc(ctx, _addr(x), _addr(y), _addr(z), _addr(q), int(n), _p(c), int(L),
                                     int(precision), _addr(Q), _addr(meta)), "tcm_moments_noalloc")


def tcm_mol_register_device(ctx, x, y, z, q, n, centre=None, precision=TCM_F32C):
    c = _f64(centre, (3,)) if centre is not None else None
    mid = C.c_int64()
    _check(lib().tcm_mol_register_device(ctx, _addr(x), _addr(y), _addr(z), _addr(q), int(n), _p(c), precision,
                                         C.byref(mid)), "tcm_mol_register_device")
    return mid.value


def tcm_mol_release(ctx, mid):
    _check(lib().tcm_mol_release(ctx, mid), "tcm_mol_release")


def tcm_mol_moments(ctx, mid, L, flags=0):
    Q = np.empty(nh(L))
    r = C.c_double()
    co = np.empty(3)
    _check(lib().tcm_mol_moments(ctx, mid, L, flags, _p(Q), C.byref(r), _p(co)), "tcm_mol_moments")
    return Q, r.value, co


def make_requests(a, b, R, L, quat_b=None, flags=0):
    """Array of tcm_pair_req from per-pair arrays; scalars and single rows broadcast to the
    longest input."""
    a = np.atleast_1d(np.asarray(a, dtype=np.int64))
    b = np.atleast_1d(np.asarray(b, dtype=np.int64))
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    L = np.atleast_1d(np.asarray(L, dtype=np.int32))
    Q = None if quat_b is None else np.asarray(quat_b, dtype=np.float64).reshape(-1, 4)
    flags = np.atleast_1d(np.asarray(flags, dtype=np.int32))
    n = max(len(a), len(b), len(R), len(L), len(flags), 0 if Q is None else len(Q))
    req = np.zeros(n, dtype=PAIR_REQ_DTYPE)
    req["a"] = np.broadcast_to(a, (n,))
    req["b"] = np.broadcast_to(b, (n,))
    req["R"] = np.broadcast_to(R, (n, 3))
    if Q is None:
        req["quat_b"][:, 0] = 1.0
    else:
        req["quat_b"] = np.broadcast_to(Q, (n, 4))
    req["L"] = np.broadcast_to(L, (n,))
    req["flags"] = np.broadcast_to(flags, (n,))
    return req


def tcm_batch_energy(ctx, reqs):
    """Returns (U[n], status[n], rc)."""
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    n = len(reqs)
    U = np.empty(max(n, 1))
    st = np.empty(max(n, 1), dtype=np.int32)
    rc = lib().tcm_batch_energy(ctx, reqs.ctypes.data if n else None, n, _p(U),
                                st.ctypes.data_as(_ip32))
    if rc in (TCM_EINVAL, TCM_ENOMEM, TCM_EDEVICE) and n and np.all(st[:n] == 0):
        raise TCMError(rc, "tcm_batch_energy")
    return U[:n], st[:n], rc


def tcm_plan_create(ctx, reqs, use_graph=True):
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    h = _vp()
    _check(lib().tcm_plan_create(ctx, reqs.ctypes.data if len(reqs) else None, len(reqs), int(use_graph),
                                 C.byref(h)), "tcm_plan_create")
    return h.value


def tcm_plan_run(ctx, plan):
    _check(lib().tcm_plan_run(ctx, plan), "tcm_plan_run")


def tcm_plan_run_phased(ctx, plan):
    _check(lib().tcm_plan_run_phased(ctx, plan), "tcm_plan_run_phased")


def tcm_plan_run_timed(ctx, plan):
    """Synchronous run; returns the (stats, tiles, finalise, pairs) kernel times in ms."""
    ms = np.zeros(4)
    _check(lib().tcm_plan_run_timed(ctx, plan, _p(ms)), "tcm_plan_run_timed")
    return ms


def tcm_plan_create_adaptive(ctx, reqs, tol, use_graph=True):
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    h = _vp()
    _check(lib().tcm_plan_create_adaptive(ctx, reqs.ctypes.data if len(reqs) else None, len(reqs), float(tol),
                                          int(use_graph), C.byref(h)), "tcm_plan_create_adaptive")
    return h.value


def tcm_plan_orders(ctx, plan, n):
    """Chosen orders and their bounds of an adaptive plan's last run."""
    Lc = np.empty(max(n, 1), dtype=np.int32)
    b = np.empty(max(n, 1))
    _check(lib().tcm_plan_orders(ctx, plan, Lc.ctypes.data_as(_ip32), _p(b)), "tcm_plan_orders")
    return Lc[:n], b[:n]


def tcm_plan_results(ctx, plan, n):
    U = np.empty(max(n, 1))
    st = np.empty(max(n, 1), dtype=np.int32)
    _check(lib().tcm_plan_results(ctx, plan, _p(U), st.ctypes.data_as(_ip32)), "tcm_plan_results")
    return U[:n], st[:n]


def tcm_plan_device_outputs(plan):
    u, s = _vp(), _vp()
    _check(lib().tcm_plan_device_outputs(plan, C.byref(u), C.byref(s)), "tcm_plan_device_outputs")
    return u.value, s.value


def tcm_plan_info(plan):
    a, t, p = C.c_int64(), C.c_int64(), C.c_int64()
    f = C.c_double()
    _check(lib().tcm_plan_info(plan, C.byref(a), C.byref(f), C.byref(t), C.byref(p)), "tcm_plan_info")
    return dict(atoms=a.value, moment_flops=f.value, tiles=t.value, pairs=p.value)


def tcm_plan_destroy(plan):
    lib().tcm_plan_destroy(plan)


def tcm_tune_get(ctx, precision, L, n):
    k = C.c_int32()
    _check(lib().tcm_tune_get(ctx, precision, L, n, C.byref(k)), "tcm_tune_get")
    return k.value


def tcm_tune_set(ctx, precision, L, n, kper):
    _check(lib().tcm_tune_set(ctx, precision, L, n, kper), "tcm_tune_set")


def tcm_set_fp32_run(ctx, kmax):
    _check(lib().tcm_set_fp32_run(ctx, int(kmax)), "tcm_set_fp32_run")


def tcm_autotune(ctx, precision, L, n):
    k = C.c_int32()
    ms = C.c_double()
    _check(lib().tcm_autotune(ctx, precision, L, n, C.byref(k), C.byref(ms)), "tcm_autotune")
    return k.value, ms.value


def tcm_autotune_batch(ctx, reqs):
    """Returns the sum of the groups' best tile times (ms)."""
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    ms = C.c_double()
    _check(lib().tcm_autotune_batch(ctx, reqs.ctypes.data if len(reqs) else None, len(reqs), C.byref(ms)),
           "tcm_autotune_batch")
    return ms.value


def tcm_scan_translations(ctx, a, b, L, R, quat_b=None, flags=0):
    """Energies of B at the positions R ([n][3], c_B - c_A) with one pose of B; returns
    (U[n], status[n]).  Host arrays (TCM_DEVICE_IO is for callers passing device addresses
    through the C ABI)."""
    R = _f64(R, (-1, 3))
    n = len(R)
    U = np.empty(max(n, 1))
    st = np.empty(max(n, 1), dtype=np.int32)
    q = _f64(quat_b, (4,)) if quat_b is not None else None
    _check(lib().tcm_scan_translations(ctx, int(a), int(b), int(L), _p(q), int(flags), _p(R), n, _p(U),
                                       st.ctypes.data_as(_ip32)), "tcm_scan_translations")
    return U[:n], st[:n]


def tcm_all_pairs(ctx, ids, L, flags=0):
    """Energies of every pair (i < j) of the resident fragments ids at their own positions;
    returns (U, status), each K(K-1)/2 long in row-major upper-triangle order."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    K = len(ids)
    n = K * (K - 1) // 2
    U = np.empty(max(n, 1))
    st = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib().tcm_all_pairs(ctx, ids.ctypes.data_as(_ip64), K, int(L), int(flags), _p(U), st.ctypes.data_as(_ip32))
    if rc in (TCM_EINVAL, TCM_ENOMEM, TCM_EDEVICE, TCM_ENOTFOUND) and np.all(st[:n] == 0):
        raise TCMError(rc, "tcm_all_pairs")
    return U[:n], st[:n]


def tcm_pair_forces(ctx, a, b, R, L, quat_b=None, flags=0, atoms=False, nA=0, nB=0):
    """Returns dict(U, F_B, tau_A, tau_B) and, with atoms=True, the per-atom forces FA[nA][3],
    FB[nB][3] (host arrays; nA, nB the molecules' atom counts).  Raises TCMError on failure
    (its code is the pair's status, e.g. TCM_EDOMAIN)."""
    R = _f64(R, (3,))
    q = _f64(quat_b, (4,)) if quat_b is not None else None
    out = np.empty(10)
    FA = np.empty((max(nA, 1), 3)) if atoms else None
    FB = np.empty((max(nB, 1), 3)) if atoms else None
    _check(lib().tcm_pair_forces(ctx, int(a), int(b), _p(R), _p(q), int(L), int(flags), _p(out),
                                 _p(FA) if atoms else None, _p(FB) if atoms else None), "tcm_pair_forces")
    res = dict(U=out[0], F_B=out[1:4].copy(), tau_A=out[4:7].copy(), tau_B=out[7:10].copy())
    if atoms:
        res["FA"], res["FB"] = FA[:nA], FB[:nB]
    return res


def tcm_alu_calibrate(ctx, precision):
    t = C.c_double()
    _check(lib().tcm_alu_calibrate(ctx, int(precision), C.byref(t)), "tcm_alu_calibrate")
    return t.value


def tcm_batch_energy_adaptive(ctx, reqs, tol):
    """Returns (U[n], L_used[n], bound[n], status[n], rc); each request's L is its maximum."""
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    n = len(reqs)
    U = np.empty(max(n, 1))
    Lu = np.empty(max(n, 1), dtype=np.int32)
    b = np.empty(max(n, 1))
    st = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib().tcm_batch_energy_adaptive(ctx, reqs.ctypes.data if n else None, n, float(tol), _p(U),
                                         Lu.ctypes.data_as(_ip32), _p(b), st.ctypes.data_as(_ip32))
    if rc in (TCM_EINVAL, TCM_ENOMEM, TCM_EDEVICE) and (n == 0 or np.all(st[:n] == 0)):
        raise TCMError(rc, "tcm_batch_energy_adaptive")
    return U[:n], Lu[:n], b[:n], st[:n], rc


def tcm_batch_forces(ctx, reqs):
    """Returns (out[n][10] = (U, F_B, tau_A, tau_B), status[n], rc)."""
    reqs = np.ascontiguousarray(reqs, dtype=PAIR_REQ_DTYPE)
    n = len(reqs)
    out = np.empty((max(n, 1), 10))
    st = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib().tcm_batch_forces(ctx, reqs.ctypes.data if n else None, n, _p(out), st.ctypes.data_as(_ip32))
    if rc in (TCM_EINVAL, TCM_ENOMEM, TCM_EDEVICE) and n and np.all(st[:n] == 0):
        raise TCMError(rc, "tcm_batch_forces")
    return out[:n], st[:n], rc


def pair_index(i, j, K):
    """Index of pair (i, j), i < j, in tcm_all_pairs' output."""
    return i * K - i * (i + 1) // 2 + (j - i - 1)


def tcm_tune_save(ctx, path):
    _check(lib().tcm_tune_save(ctx, path.encode()), "tcm_tune_save")


def tcm_tune_load(ctx, path):
    return lib().tcm_tune_load(ctx, path.encode())


def tcm_server_start(ctx, max_inflight_batches=2, max_batch_pairs=64, queue_capacity=4096):
    cfg = tcm_server_cfg(max_inflight_batches, max_batch_pairs, queue_capacity, 0)
    _check(lib().tcm_server_start(ctx, C.byref(cfg)), "tcm_server_start")


def tcm_submit(ctx, req):
    t = C.c_uint64()
    rc = lib().tcm_submit(ctx, C.byref(req), C.byref(t))
    return rc, t.value


def tcm_poll(ctx, ticket):
    U = C.c_double()
    st = C.c_int32()
    lat = C.c_double()
    rc = lib().tcm_poll(ctx, ticket, C.byref(U), C.byref(st), C.byref(lat))
    return rc, U.value, st.value, lat.value


def tcm_server_stop(ctx):
    _check(lib().tcm_server_stop(ctx), "tcm_server_stop")


def tcm_server_stats(ctx):
    v = [C.c_int64() for _ in range(8)]
    _check(lib().tcm_server_stats(ctx, *[C.byref(x) for x in v]), "tcm_server_stats")
    return dict(zip(["completed", "launches", "cache_hits", "cache_misses", "deferred", "evictions", "dropped",
                     "evicted_misses"], [x.value for x in v]))


def make_request(key_a, key_b, R, L, quat_b=(1.0, 0.0, 0.0, 0.0), atoms_a=None, n_a=0, atoms_b=None, n_b=0,
                 flags=0, precision=TCM_F32C):
    """tcm_request; atoms_* are 4 device addresses (x, y, z, q) or None for a resident fragment."""
    r = tcm_request()
    r.key_a, r.key_b = int(key_a), int(key_b)
    if atoms_a is not None:
        for i in range(4):
            r.atoms_a[i] = int(atoms_a[i])
    r.n_a = int(n_a)
    if atoms_b is not None:
        for i in range(4):
            r.atoms_b[i] = int(atoms_b[i])
    r.n_b = int(n_b)
    for i in range(3):
        r.R[i] = float(R[i])
    for i in range(4):
        r.quat_b[i] = float(quat_b[i])
    r.L, r.flags, r.precision = int(L), int(flags), int(precision)
    return r


class Context:
    """Owns a tcm_ctx; thin convenience over the functions above."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        self.h = tcm_create(device, hbm_budget_bytes)

    def close(self):
        if self.h:
            tcm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
