"""ctypes wrapper around liboracle.so (tcm_oracle.c).  Test infrastructure only.

Every function takes and returns numpy arrays in FP64.  Complex moment tables use the
oracle's layout: complex index l*l + l + m, m in [-l, l].  `complex_to_packed` converts
to the library's real-packed m >= 0 layout (index l*l for m = 0, l*l + 2m - 1 / l*l + 2m
for Re / Im of m > 0) so tests can compare the two element by element.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = C.CDLL(path)
    lib.oracle_ylm.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp]
    lib.oracle_ylm.restype = C.c_int
    lib.oracle_threej.argtypes = [C.c_int] * 6
    lib.oracle_threej.restype = C.c_double
    lib.oracle_centroid.argtypes = [_dp, C.c_int64, _dp]
    lib.oracle_centroid.restype = C.c_int
    lib.oracle_radius.argtypes = [_dp, C.c_int64, _dp]
    lib.oracle_radius.restype = C.c_double
    lib.oracle_moments.argtypes = [_dp, _dp, C.c_int64, _dp, C.c_int, _dp, _dp]
    lib.oracle_moments.restype = C.c_int
    lib.oracle_energy.argtypes = [_dp, C.c_int, _dp, C.c_int, _dp, C.c_int, _dp, _dp, _dp, _dp]
    lib.oracle_energy.restype = C.c_int
    lib.oracle_energy_shape.argtypes = [_dp, C.c_int, _dp, C.c_int, _dp, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    lib.oracle_energy_shape.restype = C.c_int
    lib.oracle_energy_sensitivity.argtypes = [_dp, _dp, C.c_int, _dp, _dp, C.c_int, _dp, C.c_int, C.c_int, _dp]
    lib.oracle_energy_sensitivity.restype = C.c_int
    lib.oracle_trunc_bound_tri.argtypes = [C.c_double] * 5 + [C.c_int]
    lib.oracle_trunc_bound_tri.restype = C.c_double
    lib.oracle_coulomb.argtypes = [_dp, _dp, C.c_int64, _dp, _dp, C.c_int64]
    lib.oracle_coulomb.restype = C.c_double
    lib.oracle_pose.argtypes = [_dp, C.c_int64, _dp, _dp, _dp, _dp]
    lib.oracle_pose.restype = C.c_int
    lib.oracle_trunc_bound.argtypes = [C.c_double] * 5 + [C.c_int]
    lib.oracle_trunc_bound.restype = C.c_double
    lib.oracle_energy_grad.argtypes = [_dp, C.c_int, _dp, C.c_int, _dp, C.c_int, _dp]
    lib.oracle_energy_grad.restype = C.c_int
    lib.oracle_energy_coeffs.argtypes = [_dp, C.c_int, _dp, C.c_int, _dp, C.c_int, C.c_int, _dp]
    lib.oracle_energy_coeffs.restype = C.c_int
    lib.oracle_atom_forces.argtypes = [_dp, C.c_int, _dp, _dp, C.c_int64, _dp, _dp]
    lib.oracle_atom_forces.restype = C.c_int
    _LIB = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(_dp)


def ylm(l, m, theta, phi):
    re, im = C.c_double(), C.c_double()
    rc = load().oracle_ylm(l, m, float(theta), float(phi), C.byref(re), C.byref(im))
    if rc != 0:
        raise ValueError("oracle_ylm: bad arguments")
    return complex(re.value, im.value)


def threej(j1, j2, j3, m1, m2, m3):
    return load().oracle_threej(j1, j2, j3, m1, m2, m3)


def centroid(xyz):
    xyz = _f64(xyz, (-1, 3))
    c = np.zeros(3)
    if load().oracle_centroid(_p(xyz), len(xyz), _p(c)) != 0:
        raise ValueError("oracle_centroid: empty input")
    return c


def radius(xyz, c):
    xyz = _f64(xyz, (-1, 3))
    c = _f64(c, (3,))
    return load().oracle_radius(_p(xyz), len(xyz), _p(c))


def moments(xyz, q, c, L, with_abs=False):
    """eq. (8) about centre c; returns complex array of length (L+1)^2 (index l*l+l+m)."""
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q, (-1,))
    c = _f64(c, (3,))
    assert len(q) == len(xyz)
    out = np.zeros(2 * (L + 1) ** 2)
    qa = np.zeros((L + 1) ** 2) if with_abs else None
    rc = load().oracle_moments(_p(xyz), _p(q), len(q), _p(c), int(L), _p(out),
                               _p(qa) if with_abs else None)
    if rc != 0:
        raise ValueError(f"oracle_moments failed ({rc})")
    Q = out[0::2] + 1j * out[1::2]
    return (Q, qa) if with_abs else Q


def order_of(Q):
    L = int(round(np.sqrt(len(Q)))) - 1
    assert (L + 1) ** 2 == len(Q)
    return L


SQUARE, TRIANGULAR = 0, 1      # truncation shapes: l1, l2 <= L  /  l1 + l2 <= L


def energy(QA, QB, R, L, full=False, shape=SQUARE):
    """eq. (9) with square (l1, l2 <= L, default) or triangular (l1 + l2 <= L) truncation.
    Returns Re U (and diagnostics if full)."""
    QA = np.asarray(QA, dtype=np.complex128)
    QB = np.asarray(QB, dtype=np.complex128)
    LA, LB = order_of(QA), order_of(QB)
    qa = np.empty(2 * len(QA)); qa[0::2] = QA.real; qa[1::2] = QA.imag
    qb = np.empty(2 * len(QB)); qb[0::2] = QB.real; qb[1::2] = QB.imag
    R = _f64(R, (3,))
    ure, uim, asum = C.c_double(), C.c_double(), C.c_double()
    terms = np.zeros((L + 1) ** 2)
    if shape == SQUARE:
        rc = load().oracle_energy(_p(qa), LA, _p(qb), LB, _p(R), int(L), C.byref(ure), C.byref(uim),
                                  _p(terms), C.byref(asum))
    else:
        rc = load().oracle_energy_shape(_p(qa), LA, _p(qb), LB, _p(R), int(L), int(shape), C.byref(ure),
                                        C.byref(uim), _p(terms), C.byref(asum))
    if rc != 0:
        raise ValueError(f"oracle_energy failed ({rc})")
    if full:
        return dict(U=ure.value, Uim=uim.value, abs_sum=asum.value,
                    terms=terms.reshape(L + 1, L + 1))
    return ure.value


def coulomb(xyzA, qA, xyzB, qB):
    """eq. (1) over absolute positions."""
    xyzA = _f64(xyzA, (-1, 3)); qA = _f64(qA, (-1,))
    xyzB = _f64(xyzB, (-1, 3)); qB = _f64(qB, (-1,))
    return load().oracle_coulomb(_p(xyzA), _p(qA), len(qA), _p(xyzB), _p(qB), len(qB))


def pose(xyz, c_old, quat, c_new):
    xyz = _f64(xyz, (-1, 3))
    out = np.empty_like(xyz)
    rc = load().oracle_pose(_p(xyz), len(xyz), _p(_f64(c_old, (3,))), _p(_f64(quat, (4,))),
                            _p(_f64(c_new, (3,))), _p(out))
    if rc != 0:
        raise ValueError("oracle_pose: bad arguments")
    return out


def trunc_bound(SA, SB, aA, aB, R, L, shape=SQUARE):
    f = load().oracle_trunc_bound if shape == SQUARE else load().oracle_trunc_bound_tri
    return f(float(SA), float(SB), float(aA), float(aB), float(R), int(L))


def energy_sensitivity(QA, AbarA, QB, AbarB, R, L, shape=SQUARE):
    """sum over the kept terms of |factor| (Abar^A |Q^B| + |Q^A| Abar^B): a moment error of
    at most e * Abar_lm per entry changes eq. (9) by at most e times this, to first order."""
    QA = np.asarray(QA, dtype=np.complex128)
    QB = np.asarray(QB, dtype=np.complex128)
    AbarA = _f64(AbarA)
    AbarB = _f64(AbarB)
    assert len(AbarA) == len(QA) and len(AbarB) == len(QB)
    qa, qb = _interleave(QA), _interleave(QB)
    out = C.c_double()
    rc = load().oracle_energy_sensitivity(_p(qa), _p(AbarA), order_of(QA), _p(qb), _p(AbarB), order_of(QB),
                                          _p(_f64(R, (3,))), int(L), int(shape), C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle_energy_sensitivity failed ({rc})")
    return out.value


def complex_to_packed(Q, L=None):
    """Complex table (index l*l+l+m) -> real-packed m >= 0 table of (L+1)^2 doubles."""
    Q = np.asarray(Q)
    if L is None:
        L = order_of(Q)
    out = np.zeros((L + 1) ** 2)
    for l in range(L + 1):
        out[l * l] = Q[l * l + l].real
        for m in range(1, l + 1):
            out[l * l + 2 * m - 1] = Q[l * l + l + m].real
            out[l * l + 2 * m] = Q[l * l + l + m].imag
    return out


def packed_to_complex(P):
    P = np.asarray(P, dtype=np.float64)
    L = order_of(P)
    Q = np.zeros((L + 1) ** 2, dtype=np.complex128)
    for l in range(L + 1):
        Q[l * l + l] = P[l * l]
        for m in range(1, l + 1):
            v = P[l * l + 2 * m - 1] + 1j * P[l * l + 2 * m]
            Q[l * l + l + m] = v
            Q[l * l + l - m] = (-1) ** m * np.conj(v)
    return Q


def pair_energy_from_atoms(xyzA, qA, cA, xyzB, qB, cB, L, full=False):
    """Oracle TCM energy of two molecules given absolute atom positions and centres."""
    QA = moments(xyzA, qA, cA, L)
    QB = moments(xyzB, qB, cB, L)
    R = _f64(cB, (3,)) - _f64(cA, (3,))
    return energy(QA, QB, R, L, full=full)


def _interleave(Q):
    Q = np.asarray(Q, dtype=np.complex128)
    out = np.empty(2 * len(Q))
    out[0::2] = Q.real
    out[1::2] = Q.imag
    return out


def energy_grad(QA, QB, R, L):
    """grad_R0 of eq. (9) with the moments fixed; the force on B is its negative."""
    qa, qb = _interleave(QA), _interleave(QB)
    g = np.zeros(3)
    rc = load().oracle_energy_grad(_p(qa), order_of(QA), _p(qb), order_of(QB), _p(_f64(R, (3,))), int(L), _p(g))
    if rc != 0:
        raise ValueError(f"oracle_energy_grad failed ({rc})")
    return g


def energy_coeffs(QA, QB, R, L, side):
    """Complex (L+1)^2 table W with U = Re sum W * Q^B (side 1) or Re sum W * Q^A (side 0)."""
    qa, qb = _interleave(QA), _interleave(QB)
    W = np.zeros(2 * (L + 1) ** 2)
    rc = load().oracle_energy_coeffs(_p(qa), order_of(QA), _p(qb), order_of(QB), _p(_f64(R, (3,))), int(L),
                                     int(side), _p(W))
    if rc != 0:
        raise ValueError(f"oracle_energy_coeffs failed ({rc})")
    return W[0::2] + 1j * W[1::2]


def atom_forces(W, xyz, q, c):
    """Per-atom forces F[n][3] = -dU/dR_i at fixed centre c for U = Re sum W * Q(eq. 8)."""
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q, (-1,))
    w = _interleave(W)
    F = np.zeros((len(q), 3))
    rc = load().oracle_atom_forces(_p(w), order_of(W), _p(xyz), _p(q), len(q), _p(_f64(c, (3,))), _p(F))
    if rc != 0:
        raise ValueError(f"oracle_atom_forces failed ({rc})")
    return F


def pair_forces(xyzA, qA, cA, xyzB, qB, cB, R, L, quat=None):
    """Forces and torques of the truncated energy of A (atoms xyzA about centre cA) and B
    (atoms xyzB about cB, posed by quat about cB, then placed at cA + R):
    U, F_B = -grad_R U (F_A = -F_B), the per-atom forces FA[nA][3] and FB[nB][3] at fixed
    centres (FB on the posed atoms), and the torques about each centre,
    tau = sum_i (x_i - c) x F_i."""
    xB = pose(xyzB, cB, quat, cB) if quat is not None else _f64(xyzB, (-1, 3))
    QA = moments(xyzA, qA, cA, L)
    QB = moments(xB, qB, cB, L)
    U = energy(QA, QB, R, L)
    FB_c = -energy_grad(QA, QB, R, L)
    FA = atom_forces(energy_coeffs(QA, QB, R, L, 0), xyzA, qA, cA)
    FB = atom_forces(energy_coeffs(QA, QB, R, L, 1), xB, qB, cB)
    tA = np.sum(np.cross(_f64(xyzA, (-1, 3)) - cA, FA), axis=0)
    tB = np.sum(np.cross(xB - cB, FB), axis=0)
    return dict(U=U, F_B=FB_c, FA=FA, FB=FB, tau_A=tA, tau_B=tB, QA=QA, QB=QB)

