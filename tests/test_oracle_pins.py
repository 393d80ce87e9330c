"""Pins for the FP64 oracle: each test ties the oracle to something other than itself --
a library routine, a closed form, the direct Coulomb sum (eq. 1) with a rigorous bound, or
an exact invariance -- so that a dropped term, wrong sign, wrong index or transposed operand
in eq. (8) or eq. (9) fails at least one of them.  No GPU needed."""
import math

import numpy as np
import pytest

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- library routines (P5)
def test_ylm_matches_scipy(orc):
    from scipy.special import sph_harm_y
    angles = [(0.0, 0.0), (math.pi, 0.3), (math.pi / 2, 1.0), (0.3, -2.0), (2.5, 3.0),
              (1e-9, 0.7), (math.pi - 1e-9, -1.2)]
    for th, ph in angles:
        for l in range(0, 25):
            for m in range(-l, l + 1):
                ref = complex(sph_harm_y(l, m, th, ph))
                got = orc.ylm(l, m, th, ph)
                assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (l, m, th, ph, got, ref)


def test_threej_matches_sympy_general_and_stretched(orc):
    from sympy.physics.wigner import wigner_3j
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(150):       # general (non-stretched) symbols
        j1, j2 = rng.integers(0, 7, 2)
        j3 = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        cases.append((int(j1), int(j2), int(j3), int(m1), int(m2), int(-m1 - m2)))
    for l1 in range(0, 9):     # stretched symbols used by eq. (9)
        for l2 in range(0, 9):
            for m1 in range(-l1, l1 + 1, max(1, l1 // 2)):
                for m2 in range(-l2, l2 + 1, max(1, l2 // 2)):
                    cases.append((l1, l2, l1 + l2, m1, m2, -m1 - m2))
    for c in cases:
        ref = float(wigner_3j(*c))
        assert abs(orc.threej(*c) - ref) <= 1e-13 * max(1.0, abs(ref)), c
    assert orc.threej(1, 1, 1, 1, 0, 0) == 0.0          # m's do not sum to 0
    assert orc.threej(1, 1, 3, 0, 0, 0) == 0.0          # triangle rule


def test_stretched_threej_closed_form(orc):
    # (l1 l2 L; m1 m2 -M), L = l1+l2: (-1)^{l1-l2+M} sqrt[(2l1)!(2l2)!(L+M)!(L-M)! /
    #  ((2L+1)!(l1+m1)!(l1-m1)!(l2+m2)!(l2-m2)!)]   (textbook closed form)
    f = math.factorial
    for l1 in range(0, 16, 3):
        for l2 in range(0, 14, 2):
            L = l1 + l2
            for m1 in range(-l1, l1 + 1):
                for m2 in (-l2, 0, l2):
                    M = m1 + m2
                    v = math.sqrt(f(2 * l1) * f(2 * l2) * f(L + M) * f(L - M) /
                                  (f(2 * L + 1) * f(l1 + m1) * f(l1 - m1) * f(l2 + m2) * f(l2 - m2)))
                    ref = (-1) ** (l1 - l2 + M) * v
                    assert orc.threej(l1, l2, L, m1, m2, -M) == pytest.approx(ref, rel=1e-13, abs=1e-300)


# ---------------------------------------------------------------- moments, eq. (8)
def test_moments_vs_scipy_all_m(orc):
    """eq. (8) evaluated with scipy's Y_lm for every m (negative m included)."""
    from scipy.special import sph_harm_y
    x = RNG.normal(size=(17, 3)) * 2.0
    q = RNG.uniform(-1, 1, 17)
    c = np.array([0.3, -0.2, 0.1])
    L = 9
    Q = orc.moments(x, q, c, L)
    d = x - c
    r = np.linalg.norm(d, axis=1)
    th = np.arccos(d[:, 2] / r)
    ph = np.arctan2(d[:, 1], d[:, 0])
    for l in range(L + 1):
        for m in range(-l, l + 1):
            ref = np.sum(q * r ** l * math.sqrt(4 * math.pi / (2 * l + 1)) * sph_harm_y(l, m, th, ph))
            assert abs(Q[l * l + l + m] - ref) <= 1e-12 * max(1.0, np.sum(np.abs(q) * r ** l))


def test_moments_low_order_cartesian_closed_forms(orc):
    """Racah solid harmonics of order <= 2: C10 = z, C11 = -(x+iy)/sqrt2, C20 = (3z^2-r^2)/2,
    C21 = -sqrt(3/2) z (x+iy), C22 = sqrt(3/8) (x+iy)^2."""
    x = RNG.normal(size=(11, 3))
    q = RNG.uniform(-1, 1, 11)
    Q = orc.moments(x, q, np.zeros(3), 2)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    w = X + 1j * Y
    r2 = X * X + Y * Y + Z * Z
    ref = {(0, 0): q.sum(), (1, 0): np.sum(q * Z), (1, 1): -np.sum(q * w) / math.sqrt(2),
           (2, 0): np.sum(q * (3 * Z * Z - r2) / 2), (2, 1): -math.sqrt(1.5) * np.sum(q * Z * w),
           (2, 2): math.sqrt(3 / 8) * np.sum(q * w * w)}
    for (l, m), v in ref.items():
        assert abs(Q[l * l + l + m] - v) < 1e-13
        assert abs(Q[l * l + l - m] - (-1) ** m * np.conj(v)) < 1e-13


def test_moments_charge_on_axis_and_at_centre(orc):
    L = 12
    Q = orc.moments([[0, 0, 1.7]], [0.6], np.zeros(3), L)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            ref = 0.6 * 1.7 ** l if m == 0 else 0.0
            assert abs(Q[l * l + l + m] - ref) <= 1e-13 * max(1, abs(ref))
    Q = orc.moments([[1.0, 2.0, 3.0]], [0.25], [1.0, 2.0, 3.0], L)   # atom at the centre
    assert Q[0] == 0.25 and np.all(Q[1:] == 0)


def test_moments_superposition_and_translation(orc):
    x = RNG.normal(size=(30, 3))
    q = RNG.uniform(-1, 1, 30)
    c = np.array([0.5, 0.1, -0.4])
    L = 10
    Q = orc.moments(x, q, c, L)
    Q1 = orc.moments(x[:13], q[:13], c, L)
    Q2 = orc.moments(x[13:], q[13:], c, L)
    assert np.max(np.abs(Q - (Q1 + Q2))) < 1e-12 * np.max(np.abs(Q))
    s = np.array([10.0, -3.0, 7.0])
    Qs = orc.moments(x + s, q, c + s, L)
    assert np.max(np.abs(Q - Qs)) < 1e-11 * np.max(np.abs(Q))


def test_pose_z_rotation_phase(orc):
    """Active rotation by gamma about z: phi -> phi + gamma, so Q'_lm = e^{i m gamma} Q_lm.
    Pins the quaternion convention of oracle_pose together with the phase of Y_lm."""
    x = RNG.normal(size=(25, 3))
    q = RNG.uniform(-1, 1, 25)
    L = 8
    g = 0.83
    quat = [math.cos(g / 2), 0, 0, math.sin(g / 2)]
    xr = orc.pose(x, np.zeros(3), quat, np.zeros(3))
    Q = orc.moments(x, q, np.zeros(3), L)
    Qr = orc.moments(xr, q, np.zeros(3), L)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            assert abs(Qr[l * l + l + m] - np.exp(1j * m * g) * Q[l * l + l + m]) < 1e-13 * np.abs(Q).max()


def test_pose_matrix_is_rotation(orc):
    for qv in RNG.normal(size=(5, 4)):
        pts = np.eye(3)
        M = orc.pose(pts, np.zeros(3), qv, np.zeros(3)).T   # columns are images of e_i
        assert np.allclose(M.T @ M, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(M) - 1) < 1e-14
    # quaternion (cos t/2, sin t/2 n): rotation by t about n (right-hand rule)
    t = 0.4
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    qv = np.r_[math.cos(t / 2), math.sin(t / 2) * n]
    v = np.array([0.3, -1.0, 0.5])
    rod = v * math.cos(t) + np.cross(n, v) * math.sin(t) + n * np.dot(n, v) * (1 - math.cos(t))
    assert np.allclose(orc.pose([v], np.zeros(3), qv, np.zeros(3))[0], rod, atol=1e-14)


# ---------------------------------------------------------------- energy, eq. (9)
def _two_clouds(seed, nA=40, nB=30, aA=1.0, aB=1.3, t=0.5, charge=(-1, 1)):
    rng = np.random.default_rng(seed)
    def cloud(n, a):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return v * (a * rng.uniform(0, 1, n) ** (1 / 3))[:, None]
    xA, xB = cloud(nA, aA), cloud(nB, aB)
    qA, qB = rng.uniform(*charge, nA), rng.uniform(*charge, nB)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    R = (aA + aB) / t * u
    cA = rng.normal(size=3)
    return xA + cA, qA, cA, xB + cA + R, qB, cA + R


@pytest.mark.parametrize("t", [0.3, 0.5, 0.7, 0.85])
def test_energy_vs_direct_sum_within_rigorous_bound(orc, t):
    """P1: |U_L - U_coulomb| <= bound(L) for every L (square truncation), and the error
    falls by orders of magnitude from L = 0 to L = 12."""
    for seed in range(3):
        xA, qA, cA, xB, qB, cB = _two_clouds(seed, t=t)
        Uc = orc.coulomb(xA, qA, xB, qB)
        aA, aB = orc.radius(xA, cA), orc.radius(xB, cB)
        R = np.linalg.norm(cB - cA)
        QA = orc.moments(xA, qA, cA, 12)
        QB = orc.moments(xB, qB, cB, 12)
        errs = []
        for L in range(13):
            U = orc.energy(QA, QB, cB - cA, L)
            b = orc.trunc_bound(np.abs(qA).sum(), np.abs(qB).sum(), aA, aB, R, L)
            assert abs(U - Uc) <= b * (1 + 1e-9) + 1e-14, (t, seed, L, U, Uc, b)
            errs.append(abs(U - Uc))
        if t <= 0.5:
            assert errs[12] < 1e-5 * max(errs[0], 1e-300) or errs[12] < 1e-13


def test_energy_tiny_brute_force_two_by_two(orc):
    """2 + 2 charges, far apart: L = 16 reproduces the 4-term direct sum to 1e-14."""
    xA = np.array([[0.1, 0.0, 0.05], [-0.1, 0.02, 0.0]])
    xB = np.array([[5.0, 3.0, 0.1], [5.05, 2.9, -0.1]])
    qA, qB = np.array([1.0, -0.5]), np.array([0.7, 0.2])
    cA, cB = xA.mean(0), xB.mean(0)
    direct = sum(qA[i] * qB[j] / np.linalg.norm(xB[j] - xA[i]) for i in range(2) for j in range(2))
    U = orc.pair_energy_from_atoms(xA, qA, cA, xB, qB, cB, 16)
    assert abs(U - direct) < 1e-14 * abs(direct) + 1e-15


def _cartesian_taylor_terms(xA, qA, cA, xB, qB, cB, lmax):
    """(l1, l2) term of the double Taylor series of sum q_i q_j / |R + b_j - a_i| about
    a_i = b_j = 0:  sum_{|al|=l1,|be|=l2} [sum_i q_i (-a_i)^al/al!][sum_j q_j b_j^be/be!]
    d^{al+be}(1/|R|), derivatives of 1/|R| from sympy."""
    import itertools
    import sympy as sp
    X, Y, Z = sp.symbols("X Y Z", real=True)
    f = 1 / sp.sqrt(X * X + Y * Y + Z * Z)
    R = np.asarray(cB, float) - np.asarray(cA, float)
    a = np.asarray(xA) - cA
    b = np.asarray(xB) - cB

    def multi(k):
        return [al for al in itertools.product(range(k + 1), repeat=3) if sum(al) == k]

    deriv = {}
    for k in range(2 * lmax + 1):
        for al in multi(k):
            e = f
            for v, p in zip((X, Y, Z), al):
                if p:
                    e = sp.diff(e, v, p)
            deriv[al] = float(e.subs({X: R[0], Y: R[1], Z: R[2]}))
    out = {}
    fac = math.factorial
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1 - l1):
            s = 0.0
            for al in multi(l1):
                ca = np.sum(qA * np.prod((-a) ** np.array(al), axis=1)) / (fac(al[0]) * fac(al[1]) * fac(al[2]))
                for be in multi(l2):
                    cb = np.sum(qB * np.prod(b ** np.array(be), axis=1)) / (fac(be[0]) * fac(be[1]) * fac(be[2]))
                    s += ca * cb * deriv[tuple(np.add(al, be))]
            out[(l1, l2)] = s
    return out


def test_energy_terms_match_cartesian_taylor(orc):
    """P2: every (l1, l2) block with l1 + l2 <= 4 of eq. (9) equals the Cartesian Taylor term
    (charge-charge, charge-dipole, dipole-dipole, quadrupole terms, ...)."""
    xA, qA, cA, xB, qB, cB = _two_clouds(3, nA=5, nB=4, t=0.4)
    L = 4
    d = orc.pair_energy_from_atoms(xA, qA, cA, xB, qB, cB, L, full=True)
    ref = _cartesian_taylor_terms(xA, qA, cA, xB, qB, cB, 4)
    scale = max(abs(v) for v in ref.values())
    for (l1, l2), v in ref.items():
        assert abs(d["terms"][l1, l2] - v) < 1e-12 * scale, (l1, l2, d["terms"][l1, l2], v)


def test_energy_low_order_physics_closed_forms(orc):
    """Explicit textbook forms: qq/R, q_B p_A.R/R^3, -q_A p_B.R/R^3, dipole-dipole."""
    xA, qA, cA, xB, qB, cB = _two_clouds(4, nA=6, nB=5, t=0.3)
    d = orc.pair_energy_from_atoms(xA, qA, cA, xB, qB, cB, 1, full=True)
    Rv = cB - cA
    R = np.linalg.norm(Rv)
    n = Rv / R
    pA = (qA[:, None] * (xA - cA)).sum(0)
    pB = (qB[:, None] * (xB - cB)).sum(0)
    T = d["terms"]
    assert T[0, 0] == pytest.approx(qA.sum() * qB.sum() / R, rel=1e-13)
    assert T[1, 0] == pytest.approx(qB.sum() * pA.dot(Rv) / R ** 3, rel=1e-12)
    assert T[0, 1] == pytest.approx(-qA.sum() * pB.dot(Rv) / R ** 3, rel=1e-12)
    assert T[1, 1] == pytest.approx((pA.dot(pB) - 3 * pA.dot(n) * pB.dot(n)) / R ** 3, rel=1e-12)


def test_energy_collinear_closed_form(orc):
    """P3: charges on the line of centres -> 1/(R + z_B - z_A) = sum C(l1+l2,l1) z_A^l1
    (-z_B)^l2 / R^{l1+l2+1}; every (l1, l2) block up to L = 10 must match."""
    rng = np.random.default_rng(9)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    zA = rng.uniform(-1, 1, 7)
    zB = rng.uniform(-1.2, 1.2, 6)
    qA, qB = rng.uniform(-1, 1, 7), rng.uniform(-1, 1, 6)
    R = 6.0
    cA = np.array([1.0, 2.0, 3.0])
    cB = cA + R * u
    L = 10
    d = orc.pair_energy_from_atoms(cA + zA[:, None] * u, qA, cA, cB + zB[:, None] * u, qB, cB, L, full=True)
    for l1 in range(L + 1):
        for l2 in range(L + 1):
            ref = (-1) ** l2 * math.comb(l1 + l2, l1) * np.sum(qA * zA ** l1) * np.sum(qB * zB ** l2) / R ** (l1 + l2 + 1)
            assert abs(d["terms"][l1, l2] - ref) < 1e-13 * (abs(ref) + 1e-3 * math.comb(l1 + l2, l1) / R ** (l1 + l2 + 1))


def test_energy_invariants(orc):
    """P4: rotation of the whole system, swap of A and B, length scaling, bilinearity,
    reality of eq. (9)."""
    xA, qA, cA, xB, qB, cB = _two_clouds(5, t=0.45)
    L = 8
    U = orc.pair_energy_from_atoms(xA, qA, cA, xB, qB, cB, L, full=True)
    assert abs(U["Uim"]) < 1e-14 * U["abs_sum"]
    quat = np.array([0.3, -0.5, 0.7, 0.2])
    o = np.zeros(3)
    rot = lambda v: orc.pose(np.atleast_2d(v), o, quat, o)
    Ur = orc.pair_energy_from_atoms(rot(xA), qA, rot(cA)[0], rot(xB), qB, rot(cB)[0], L)
    assert Ur == pytest.approx(U["U"], rel=1e-12)
    Us = orc.pair_energy_from_atoms(xB, qB, cB, xA, qA, cA, L)
    assert Us == pytest.approx(U["U"], rel=1e-13)
    s = 3.7
    Uk = orc.pair_energy_from_atoms(s * xA, qA, s * cA, s * xB, qB, s * cB, L)
    assert Uk == pytest.approx(U["U"] / s, rel=1e-12)
    U2 = orc.pair_energy_from_atoms(xA, 2 * qA, cA, xB, -0.5 * qB, cB, L)
    assert U2 == pytest.approx(-U["U"], rel=1e-13)


def test_energy_direction_along_z_axis(orc):
    """R0 parallel to +z or -z (Phi = atan2(0, 0)) gives the same U as the whole system
    rotated off the axis."""
    xA, qA, cA, xB, qB, cB = _two_clouds(6, t=0.4)
    R = np.linalg.norm(cB - cA)
    for sgn in (1.0, -1.0):
        cB2 = cA + sgn * np.array([0.0, 0.0, R])
        xB2 = xB - cB + cB2
        U = orc.pair_energy_from_atoms(xA, qA, cA, xB2, qB, cB2, 8)
        quat = [0.9, 0.3, -0.2, 0.1]
        rot = lambda v: orc.pose(np.atleast_2d(v), cA, quat, cA)
        Ur = orc.pair_energy_from_atoms(rot(xA), qA, cA, rot(xB2), qB, rot(cB2)[0], 8)
        assert U == pytest.approx(Ur, rel=1e-12)


def test_energy_uses_prefix_of_higher_order_tables(orc):
    xA, qA, cA, xB, qB, cB = _two_clouds(7)
    QA8, QB8 = orc.moments(xA, qA, cA, 8), orc.moments(xB, qB, cB, 8)
    QA4, QB4 = orc.moments(xA, qA, cA, 4), orc.moments(xB, qB, cB, 4)
    assert orc.energy(QA8, QB8, cB - cA, 4) == orc.energy(QA4, QB4, cB - cA, 4)


def test_energy_convergence_in_distance(orc):
    """At fixed L the error of the truncated series falls at least like (1/R)^{L+2}."""
    xA, qA, cA, xB, qB, _ = _two_clouds(8, t=0.5)
    xb = xB - xB.mean(0)
    u = np.array([0.0, 0.6, 0.8])
    L = 4
    errs = []
    for R in (8.0, 16.0, 32.0):
        cB = cA + R * u
        U = orc.pair_energy_from_atoms(xA, qA, cA, xb + cB, qB, cB, L)
        errs.append(abs(U - orc.coulomb(xA, qA, xb + cB, qB)))
    assert errs[1] < errs[0] * 2.0 ** -(L + 1) and errs[2] < errs[1] * 2.0 ** -(L + 1)


def test_radius_and_centroid(orc):
    x = RNG.normal(size=(50, 3)) + 4
    c = orc.centroid(x)
    assert np.allclose(c, x.mean(0), atol=1e-14)
    assert orc.radius(x, c) == pytest.approx(np.max(np.linalg.norm(x - c, axis=1)), rel=1e-15)


def test_trunc_bound_outside_domain_is_infinite(orc):
    assert math.isinf(orc.trunc_bound(1, 1, 1.0, 1.0, 2.0, 4))


def test_packed_roundtrip(orc):
    x = RNG.normal(size=(9, 3))
    q = RNG.uniform(-1, 1, 9)
    Q = orc.moments(x, q, np.zeros(3), 6)
    P = orc.complex_to_packed(Q)
    assert len(P) == 49
    assert np.max(np.abs(orc.packed_to_complex(P) - Q)) < 1e-15


# ---------------------------------------------------------------- truncation bounds, by value
def _taylor_tail_sums(al, be, L, nmax=None):
    """Brute-force sums of the per-term bounds C(l1+l2, l1) al^l1 be^l2 of the double Taylor
    series of 1/|R + r_B - r_A| (R = 1): over the blocks outside the square l1, l2 <= L
    (union), over those with both orders above L (intersection, which the closed form of the
    square bound counts twice), and over those outside the triangle l1 + l2 <= L.  Summed by
    total order n = l1 + l2 until the terms are below 1e-300 of the sum."""
    from scipy.special import gammaln
    t = al + be
    if nmax is None:
        nmax = int(np.ceil(np.log(1e-19) / np.log(t))) + L + 60
    union, inter, tri = [], [], []
    for n in range(nmax + 1):
        l1 = np.arange(n + 1)
        l2 = n - l1
        lt = gammaln(n + 1) - gammaln(l1 + 1) - gammaln(l2 + 1)
        with np.errstate(divide="ignore"):
            lt = lt + l1 * np.log(al) + l2 * np.log(be)
        v = np.exp(lt)
        union.extend(v[(l1 > L) | (l2 > L)])
        inter.extend(v[(l1 > L) & (l2 > L)])
        if n > L:
            tri.extend(v)
    return math.fsum(union), math.fsum(inter), math.fsum(tri)


@pytest.mark.parametrize("al,be", [(0.1, 0.2), (0.3, 0.3), (0.45, 0.15), (0.05, 0.6), (0.4, 0.45)])
def test_trunc_bound_value_equals_tail_sum(orc, al, be):
    """The closed forms of both bounds equal the brute-force sums of the term bounds they
    claim to add up (square: the two one-sided tails, i.e. the union of the dropped blocks plus
    their intersection once more; triangle: every block of total order > L), so a wrong
    exponent, a dropped (1 - alpha - beta) or a swapped ratio fails.  SA, SB and R scale it."""
    SA, SB, R = 2.5, 0.7, 3.0
    for L in (0, 1, 2, 4, 7, 10, 16):
        union, inter, tri = _taylor_tail_sums(al, be, L)
        b = orc.trunc_bound(SA, SB, al * R, be * R, R, L)
        assert b == pytest.approx(SA * SB / R * (union + inter), rel=1e-12), (al, be, L)
        assert b >= SA * SB / R * union
        bt = orc.trunc_bound(SA, SB, al * R, be * R, R, L, shape=orc.TRIANGULAR)
        assert bt == pytest.approx(SA * SB / R * tri, rel=1e-12), (al, be, L)


def _tight_collinear(al, be, R=5.0):
    """One unit charge in each molecule on the line of centres, each at its molecule's radius
    and facing the other: every term of the double Taylor series is positive, so the error of
    a truncation equals the sum of the bounds of the terms it drops."""
    u = np.array([0.36, -0.48, 0.8])
    cA = np.array([0.5, 1.0, -2.0])
    cB = cA + R * u
    xA = (cA + al * R * u)[None, :]
    xB = (cB - be * R * u)[None, :]
    return xA, np.ones(1), cA, xB, np.ones(1), cB, R


@pytest.mark.parametrize("al,be", [(0.3, 0.3), (0.2, 0.45), (0.5, 0.1)])
def test_trunc_bound_tight_collinear(orc, al, be):
    xA, qA, cA, xB, qB, cB, R = _tight_collinear(al, be)
    Uc = orc.coulomb(xA, qA, xB, qB)
    assert Uc == pytest.approx(1.0 / (R * (1.0 - al - be)), rel=1e-14)
    QA, QB = orc.moments(xA, qA, cA, 12), orc.moments(xB, qB, cB, 12)
    for L in range(1, 11):
        union, inter, tri = _taylor_tail_sums(al, be, L)
        err_sq = Uc - orc.energy(QA, QB, cB - cA, L)
        err_tri = Uc - orc.energy(QA, QB, cB - cA, L, shape=orc.TRIANGULAR)
        # the square truncation misses exactly the union of the dropped blocks
        assert err_sq == pytest.approx(union / R, rel=1e-9, abs=1e-15 / R), (L, err_sq, union / R)
        b = orc.trunc_bound(1.0, 1.0, al * R, be * R, R, L)
        assert err_sq <= b and b == pytest.approx((union + inter) / R, rel=1e-12)
        # the triangular truncation misses exactly its bound: the bound is attained
        bt = orc.trunc_bound(1.0, 1.0, al * R, be * R, R, L, shape=orc.TRIANGULAR)
        assert err_tri == pytest.approx(bt, rel=1e-9), (L, err_tri, bt)


# ---------------------------------------------------------------- triangular truncation
def test_triangular_collinear_closed_form(orc):
    """Charges on the line of centres: the triangular sum keeps exactly the blocks
    l1 + l2 <= L of the 1-D Taylor double series, and drops the others."""
    rng = np.random.default_rng(19)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    zA, zB = rng.uniform(-1, 1, 6), rng.uniform(-1.1, 1.1, 5)
    qA, qB = rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 5)
    R = 5.5
    cA = np.array([-1.0, 0.5, 2.0])
    cB = cA + R * u
    xA, xB = cA + zA[:, None] * u, cB + zB[:, None] * u
    QA, QB = orc.moments(xA, qA, cA, 9), orc.moments(xB, qB, cB, 9)
    for L in (0, 1, 3, 6, 9):
        d = orc.energy(QA, QB, cB - cA, L, full=True, shape=orc.TRIANGULAR)
        tot = 0.0
        for l1 in range(L + 1):
            for l2 in range(L + 1):
                ref = 0.0
                if l1 + l2 <= L:
                    ref = (-1) ** l2 * math.comb(l1 + l2, l1) * np.sum(qA * zA ** l1) * np.sum(qB * zB ** l2) \
                        / R ** (l1 + l2 + 1)
                tot += ref
                scale = abs(ref) + 1e-3 * math.comb(l1 + l2, l1) / R ** (l1 + l2 + 1)
                assert abs(d["terms"][l1, l2] - ref) < 1e-13 * scale, (L, l1, l2)
        assert d["U"] == pytest.approx(tot, rel=1e-12, abs=1e-15)


def test_triangular_equals_taylor_orders(orc):
    """The triangular sum at L is the Taylor series of eq. (1) through total order L:
    the sum of the Cartesian Taylor blocks with l1 + l2 <= L (sympy derivatives of 1/R)."""
    xA, qA, cA, xB, qB, cB = _two_clouds(13, nA=5, nB=4, t=0.45)
    ref = _cartesian_taylor_terms(xA, qA, cA, xB, qB, cB, 4)
    QA, QB = orc.moments(xA, qA, cA, 4), orc.moments(xB, qB, cB, 4)
    scale = max(abs(v) for v in ref.values())
    for L in range(5):
        U = orc.energy(QA, QB, cB - cA, L, shape=orc.TRIANGULAR)
        want = sum(v for (l1, l2), v in ref.items() if l1 + l2 <= L)
        assert abs(U - want) < 1e-12 * scale, (L, U, want)


@pytest.mark.parametrize("t", [0.3, 0.6, 0.85])
def test_triangular_vs_direct_sum_within_bound(orc, t):
    """P1 for the triangular truncation: |U_tri(L) - eq. (1)| <= S_A S_B t^{L+1}/(R(1-t)),
    and at equal L the square truncation (which keeps more blocks) is at least as close on
    average over the seeds."""
    e_sq, e_tri = 0.0, 0.0
    for seed in range(3):
        xA, qA, cA, xB, qB, cB = _two_clouds(40 + seed, t=t)
        Uc = orc.coulomb(xA, qA, xB, qB)
        aA, aB = orc.radius(xA, cA), orc.radius(xB, cB)
        R = np.linalg.norm(cB - cA)
        QA, QB = orc.moments(xA, qA, cA, 12), orc.moments(xB, qB, cB, 12)
        for L in range(13):
            U = orc.energy(QA, QB, cB - cA, L, shape=orc.TRIANGULAR)
            b = orc.trunc_bound(np.abs(qA).sum(), np.abs(qB).sum(), aA, aB, R, L, shape=orc.TRIANGULAR)
            assert abs(U - Uc) <= b * (1 + 1e-9) + 1e-14, (t, seed, L, U, Uc, b)
        e_tri += abs(orc.energy(QA, QB, cB - cA, 8, shape=orc.TRIANGULAR) - Uc)
        e_sq += abs(orc.energy(QA, QB, cB - cA, 8) - Uc)
    assert e_sq <= e_tri


def test_square_minus_triangular_is_the_high_blocks(orc):
    xA, qA, cA, xB, qB, cB = _two_clouds(14, t=0.5)
    L = 7
    QA, QB = orc.moments(xA, qA, cA, L), orc.moments(xB, qB, cB, L)
    sq = orc.energy(QA, QB, cB - cA, L, full=True)
    tri = orc.energy(QA, QB, cB - cA, L, full=True, shape=orc.TRIANGULAR)
    hi = sum(sq["terms"][l1, l2] for l1 in range(L + 1) for l2 in range(L + 1) if l1 + l2 > L)
    assert sq["U"] - tri["U"] == pytest.approx(hi, rel=1e-10, abs=1e-14 * sq["abs_sum"])
    for l1 in range(L + 1):
        for l2 in range(L + 1 - l1):
            assert tri["terms"][l1, l2] == sq["terms"][l1, l2]


# ---------------------------------------------------------------- sensitivity of eq. (9)
def test_sensitivity_single_charges_is_twice_abs_sum(orc):
    """With one charge per molecule the absolute sums equal the moduli of the moments
    (Abar_lm = |Q_lm|), so the sensitivity is 2 sum_t |f_t Q^A Q^B| = 2 abs_sum."""
    xA, qA, cA, xB, qB, cB = _two_clouds(15, nA=1, nB=1, t=0.5)
    for shape in (orc.SQUARE, orc.TRIANGULAR):
        for L in (0, 3, 8):
            QA, AA = orc.moments(xA, qA, cA, L, with_abs=True)
            QB, AB = orc.moments(xB, qB, cB, L, with_abs=True)
            assert np.allclose(AA, np.abs(QA), rtol=1e-13) and np.allclose(AB, np.abs(QB), rtol=1e-13)
            d = orc.energy(QA, QB, cB - cA, L, full=True, shape=shape)
            s = orc.energy_sensitivity(QA, AA, QB, AB, cB - cA, L, shape=shape)
            assert s == pytest.approx(2.0 * d["abs_sum"], rel=1e-12), (shape, L)


def test_sensitivity_brute_force_small_order(orc):
    """Independent evaluation for L <= 2: each term's factor from sympy's 3j symbol and scipy's
    Y_lm, summed in Python."""
    from scipy.special import sph_harm_y
    from sympy.physics.wigner import wigner_3j
    xA, qA, cA, xB, qB, cB = _two_clouds(16, nA=4, nB=3, t=0.5)
    Rv = cB - cA
    R = np.linalg.norm(Rv)
    th, ph = math.acos(Rv[2] / R), math.atan2(Rv[1], Rv[0])
    for shape in (orc.SQUARE, orc.TRIANGULAR):
        L = 2
        QA, AA = orc.moments(xA, qA, cA, L, with_abs=True)
        QB, AB = orc.moments(xB, qB, cB, L, with_abs=True)
        ref = 0.0
        for l1 in range(L + 1):
            for l2 in range(L + 1):
                if shape == orc.TRIANGULAR and l1 + l2 > L:
                    continue
                Lp = l1 + l2
                coef = math.sqrt(4 * math.pi * math.factorial(2 * Lp) / (math.factorial(2 * l1) * math.factorial(2 * l2)))
                for m1 in range(-l1, l1 + 1):
                    for m2 in range(-l2, l2 + 1):
                        M = m1 + m2
                        f = abs(R ** -(Lp + 1) * coef * float(wigner_3j(l1, l2, Lp, m1, m2, -M))
                                * complex(sph_harm_y(Lp, M, th, ph)))
                        ka, kb = l1 * l1 + l1 + m1, l2 * l2 + l2 + m2
                        ref += f * (AA[ka] * abs(QB[kb]) + abs(QA[ka]) * AB[kb])
        s = orc.energy_sensitivity(QA, AA, QB, AB, Rv, L, shape=shape)
        assert s == pytest.approx(ref, rel=1e-12), shape


def test_sensitivity_bounds_moment_perturbations(orc):
    """Moments perturbed by e * Abar with random phases change eq. (9) by at most
    e * sensitivity + e^2 * (the bilinear remainder)."""
    xA, qA, cA, xB, qB, cB = _two_clouds(17, t=0.6)
    L = 8
    QA, AA = orc.moments(xA, qA, cA, L, with_abs=True)
    QB, AB = orc.moments(xB, qB, cB, L, with_abs=True)
    U0 = orc.energy(QA, QB, cB - cA, L)
    s = orc.energy_sensitivity(QA, AA, QB, AB, cB - cA, L)
    rng = np.random.default_rng(3)
    e = 1e-7
    for _ in range(5):
        dA = e * AA * np.exp(2j * np.pi * rng.uniform(size=len(AA)))
        dB = e * AB * np.exp(2j * np.pi * rng.uniform(size=len(AB)))
        dU = orc.energy(QA + dA, QB + dB, cB - cA, L) - U0
        assert abs(dU) <= e * s * (1 + 1e-6)
