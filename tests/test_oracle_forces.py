"""Pins of the oracle's forces and torques (CPU only).

The oracle differentiates eq. (9) term by term in spherical coordinates (textbook derivative
of the normalised Legendre functions).  These tests pin it to things other than itself:
finite differences of the oracle's energy (in R0, in one atom's position with the moments
recomputed from eq. (8), in a small rotation of B), closed forms (charge-charge,
charge-dipole), the exact identity tau_A + tau_B + R0 x F_B = 0 that rotational invariance of
the truncated energy implies, and convergence to the direct Coulomb forces of eq. (1).
"""
import numpy as np
import pytest

import oracle as orc


def ball(rng, n, radius, centre):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return centre + d * radius * rng.uniform(0, 1, n)[:, None] ** (1 / 3), rng.uniform(-1, 1, n)


def fd5(f, x0, h):
    return (-f(x0 + 2 * h) + 8 * f(x0 + h) - 8 * f(x0 - h) + f(x0 - 2 * h)) / (12 * h)


def small_pair(seed, nA=30, nB=25, dist=9.0, direction=None):
    rng = np.random.default_rng(seed)
    xA, qA = ball(rng, nA, 2.0, np.zeros(3))
    u = rng.normal(size=3) if direction is None else np.asarray(direction, float)
    u /= np.linalg.norm(u)
    xB, qB = ball(rng, nB, 1.5, dist * u)
    cA, cB = orc.centroid(xA), orc.centroid(xB)
    return xA, qA, cA, xB, qB, cB


@pytest.mark.parametrize("L", [0, 1, 3, 6])
@pytest.mark.parametrize("axial", [False, True])
def test_energy_grad_matches_finite_differences(L, axial):
    xA, qA, cA, xB, qB, cB = small_pair(1 + L, direction=[0, 0, -1] if axial else None)
    QA, QB = orc.moments(xA, qA, cA, L), orc.moments(xB, qB, cB, L)
    R = cB - cA
    if axial:
        R = np.array([0.0, 0.0, -np.linalg.norm(R)])
    g = orc.energy_grad(QA, QB, R, L)
    h = 1e-3 * np.linalg.norm(R)
    scale = orc.energy(QA, QB, R, L, full=True)["abs_sum"] / np.linalg.norm(R)
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        fd = fd5(lambda t: orc.energy(QA, QB, R + t * e, L), 0.0, h)
        assert abs(g[d] - fd) <= 1e-9 * scale, (d, g[d], fd)


def test_energy_grad_closed_forms():
    rng = np.random.default_rng(3)
    R = rng.normal(size=3) * 5
    Rn = np.linalg.norm(R)
    # L = 0: U = qA qB / R, grad U = -qA qB R / R^3
    QA = orc.moments([[0.2, -0.1, 0.3]], [1.5], [0, 0, 0], 0)
    QB = orc.moments([[0.1, 0.1, -0.2]], [-0.7], [0, 0, 0], 0)
    assert np.allclose(orc.energy_grad(QA, QB, R, 0), -1.5 * -0.7 * R / Rn ** 3, rtol=1e-14, atol=0)
    # a point charge at A's centre and a neutral dipole at B's: U_1 = -qA pB.R / R^3
    q = 0.8
    d = np.array([0.05, -0.02, 0.04])
    QA = orc.moments([[0, 0, 0]], [q], [0, 0, 0], 1)
    QB = orc.moments([d, -d], [1.0, -1.0], [0, 0, 0], 1)
    p = 2 * d
    want = -q * (p / Rn ** 3 - 3 * np.dot(p, R) * R / Rn ** 5)
    assert np.allclose(orc.energy_grad(QA, QB, R, 1), want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("side", [0, 1])
def test_energy_coeffs_reproduce_energy(side):
    xA, qA, cA, xB, qB, cB = small_pair(4)
    L = 5
    QA, QB = orc.moments(xA, qA, cA, L), orc.moments(xB, qB, cB, L)
    R = cB - cA
    W = orc.energy_coeffs(QA, QB, R, L, side)
    U = np.sum(W * (QB if side else QA)).real
    assert abs(U - orc.energy(QA, QB, R, L)) <= 1e-13 * orc.energy(QA, QB, R, L, full=True)["abs_sum"]


@pytest.mark.parametrize("L", [1, 4, 7])
def test_atom_forces_match_finite_differences(L):
    xA, qA, cA, xB, qB, cB = small_pair(10 + L)
    # two special atoms: one at A's centre, one on B's z-axis through its centre
    xA = np.vstack([xA, cA])
    qA = np.append(qA, 0.6)
    xB = np.vstack([xB, cB + [0, 0, 0.7]])
    qB = np.append(qB, -0.4)
    R = cB - cA
    f = orc.pair_forces(xA, qA, cA, xB, qB, cB, R, L)
    QA, QB = f["QA"], f["QB"]
    scale = orc.energy(QA, QB, R, L, full=True)["abs_sum"]
    h = 1e-4
    for side, xs, qs, c, F in ((0, xA, qA, cA, f["FA"]), (1, xB, qB, cB, f["FB"])):
        for i in (0, 7, len(qs) - 1):
            for d in range(3):
                def U(t):
                    x = xs.copy()
                    x[i, d] += t
                    Q = orc.moments(x, qs, c, L)
                    return orc.energy(Q, QB, R, L) if side == 0 else orc.energy(QA, Q, R, L)
                fd = -fd5(U, 0.0, h)
                assert abs(F[i, d] - fd) <= 1e-9 * scale, (side, i, d, F[i, d], fd)


@pytest.mark.parametrize("L", [2, 6])
def test_torques_identity_and_rotation(L):
    xA, qA, cA, xB, qB, cB = small_pair(20 + L)
    quat = np.array([0.9, 0.2, -0.3, 0.25])
    quat /= np.linalg.norm(quat)
    R = cB - cA
    f = orc.pair_forces(xA, qA, cA, xB, qB, cB, R, L, quat=quat)
    scale = np.sum(np.abs(np.cross(xA - cA, f["FA"]))) + np.sum(np.abs(np.cross(xB - cB, f["FB"])))
    # rotational invariance of the truncated energy: tau_A + tau_B + R x F_B = 0
    assert np.all(np.abs(f["tau_A"] + f["tau_B"] + np.cross(R, f["F_B"])) <= 1e-12 * scale)
    # tau_B = -dU/dtheta for a rotation of B about its centre (moments recomputed)
    xBp = orc.pose(xB, cB, quat, cB)
    QA = orc.moments(xA, qA, cA, L)
    for k in range(3):
        def U(t):
            ax = np.zeros(3)
            ax[k] = 1.0
            qk = np.concatenate([[np.cos(t / 2)], np.sin(t / 2) * ax])
            return orc.energy(QA, orc.moments(orc.pose(xBp, cB, qk, cB), qB, cB, L), R, L)
        fd = -fd5(U, 0.0, 1e-3)
        assert abs(f["tau_B"][k] - fd) <= 1e-9 * scale, (k, f["tau_B"][k], fd)


def test_forces_converge_to_coulomb():
    xA, qA, cA, xB, qB, cB = small_pair(40, nA=40, nB=40, dist=12.0)
    R = cB - cA
    # direct eq. (1) forces on B's atoms
    d = xB[:, None, :] - xA[None, :, :]
    Fc = qB[:, None] * np.sum(qA[None, :, None] * d / np.linalg.norm(d, axis=2)[:, :, None] ** 3, axis=1)
    errs = []
    for L in (2, 6, 12):
        f = orc.pair_forces(xA, qA, cA, xB, qB, cB, R, L)
        errs.append(np.max(np.abs(f["FB"] - Fc)) / np.max(np.abs(Fc)))
        # the sum of B's atom forces approaches the force on its centre, F_A = -F_B
        assert np.linalg.norm(np.sum(f["FB"], axis=0) - f["F_B"]) <= 10 * errs[-1] * np.max(np.abs(Fc)) * len(qB)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-7, errs
