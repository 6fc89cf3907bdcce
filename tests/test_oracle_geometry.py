"""Pins for the oracle's kinematics and angular factors (paper Sec. 2.1-2.2).

P8: the reduced Jacobi sets built from explicit particle positions satisfy
eq. (JacobiTrans) with the paper's c, s; the scalar formulas for x_b, y_b, z_b
agree with the vectors; rotations compose.
P11: Wigner d from the explicit sum agrees with the Jacobi-polynomial form
(with the corrected prefactor), is orthogonal, and d^1_00 = cos.
P12: the frame angle w_ba agrees with the body-fixed frames built from the
vectors (eq. (euler-ba)), and the F functions obey eq. (F-ba).
"""
import math

import numpy as np
import pytest
from scipy.special import eval_jacobi

from oracle import physics as ph
from oracle.wigner import F_rot, w_angle, wigner_d

CYCLIC = [(0, 1, 2), (1, 2, 0), (2, 0, 1)]


def jacobi_vectors(r, m):
    """Reduced Jacobi vectors per set: x_a = r_c - r_b for (a, b, c) cyclic,
    y_a = r_a - centre of mass of (b, c); scaled by sqrt(2 mu)."""
    mu, mu_abc = ph.reduced_masses(m)
    X, Y = {}, {}
    for a, b, c in CYCLIC:
        x = r[c] - r[b]
        y = r[a] - (m[b] * r[b] + m[c] * r[c]) / (m[b] + m[c])
        X[a] = math.sqrt(2 * mu[a]) * x
        Y[a] = math.sqrt(2 * mu_abc[a]) * y
    return X, Y


MASSES = [(1.0, 1.0, 1.0), (1.0, 1.0, 1836.0), (1e15, 1.0, 1.0), (3.0, 7.0, 2.0)]


@pytest.mark.parametrize("m", MASSES)
def test_jacobi_rotation_from_positions(m):
    rng = np.random.default_rng(5)
    for _ in range(20):
        r = rng.standard_normal((3, 3))
        X, Y = jacobi_vectors(r, m)
        for a in range(3):
            xa, ya = X[a], Y[a]
            x, y = np.linalg.norm(xa), np.linalg.norm(ya)
            z = xa @ ya / (x * y)
            for b in range(3):
                if b == a:
                    continue
                c, s = ph.rotation_cs(m, b, a)
                np.testing.assert_allclose(X[b], c * xa + s * ya, atol=1e-10 * (x + y))
                np.testing.assert_allclose(Y[b], -s * xa + c * ya, atol=1e-10 * (x + y))
                xb, yb, zb = ph.rotated_coords(np.array([x]), np.array([y]), np.array([z]), c, s)
                assert abs(xb[0] - np.linalg.norm(X[b])) < 1e-10 * (x + y)
                assert abs(yb[0] - np.linalg.norm(Y[b])) < 1e-10 * (x + y)
                assert abs(zb[0] - X[b] @ Y[b] / (np.linalg.norm(X[b]) * np.linalg.norm(Y[b]))) < 1e-9
                assert abs(xb[0] ** 2 + yb[0] ** 2 - x * x - y * y) < 1e-10 * (x * x + y * y)


@pytest.mark.parametrize("m", MASSES)
def test_rotations_compose(m):
    for a in range(3):
        for b in range(3):
            for g in range(3):
                c1, s1 = ph.rotation_cs(m, b, a)
                c2, s2 = ph.rotation_cs(m, g, b)
                c3, s3 = ph.rotation_cs(m, g, a)
                R1 = np.array([[c1, s1], [-s1, c1]])
                R2 = np.array([[c2, s2], [-s2, c2]])
                np.testing.assert_allclose(R2 @ R1, [[c3, s3], [-s3, c3]], atol=1e-12)


def body_frame(xv, yv):
    """Body-fixed axes: z''' along y, x in the x'''z''' plane with a positive
    x''' component (Sec. 2.2)."""
    ez = yv / np.linalg.norm(yv)
    xp = xv - (xv @ ez) * ez
    ex = xp / np.linalg.norm(xp)
    ey = np.cross(ez, ex)
    return np.column_stack([ex, ey, ez])


@pytest.mark.parametrize("m", MASSES[:2] + MASSES[3:])
def test_frame_angle_w(m):
    rng = np.random.default_rng(9)
    for _ in range(20):
        r = rng.standard_normal((3, 3))
        X, Y = jacobi_vectors(r, m)
        for a in range(3):
            x, y = np.linalg.norm(X[a]), np.linalg.norm(Y[a])
            z = X[a] @ Y[a] / (x * y)
            Ra = body_frame(X[a], Y[a])
            for b in range(3):
                if b == a:
                    continue
                Rb = body_frame(X[b], Y[b])
                Rw = Ra.T @ Rb                        # must be R(0, w, 0)
                yb = np.linalg.norm(Y[b])
                w = w_angle(m, b, a, np.array([x]), np.array([y]), np.array([z]), np.array([yb]))[0]
                want = np.array([[math.cos(w), 0, math.sin(w)], [0, 1, 0], [-math.sin(w), 0, math.cos(w)]])
                np.testing.assert_allclose(Rw, want, atol=1e-9)


def test_wigner_d_forms():
    th = np.linspace(0.05, 3.1, 17)
    np.testing.assert_allclose(wigner_d(1, 0, 0, th), np.cos(th), atol=1e-14)
    for J in range(0, 5):
        for M in range(-J, J + 1):
            for Mp in range(abs(M), J + 1):     # the Jacobi form holds for M' >= |M|
                pref = math.sqrt(math.factorial(J + Mp) * math.factorial(J - Mp)
                                 / (math.factorial(J + M) * math.factorial(J - M)))
                jac = (pref * np.sin(th / 2) ** (Mp - M) * np.cos(th / 2) ** (Mp + M)
                       * eval_jacobi(J - Mp, Mp - M, Mp + M, np.cos(th)))
                np.testing.assert_allclose(wigner_d(J, M, Mp, th), jac, atol=1e-12)
        # orthogonal matrix in (M, M')
        for t in (0.3, 1.7, 2.9):
            d = np.array([[wigner_d(J, M, Mp, t) for Mp in range(-J, J + 1)] for M in range(-J, J + 1)])
            np.testing.assert_allclose(d @ d.T, np.eye(2 * J + 1), atol=1e-12)


def euler_zyz(R):
    th = math.acos(max(-1.0, min(1.0, R[2, 2])))
    phi = math.atan2(R[1, 2], R[0, 2])
    psi = math.atan2(R[2, 1], -R[2, 0])
    return phi, th, psi


def D(J, M, Mp, ang):
    phi, th, psi = ang
    return np.exp(-1j * M * phi) * wigner_d(J, M, Mp, th) * np.exp(-1j * Mp * psi)


def F(J, tau, M, Mp, ang):
    return (D(J, M, Mp, ang) + tau * (-1) ** Mp * D(J, M, -Mp, ang)) / math.sqrt(2 + 2 * (Mp == 0))


@pytest.mark.parametrize("J,tau", [(1, 1), (2, 1), (2, -1), (3, 1), (10, 1)])
def test_F_addition_theorem(J, tau):
    """F_{MM'}(Omega_b) = sum_{M''=M0}^J (-1)^{M'-M''} 2/sqrt(2+2 delta_{M'0})
    F_{M'M''}(0, w_ba, 0) F_{MM''}(Omega_a), eq. (F-ba)."""
    m = (1.0, 1.0, 1836.0)
    M0 = (1 - tau) // 2
    rng = np.random.default_rng(21)
    for _ in range(6):
        r = rng.standard_normal((3, 3))
        X, Y = jacobi_vectors(r, m)
        # random lab orientation
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        for a in range(3):
            for b in range(3):
                if a == b:
                    continue
                xa, ya = q @ X[a], q @ Y[a]
                xb, yb = q @ X[b], q @ Y[b]
                ang_a = euler_zyz(body_frame(xa, ya))
                ang_b = euler_zyz(body_frame(xb, yb))
                x, y = np.linalg.norm(xa), np.linalg.norm(ya)
                z = xa @ ya / (x * y)
                w = w_angle(m, b, a, np.array([x]), np.array([y]), np.array([z]),
                            np.array([np.linalg.norm(yb)]))[0]
                for M in range(-J, J + 1):
                    for Mp in range(M0, J + 1):
                        lhs = F(J, tau, M, Mp, ang_b)
                        rhs = sum((-1) ** (Mp - Mpp) * 2 / math.sqrt(2 + 2 * (Mp == 0))
                                  * F_rot(J, tau, Mp, Mpp, w) * F(J, tau, M, Mpp, ang_a)
                                  for Mpp in range(M0, J + 1))
                        assert abs(lhs - rhs) < 1e-10, (a, b, M, Mp, lhs, rhs)
