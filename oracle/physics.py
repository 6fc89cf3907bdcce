"""Oracle: particle kinematics and potentials.

Test infrastructure only (see oracle/__init__.py).

Paper Sec. 2.1: reduced masses, the orthogonal map between reduced Jacobi
sets, eq. (JacobiTrans) with its c, s coefficients; the Coulomb pair
potential sqrt(2 mu_a) Z_b Z_c / x_a; the Merkuriev split, eq. (split3b), with
the cut-off of eq. (Mcutoff0).  Sec. 2.2: x_beta, y_beta, z_beta as functions of
(x_alpha, y_alpha, z_alpha).  Sec. 3.1: the potential Vhat_alpha(y) chosen for
bound states (the form with sqrt(2 mu_a(bc)) in the numerator).
Particle and component indices are 0-based here (paper: 1, 2, 3).
"""
import math

import numpy as np


def others(a):
    """The pair (b, c) complementary to particle a, in increasing order."""
    return [b for b in range(3) if b != a]


def reduced_masses(masses):
    """mu_a = m_b m_c / (m_b + m_c),  mu_a(bc) = m_a (m_b + m_c) / M."""
    m = masses
    M = sum(m)
    mu, mu_abc = [], []
    for a in range(3):
        b, c = others(a)
        mu.append(m[b] * m[c] / (m[b] + m[c]))
        mu_abc.append(m[a] * (m[b] + m[c]) / M)
    return mu, mu_abc


def rotation_cs(masses, b, a):
    """Coefficients (c_ba, s_ba) of x_b = c x_a + s y_a, y_b = -s x_a + c y_a."""
    m = masses
    M = sum(m)
    if a == b:
        return 1.0, 0.0
    c = -math.sqrt(m[b] * m[a] / ((M - m[b]) * (M - m[a])))
    # (-1)^(b-a) sgn(a-b); the parity of b-a is the same with 0- or 1-based labels
    s = (-1.0) ** (b - a) * math.copysign(1.0, a - b) * math.sqrt(max(0.0, 1.0 - c * c))
    return c, s


def rotated_coords(x, y, z, c, s):
    """(x_b, y_b, z_b) from (x_a, y_a, z_a) for the pair of sets (b, a)."""
    xb = np.sqrt(np.maximum(c * c * x * x + 2 * s * c * x * y * z + s * s * y * y, 0.0))
    yb = np.sqrt(np.maximum(s * s * x * x - 2 * s * c * x * y * z + c * c * y * y, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        zb = (s * c * (y * y - x * x) + (c * c - s * s) * x * y * z) / (xb * yb)
    zb = np.clip(np.nan_to_num(zb, nan=0.0), -1.0, 1.0)
    return xb, yb, zb


def coulomb(masses, charges, a, x):
    """V_a^C(x) = sqrt(2 mu_a) Z_b Z_c / x."""
    mu, _ = reduced_masses(masses)
    b, c = others(a)
    return math.sqrt(2.0 * mu[a]) * charges[b] * charges[c] / x


def cutoff(x, y, x0, y0, nu):
    """chi(x, y) = 2 / (1 + exp[(x/x0)^nu / (1 + y/y0)]); y0 = inf allowed."""
    denom = 1.0 + (y / y0 if math.isfinite(y0) else 0.0)
    arg = (x / x0) ** nu / denom
    return 2.0 / (1.0 + np.exp(np.minimum(arg, 700.0)))


def v_short(desc, a, x, y):
    """V_a^(s) = chi_a V_a^C (no short-range pair potential)."""
    return cutoff(x, y, desc["x0"], desc["y0"], desc["nu"]) * coulomb(desc["masses"], desc["charges"], a, x)


def v_long(desc, a, x, y):
    """V_a^(l) = (1 - chi_a) V_a^C."""
    return (1.0 - cutoff(x, y, desc["x0"], desc["y0"], desc["nu"])) * coulomb(desc["masses"], desc["charges"], a, x)


def v_hat(desc, a, y):
    """Vhat_a(y) = Z_a (Z_b + Z_c) sqrt(2 mu_a(bc)) / (y + 1)."""
    if desc.get("vhat", 0) != 0:
        raise ValueError("only vhat = 0 is defined")
    _, mu_abc = reduced_masses(desc["masses"])
    Z = desc["charges"]
    b, c = others(a)
    return Z[a] * (Z[b] + Z[c]) * math.sqrt(2.0 * mu_abc[a]) / (y + 1.0)


def potential_field(desc, a, x, y, z):
    """P_a = V_a(x_a) + sum_{b != a} V_b^(l)(x_b, y_b), at points of set a."""
    P = coulomb(desc["masses"], desc["charges"], a, x)
    for b in others(a):
        c, s = rotation_cs(desc["masses"], b, a)
        xb, yb, _ = rotated_coords(x, y, z, c, s)
        P = P + v_long(desc, b, xb, yb)
    return P
