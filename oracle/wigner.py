"""Oracle: Wigner d-functions and the parity-adapted F functions.

Test infrastructure only (see oracle/__init__.py).

Paper Sec. 2.2: D^J_{MM'}(phi, theta, varphi) = exp(-iM phi) d^J_{MM'}(theta)
exp(-iM' varphi), eq. (D-def); the parity-adapted combination F^{J tau}_{MM'},
eq. (F-def); the frame-rotation angle w_{beta alpha}, eq. (euler-ba) and the
branch rule that follows it.

d is evaluated with Wigner's explicit sum.  The paper prints d through a
Jacobi polynomial whose prefactor contains (J-M)! in both numerator and
denominator; the reading taken is sqrt((J+M')!(J-M')!/((J+M)!(J-M)!)),
which is the form the tests compare the sum against.
"""
import math

import numpy as np

from .physics import rotation_cs


def wigner_d(J, M, Mp, theta):
    """d^J_{M M'}(theta) in the paper's index convention (first index M
    multiplies phi, second index M' multiplies varphi)."""
    theta = np.asarray(theta, dtype=np.float64)
    if abs(M) > J or abs(Mp) > J:
        return np.zeros_like(theta)
    c = np.cos(theta / 2.0)
    s = np.sin(theta / 2.0)
    pref = math.sqrt(math.factorial(J + M) * math.factorial(J - M)
                     * math.factorial(J + Mp) * math.factorial(J - Mp))
    total = np.zeros_like(theta)
    for k in range(0, 2 * J + 1):
        a1, a2, a3, a4 = J + Mp - k, k, M - Mp + k, J - M - k
        if min(a1, a2, a3, a4) < 0:
            continue
        den = math.factorial(a1) * math.factorial(a2) * math.factorial(a3) * math.factorial(a4)
        total = total + ((-1.0) ** (M - Mp + k) / den
                         * c ** (2 * J + Mp - M - 2 * k) * s ** (M - Mp + 2 * k))
    return pref * total


def F_rot(J, tau, M, Mp, w):
    """F^{J tau}_{M M'}(0, w, 0) = (d^J_{MM'}(w) + tau (-1)^M' d^J_{M,-M'}(w)) / sqrt(2 + 2 delta_{M'0})."""
    return (wigner_d(J, M, Mp, w) + tau * (-1.0) ** Mp * wigner_d(J, M, -Mp, w)) / math.sqrt(
        2.0 + 2.0 * (Mp == 0))


CYCLIC = {(0, 1), (1, 2), (2, 0)}   # (beta, alpha) pairs (1,2), (2,3), (3,1) of the paper


def w_angle(masses, b, a, x, y, z, yb):
    """w_{beta alpha}: arccos((-s x z + c y)/y_beta) for (beta, alpha) cyclic,
    2 pi minus that otherwise."""
    c, s = rotation_cs(masses, b, a)
    with np.errstate(divide="ignore", invalid="ignore"):
        arg = (-s * x * z + c * y) / yb
    arg = np.clip(np.nan_to_num(arg, nan=1.0), -1.0, 1.0)
    w = np.arccos(arg)
    return w if (b, a) in CYCLIC else 2.0 * np.pi - w


def lam(J, Mp):
    """lambda^{J M'} = sqrt(J(J+1) - M'(M'+1))."""
    return math.sqrt(max(0.0, J * (J + 1) - Mp * (Mp + 1)))


def lam_hat_plus(J, Mp):
    """lambda-hat^{J, M'} = lambda^{J, M'} sqrt(1 + delta_{M'0})."""
    return lam(J, Mp) * math.sqrt(1.0 + (Mp == 0))


def lam_hat_minus(J, Mp):
    """lambda-hat^{J, -M'} = lambda^{J, -M'} sqrt(1 + delta_{M'1})."""
    return lam(J, -Mp) * math.sqrt(1.0 + (Mp == 1))
