"""Pins for the 1D pencils the preconditioner diagonalises (paper Sec. 3.2 and
the Appendix).

P4: z pencil (d_z^{M'}, S_z).  With a single interval the spline space is all
polynomials of degree 2q-1 and the collocation points are the roots of the
Legendre polynomial P_{2q}; the Appendix (statement 2) then makes the
eigenvalues exactly -l(l+1).  With many intervals the low modes approach
-l(l+1), l = M', M'+1, ... (statement 1).

P5: the x pencil with a Coulomb pair potential reproduces hydrogen-like levels
-mu Z^2 / (2 n^2), n >= l + 1, in reduced Jacobi coordinates.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import physics as ph
from oracle.basis import Basis1D


def z_operator(b, Mp):
    z = b.points
    return (np.diag(1 - z * z) @ b.matrix(2) - 2 * (Mp + 1) * np.diag(z) @ b.matrix(1)
            - Mp * (Mp + 1) * b.matrix(0))


@pytest.mark.parametrize("deg,n", [(3, 4), (5, 6)])
def test_z_pencil_single_interval_exact(deg, n):
    b = Basis1D(deg, n, "z", 2.0, "sin")
    np.testing.assert_allclose(np.sort(b.points),
                               np.sort(np.polynomial.legendre.leggauss(n)[0]), atol=1e-15)
    lam = sla.eigvals(z_operator(b, 0), b.matrix(0))
    assert np.abs(lam.imag).max() < 1e-9
    want = -np.array([l * (l + 1) for l in range(n)], dtype=float)
    np.testing.assert_allclose(np.sort(lam.real)[::-1], want, atol=1e-9)


@pytest.mark.parametrize("deg,n,Mp", [(5, 24, 0), (3, 32, 0), (3, 32, 1), (3, 32, 2), (5, 24, 2)])
def test_z_pencil_low_modes(deg, n, Mp):
    b = Basis1D(deg, n, "z", 2.0, "sin")
    lam = sla.eigvals(z_operator(b, Mp), b.matrix(0))
    assert np.abs(lam.imag).max() < 1e-9 * np.abs(lam).max()
    low = np.sort(lam.real)[::-1][:5]
    want = -np.array([l * (l + 1) for l in range(Mp, Mp + 5)], dtype=float)
    np.testing.assert_allclose(low, want, rtol=1e-6 if deg == 5 else 1e-4, atol=1e-7)


@pytest.mark.parametrize("masses,charges,a", [((1.0, 1.0, 1.0), (1.0, -1.0, -1.0), 1),
                                              ((1.0, 1.0, 1836.0), (-1.0, -1.0, 1.0), 0)])
@pytest.mark.parametrize("l", [0, 1])
def test_coulomb_pencil_hydrogen_levels(masses, charges, a, l):
    mu, _ = ph.reduced_masses(masses)
    b_, c_ = ph.others(a)
    Z = charges[b_] * charges[c_]
    assert Z < 0
    b = Basis1D(5, 130, "xy", 150.0, "quadratic")
    x = b.points
    S = b.matrix(0)
    A1 = -b.matrix(2) + np.diag(l * (l + 1) / x ** 2 + ph.coulomb(masses, charges, a, x)) @ S
    lam = np.sort(sla.eigvals(A1, S).real)
    for k, n in enumerate(range(l + 1, l + 4)):
        want = -mu[a] * Z * Z / (2.0 * n * n)
        assert abs(lam[k] - want) < 5e-7 * abs(want), (n, lam[k], want)
