"""Pins for the oracle's 1D spline bases (paper Sec. 3.1, Sec. 4).

P1: the collocation matrices reproduce every polynomial of the spline degree
that meets the closure exactly (values, first and second derivatives), at the
collocation points and at arbitrary points.  A wrong shape function, scaling,
derivative factor or index map fails it.
"""
import math

import numpy as np
import pytest

from oracle.basis import Basis1D, hermite_shape_monomials

P = np.polynomial.polynomial


def _random_poly(rng, basis):
    """A random polynomial of degree 2q-1 meeting the basis closure."""
    deg = 2 * basis.q - 1
    if basis.kind == "z":
        return rng.standard_normal(deg + 1)
    # vanishes at 0 and R: t (R - t) r(t)
    r = rng.standard_normal(deg - 1)
    return P.polymul(P.polymul([0.0, 1.0], [basis.R, -1.0]), r)


CASES = [
    (3, 8, "xy", 20.0, "uniform"), (3, 16, "xy", 20.0, "uniform"), (3, 12, "xy", 40.0, "quadratic"),
    (5, 7, "xy", 20.0, "uniform"), (5, 22, "xy", 36.0, "pow"), (5, 64, "xy", 40.0, "quadratic"),
    (5, 31, "xy", 20.0, "uniform"),
    (3, 4, "z", 2.0, "sin"), (3, 8, "z", 2.0, "sin"), (3, 32, "z", 2.0, "sin"),
    (5, 6, "z", 2.0, "sin"), (5, 9, "z", 2.0, "uniform"), (5, 24, "z", 2.0, "sin"),
]


@pytest.mark.parametrize("deg,n,kind,R,mapname", CASES)
def test_polynomial_reproduction(deg, n, kind, R, mapname):
    b = Basis1D(deg, n, kind, R, mapname)
    rng = np.random.default_rng(17 + n + deg)
    p = _random_poly(rng, b)
    c = b.coefficients_of(lambda d, t: P.polyval(t, P.polyder(p, d)))
    scale = max(1.0, np.abs(P.polyval(b.points, p)).max())
    lo = b.nodes[0]
    hi = b.nodes[-1]
    t_rand = rng.uniform(lo, hi, 50)
    for t in (b.points, t_rand):
        for d in range(3):
            got = b.matrix(d, t) @ c
            want = P.polyval(t, P.polyder(p, d))
            sc = max(1.0, np.abs(want).max(), scale)
            assert np.abs(got - want).max() <= 1e-11 * sc, (d, np.abs(got - want).max())


@pytest.mark.parametrize("q", [2, 3])
def test_hermite_shape_conditions(q):
    A = hermite_shape_monomials(q)
    for e, s0 in enumerate((0.0, 1.0)):
        for d in range(q):
            for e2, s1 in enumerate((0.0, 1.0)):
                for d2 in range(q):
                    v = P.polyval(s1, P.polyder(A[e, d], d2)) if d2 else P.polyval(s1, A[e, d])
                    assert abs(v - (1.0 if (e, d) == (e2, d2) else 0.0)) < 1e-12


@pytest.mark.parametrize("deg,n,kind,R,mapname", CASES)
def test_square_system_and_points(deg, n, kind, R, mapname):
    b = Basis1D(deg, n, kind, R, mapname)
    assert b.points.size == b.n == n
    assert np.all(np.diff(b.points) > 0)
    lo, hi = b.nodes[0], b.nodes[-1]
    assert np.all(b.points > lo) and np.all(b.points < hi)
    S = b.matrix(0)
    assert np.linalg.cond(S) < 1e7
    # at most 2q nonzero functions per point
    assert np.max((np.abs(S) > 0).sum(axis=1)) <= 2 * b.q
    if kind == "z" and mapname in ("sin", "uniform"):
        np.testing.assert_allclose(b.points, -b.points[::-1], atol=1e-15)


# Every x, y basis size printed in the paper's tables and figure captions
# (Sec. 4, Tables 1-3, Fig. 4) is admissible for the quintic x, y closure, and
# every printed z size for the quintic z closure.
PAPER_XY = [22, 31, 40, 49, 58, 19, 25, 28, 238, 52, 88, 118, 148, 178, 208, 223, 4, 7]
PAPER_Z = [9, 12, 15, 18, 21, 24, 27, 6]


def test_paper_sizes_admissible():
    for n in PAPER_XY:
        Basis1D(5, n, "xy", 10.0, "uniform")
    for n in PAPER_Z:
        Basis1D(5, n, "z", 2.0, "sin")


def test_unknown_count_matches_paper_table():
    """N = n_M * sum_alpha n_x n_y n_z (Sec. 3.1), with the two components kept
    by the electron symmetry; sizes and N printed in Table 3 (J = 10, tau = 1)."""
    J, tau = 10, 1
    nM = J - (1 - tau) // 2 + 1
    rows = [((58, 58, 6), (4, 4, 6), 223080), ((88, 88, 9), (7, 7, 9), 771507),
            ((118, 118, 9), (7, 7, 9), 1383327), ((118, 118, 12), (7, 7, 12), 1844436)]
    for c1, c3, N in rows:
        assert nM * (math.prod(c1) + math.prod(c3)) == N
