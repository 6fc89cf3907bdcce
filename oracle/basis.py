"""Oracle: 1D Hermite spline bases and collocation grids.

Test infrastructure only (see oracle/__init__.py).

Paper: Sec. 3.1 (local basis functions, zero Dirichlet conditions at the x and
y endpoints, collocation grids) and Sec. 4 (quintic Hermite splines S_5^3,
three functions per node, support of two intervals, node maps, collocation
at Gaussian points).  Cubic Hermite splines (two functions per node) are the
same construction with q = 2.

Readings taken where the paper is silent:
  * q Gauss-Legendre points per interval; the shape functions are derived here
    by solving the Hermite interpolation conditions in the monomial basis.
  * x, y closure (Dirichlet): drop the value function at both ends.  Cubic:
    n = 2K, two Gauss points per interval.  Quintic: n = 3K + 1 (the form of
    every x, y basis size printed in Sec. 4); three Gauss points per interval
    and four in the first interval [t_0, t_1].
  * z closure (no boundary condition): keep all q(K+1) functions; the end
    intervals get one extra Gauss point each; quintic adds one more extra
    point: the middle interval (K odd) or the middle node (K even).
  * The coefficient of the derivative-order-d function at a node is
    hbar^d psi^(d)(node), hbar = R/K (x, y) or 2/K (z).
"""
import math

import numpy as np


def hermite_shape_monomials(q):
    """Monomial coefficients of the 2q Hermite shape functions on [0, 1].

    Returns A of shape (2, q, 2q): A[e, d, p] is the coefficient of s^p in the
    function whose d-th derivative is 1 at end e (0: s=0, 1: s=1) and whose
    other derivatives of order < q vanish at both ends.
    """
    deg = 2 * q
    rows = []
    for e, s0 in enumerate((0.0, 1.0)):
        for d in range(q):
            row = np.zeros(deg)
            for p in range(d, deg):
                row[p] = math.factorial(p) / math.factorial(p - d) * s0 ** (p - d)
            rows.append(row)
    M = np.array(rows)                       # M @ a = (conditions)
    inv = np.linalg.solve(M, np.eye(deg))    # column c = function with condition c set
    A = np.zeros((2, q, deg))
    for e in range(2):
        for d in range(q):
            A[e, d] = inv[:, e * q + d]
    return A


def _poly_eval(coef, s, deriv):
    """Evaluate the deriv-th derivative of sum_p coef[p] s^p."""
    c = np.polynomial.polynomial.polyder(coef, deriv) if deriv else coef
    return np.polynomial.polynomial.polyval(s, c)


def map_nodes(K, R, mapname):
    """Spline nodes t_0 < ... < t_K (Sec. 4 node maps)."""
    i = np.arange(K + 1, dtype=np.float64)
    if mapname == "uniform":
        return R * i / K
    if mapname == "quadratic":
        return R * (i / K) ** 2
    if mapname == "pow":                     # eq. (map-pow)
        return 4.0 * ((1.0 + R / 4.0) ** (i / K) - 1.0)
    if mapname == "sin":                     # z: sin(pi u / 2), u equidistant on [-1, 1]
        u = -1.0 + 2.0 * i / K
        t = np.sin(np.pi * u / 2.0)
        t[0], t[-1] = -1.0, 1.0
        return t
    if mapname == "zuniform":
        return -1.0 + 2.0 * i / K
    raise ValueError(f"unknown node map {mapname!r}")


class Basis1D:
    """A 1D Hermite spline basis with its collocation points.

    kind "xy": Dirichlet at both ends of [0, R].  kind "z": [-1, 1], no condition.
    """

    def __init__(self, degree, n, kind, R=2.0, mapname="uniform", parity=0):
        """kind "zhalf": the part on [0, 1] of the z basis of n functions (n of
        the full basis, an even number K of intervals) for functions of parity
        `parity` (+1 even, -1 odd) about z = 0 (Sec. 2, "Permutational
        symmetry": the symmetric component's z-domain reduced to [0, 1]).  The
        nodes and points are the full basis's ones in [0, 1]; at z = 0 the
        functions of the other parity's derivative orders are dropped (an even
        function has zero odd derivatives there, an odd one zero even ones),
        and z = 0 stays a collocation point only where the full basis has it
        (quintic) and the function can be nonzero there (even)."""
        if degree not in (3, 5):
            raise ValueError("degree must be 3 or 5")
        q = (degree + 1) // 2
        self.degree, self.q, self.kind = degree, q, kind
        dropped = set()
        extra_node_point = None
        if kind == "zhalf":
            full = Basis1D(degree, n, "z", 2.0, mapname)
            if full.K % 2 or parity not in (1, -1):
                raise ValueError("half z basis needs an even number of intervals and parity +-1")
            K = full.K // 2
            self.parity = parity
            self.K, self.R, self.lo = K, 1.0, 0.0
            self.nodes = full.nodes[K:].copy()
            self.nodes[0] = 0.0
            self.hbar = full.hbar
            dropped = {(0, d) for d in range(q) if (d % 2 == 0) != (parity == 1)}
            self.funcs = [(m, d) for m in range(K + 1) for d in range(q) if (m, d) not in dropped]
            self.index = {f: g for g, f in enumerate(self.funcs)}
            self.n = len(self.funcs)
            keep = full.points >= 0.0 if parity == 1 else full.points > 0.0
            self.points = full.points[keep].copy()
            if len(self.points) != self.n:
                raise AssertionError("half closure does not give n points")
            self.shape = hermite_shape_monomials(q)
            return
        self.n = n
        if kind == "xy":
            if degree == 3:
                if n % 2 or n < 2:
                    raise ValueError("cubic x/y basis needs an even n >= 2")
                K = n // 2
                counts = [2] * K
            else:
                if n % 3 != 1 or n < 4:
                    raise ValueError("quintic x/y basis needs n = 3K + 1, K >= 1")
                K = (n - 1) // 3
                counts = [3] * K
                counts[0] = 4
            dropped.update({(0, 0), (K, 0)})
            lo = 0.0
            mapname_eff = mapname
        elif kind == "z":
            if degree == 3:
                if n % 2 or n < 4:
                    raise ValueError("cubic z basis needs an even n >= 4")
                K = (n - 2) // 2
            else:
                if n % 3 or n < 6:
                    raise ValueError("quintic z basis needs n divisible by 3, n >= 6")
                K = n // 3 - 1
            counts = [q] * K
            counts[0] += 1
            counts[-1] += 1
            if degree == 5:
                if K % 2 == 1:
                    counts[(K - 1) // 2] += 1
                else:
                    extra_node_point = K // 2
            R = 2.0
            lo = -1.0
            mapname_eff = "zuniform" if mapname == "uniform" else mapname
        else:
            raise ValueError("kind must be 'xy' or 'z'")
        self.K, self.R, self.lo = K, R, lo
        self.nodes = map_nodes(K, R, mapname_eff)
        self.hbar = R / K
        # global numbering of the kept functions: (node, order) lexicographic
        self.funcs = [(m, d) for m in range(K + 1) for d in range(q) if (m, d) not in dropped]
        self.index = {f: g for g, f in enumerate(self.funcs)}
        if len(self.funcs) != n:
            raise AssertionError("closure does not give n functions")
        # collocation points: Gauss-Legendre per interval (+ extra node point)
        pts = []
        for m in range(K):
            g, _ = np.polynomial.legendre.leggauss(counts[m])
            a, b = self.nodes[m], self.nodes[m + 1]
            pts.extend(0.5 * (a + b) + 0.5 * (b - a) * g)
        if extra_node_point is not None:
            pts.append(self.nodes[extra_node_point])
        self.points = np.sort(np.array(pts))
        if len(self.points) != n:
            raise AssertionError("closure does not give n points")
        self.shape = hermite_shape_monomials(q)

    def interval(self, t):
        """Interval index per point; a point on a node belongs to the interval
        on its right, the last node to the last interval."""
        t = np.asarray(t, dtype=np.float64)
        m = np.searchsorted(self.nodes, t, side="right") - 1
        return np.clip(m, 0, self.K - 1)

    def local(self, t, deriv):
        """Values of the 2q functions nonzero on each point's interval.

        Returns (idx, val) of shape (npts, 2q): global function index (-1 for a
        dropped function, whose value is then 0) and the deriv-th derivative.
        """
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        m = self.interval(t)
        h = self.nodes[m + 1] - self.nodes[m]
        s = (t - self.nodes[m]) / h
        q = self.q
        idx = np.full((t.size, 2 * q), -1, dtype=np.int64)
        val = np.zeros((t.size, 2 * q))
        for e in range(2):
            for d in range(q):
                col = e * q + d
                node = m + e
                g = np.array([self.index.get((int(nd), d), -1) for nd in node])
                v = _poly_eval(self.shape[e, d], s, deriv) * (h / self.hbar) ** d / h ** deriv
                idx[:, col] = g
                val[:, col] = np.where(g >= 0, v, 0.0)
        return idx, val

    def matrix(self, deriv, t=None):
        """Dense matrix B[p, g] = (d/dt)^deriv S^g (t_p) at the given points
        (default: the collocation points)."""
        t = self.points if t is None else np.atleast_1d(t)
        idx, val = self.local(t, deriv)
        B = np.zeros((t.size, self.n))
        for col in range(idx.shape[1]):
            ok = idx[:, col] >= 0
            B[np.nonzero(ok)[0], idx[ok, col]] += val[ok, col]
        return B

    def coefficients_of(self, derivs):
        """Coefficients of a function given its derivatives at the nodes.

        derivs(d, t) -> d-th derivative at t.  c_g = hbar^d f^(d)(t_m).
        """
        c = np.zeros(self.n)
        for g, (m, d) in enumerate(self.funcs):
            c[g] = self.hbar ** d * derivs(d, self.nodes[m])
        return c


def basis_for(dim, kind):
    return Basis1D(dim["degree"], dim["n"], kind, dim.get("R", 2.0), dim.get("map", "uniform"))


def half_z_basis(dim, parity):
    """The z basis of dim restricted to [0, 1] for functions of the given parity."""
    return Basis1D(dim["degree"], dim["n"], "zhalf", 2.0, dim.get("map", "uniform"), parity=parity)
