"""Pins for the oracle of the coupled L > 0 preconditioner (paper Sec. 3.2, the
approximate matrix script-L, and the Appendix).

P-V2a  g_l^{M'} of eq. (g-def) against SciPy's associated Legendre functions
       and against their orthonormality with weight (1-z^2)^{M'}.
P-V2b  The eigen and ladder relations (g-ev), (g-ud) that the Appendix states
       for g, on exact polynomial interpolants of the oracle's values.
P-V2c  Appendix statement 2: with a polynomial basis and collocation at the
       roots of g_{M'+n_z}^{M'}, W-bar^{M'} D^{M'+-} W^{M'+-1} equals the
       oracle's Lambda^{M'+-} and W-bar^{M'} D^{M'} W^{M'} its Lambda_z^{M'}.
P-V2d  The same statement on the library's own z grid where it applies (one
       interval, M' = 0: Gauss points are the roots of P_{n_z}): the oracle's
       normalised pencil is exact and script-L equals the separable operator.
P-V2e  On a many-interval spline grid the oracle's normalised pencils make the
       low-mode corner of W-bar D^{M'+-} W close to Lambda^{M'+-} (statement 1),
       which fixes their sign and scale.
P-V2f  The coupled preconditioner cuts the GMRES iteration count against the
       block-Jacobi one on an L = 2 problem (the purpose stated in Sec. 3.2).
P-V2g  Modes whose eigenvector does not fit g_l^{M'}: with no mode resolved
       script-L is the block-Jacobi separable operator; with some modes left
       out it acts on those modes as that operator does and on a vector of
       resolved modes away from them as the paper's matrix does; the fit
       residuals are ~1e-14 up to the spline's polynomial degree and the
       highest modes of a short quintic grid are not resolved at the default.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import scipy.special as sps
from numpy.polynomial import legendre as npleg

from oracle.assemble import Problem
from oracle.basis import Basis1D
from oracle.precond_v2 import (approx_operator, g_assoc, lam_z, lam_z_minus, lam_z_plus,
                               precond_v2_factory, precond_v2_reference, z_operators,
                               z_pencil)
from paper_2005_05398_amd import workloads as W


@pytest.mark.parametrize("Mp", [0, 1, 2, 4])
def test_g_matches_scipy_and_is_orthonormal(Mp):
    z = np.linspace(-0.97, 0.97, 41)
    for l in range(Mp, Mp + 9):
        norm = math.sqrt((2 * l + 1) / 2 * math.factorial(l - Mp) / math.factorial(l + Mp))
        want = norm * sps.lpmv(Mp, l, z) / (1 - z * z) ** (Mp / 2)
        np.testing.assert_allclose(g_assoc(l, Mp, z), want, rtol=1e-11, atol=1e-11)
    assert np.all(g_assoc(Mp - 1, Mp, z) == 0) if Mp > 0 else True
    t, w = npleg.leggauss(40)
    G = np.stack([g_assoc(l, Mp, t) for l in range(Mp, Mp + 9)])
    gram = (G * (w * (1 - t * t) ** Mp)) @ G.T
    np.testing.assert_allclose(gram, np.eye(9), atol=1e-12)


def _poly(l, Mp):
    """Exact polynomial (Legendre series) through the oracle's g values."""
    deg = max(l - Mp, 0)
    t = np.cos(np.pi * (np.arange(deg + 8) + 0.5) / (deg + 8))
    return npleg.Legendre.fit(t, g_assoc(l, Mp, t), deg, domain=[-1, 1])


@pytest.mark.parametrize("Mp", [0, 1, 2, 3])
def test_g_eigen_and_ladder_relations(Mp):
    z = np.linspace(-0.9, 0.9, 13)
    for l in range(max(Mp, 1), Mp + 7):
        g = _poly(l, Mp)
        d0 = (1 - z * z) * g.deriv(2)(z) - 2 * (Mp + 1) * z * g.deriv(1)(z) - Mp * (Mp + 1) * g(z)
        np.testing.assert_allclose(d0, -l * (l + 1) * g(z), atol=1e-9 * l * l)
        if l >= Mp + 1:        # d^{M'+} g_l^{M'+1} = -lambda^{l, M'} g_l^{M'}
            gp = _poly(l, Mp + 1)
            dp = -(1 - z * z) * gp.deriv(1)(z) + 2 * (Mp + 1) * z * gp(z)
            lam_p = math.sqrt(l * (l + 1) - Mp * (Mp + 1))
            np.testing.assert_allclose(dp, -lam_p * g(z), atol=1e-9 * l * l)
        if Mp >= 1:            # d^{M'-} g_l^{M'-1} = +lambda^{l, -M'} g_l^{M'}
            gm = _poly(l, Mp - 1)
            lam_m = math.sqrt(l * (l + 1) - Mp * (Mp - 1))
            np.testing.assert_allclose(-gm.deriv(1)(z), lam_m * g(z), atol=1e-9 * l * l)


def _legendre_collocation(Mp, nz):
    """Statement 2 set-up for block M': Legendre-series basis P_0..P_{nz-1},
    collocation at the roots of g_{M'+nz}^{M'}; returns points, S, and the
    coefficient matrix W whose column k represents g_{M'+k}^{M'}."""
    pts = np.sort(_poly(Mp + nz, Mp).roots().real)
    assert len(pts) == nz and np.all(np.abs(pts) < 1)
    S = npleg.legvander(pts, nz - 1)
    Wc = np.zeros((nz, nz))
    for k in range(nz):
        c = _poly(Mp + k, Mp).coef
        Wc[:len(c), k] = c
    return pts, S, Wc


def _apply(op, Mp, pts, coef_cols):
    """Values at pts of d_z^{M'} (op 0), d_z^{M'+} (op 1) or d_z^{M'-} (op 2)
    applied to the Legendre series in the columns of coef_cols."""
    out = np.zeros((len(pts), coef_cols.shape[1]))
    for j in range(coef_cols.shape[1]):
        f = npleg.Legendre(coef_cols[:, j])
        if op == 0:
            v = (1 - pts ** 2) * f.deriv(2)(pts) - 2 * (Mp + 1) * pts * f.deriv(1)(pts) - Mp * (Mp + 1) * f(pts)
        elif op == 1:
            v = -(1 - pts ** 2) * f.deriv(1)(pts) + 2 * (Mp + 1) * pts * f(pts)
        else:
            v = -f.deriv(1)(pts)
        out[:, j] = v
    return out


@pytest.mark.parametrize("Mp,nz", [(0, 5), (1, 6), (2, 7), (3, 5)])
def test_lambda_matrices_exact_for_legendre_root_collocation(Mp, nz):
    pts, S, Wm = _legendre_collocation(Mp, nz)
    Wbar = np.linalg.inv(S @ Wm)
    np.testing.assert_allclose(Wbar @ _apply(0, Mp, pts, Wm), lam_z(Mp, nz), atol=1e-8 * nz ** 4)
    _, _, Wp = _legendre_collocation(Mp + 1, nz)
    np.testing.assert_allclose(Wbar @ _apply(1, Mp, pts, Wp), lam_z_plus(Mp, nz), atol=1e-9 * nz ** 3)
    if Mp >= 1:
        _, _, Wn = _legendre_collocation(Mp - 1, nz)
        np.testing.assert_allclose(Wbar @ _apply(2, Mp, pts, Wn), lam_z_minus(Mp, nz), atol=1e-9 * nz ** 3)


@pytest.mark.parametrize("deg,n", [(3, 4), (5, 6)])
def test_normalised_z_pencil_exact_on_one_interval(deg, n):
    b = Basis1D(deg, n, "z", 2.0, "sin")
    Wbar, Wz, lam_t = z_pencil(b, 0)
    np.testing.assert_allclose(lam_t, np.diag(lam_z(0, n)), atol=1e-9)
    vals = b.matrix(0) @ Wz
    for k in range(n):
        np.testing.assert_allclose(vals[:, k], g_assoc(k, 0, b.points), atol=1e-10)
    d0, _, _ = z_operators(b, 0)
    np.testing.assert_allclose(Wbar @ d0 @ Wz, lam_z(0, n), atol=1e-9)
    np.testing.assert_allclose(Wbar @ b.matrix(0) @ Wz, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("deg_z", [3, 5])
def test_script_L_equals_separable_when_statement_2_holds(deg_z):
    nz = 4 if deg_z == 3 else 6
    desc = W.make_desc(*W.PS_MINUS, 8, nz, J=0, tau=1, deg_xy=3, deg_z=deg_z, R=20.0)
    P = Problem(desc)
    E = -0.3
    got = approx_operator(P, E)
    want = P.separable(E).toarray()
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    r = W.rhs(11, P.N)
    z = precond_v2_reference(P, E, r)
    np.testing.assert_allclose(want @ z, r, atol=1e-9 * np.abs(r).max())


# cubic z pencils with M' >= 3 have complex pairs on these grids, so the cubic
# cases stop at M'+1 = 2
@pytest.mark.parametrize("deg,n,Mp", [(3, 32, 0), (3, 32, 1), (5, 24, 0), (5, 24, 1), (5, 24, 2), (5, 24, 3)])
def test_normalised_pencils_approach_lambda_pm(deg, n, Mp):
    b = Basis1D(deg, n, "z", 2.0, "sin")
    Wbar, _, _ = z_pencil(b, Mp)
    _, dp, dm = z_operators(b, Mp)
    k = 4
    _, Wp, _ = z_pencil(b, Mp + 1)
    got = (Wbar @ dp @ Wp)[:k, :k]
    np.testing.assert_allclose(got, lam_z_plus(Mp, n)[:k, :k], atol=2e-3 * abs(lam_z_plus(Mp, n)[1, 0]))
    if Mp >= 1:
        _, Wn, _ = z_pencil(b, Mp - 1)
        got = (Wbar @ dm @ Wn)[:k, :k]
        np.testing.assert_allclose(got, lam_z_minus(Mp, n)[:k, :k], atol=2e-3 * abs(lam_z_minus(Mp, n)[0, 1]))


def test_coupled_preconditioner_cuts_iterations():
    desc = W.make_desc(*W.PS_MINUS, 12, 8, J=2, tau=1, deg_xy=3, deg_z=3, R=20.0)
    P = Problem(desc)
    E = -0.2
    A = P.assemble(E).tocsc()
    b = W.rhs(4001, P.N)
    v1 = spla.splu(P.separable(E).tocsc()).solve
    counts = {}
    for name, f in (("v1", v1), ("v2", precond_v2_factory(P, E))):
        it = [0]

        def cb(_):
            it[0] += 1

        x, info = spla.gmres(A, b, M=spla.LinearOperator(A.shape, matvec=f), rtol=1e-10, restart=200,
                             maxiter=2000, callback=cb, callback_type="pr_norm")
        assert info == 0
        assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b)
        counts[name] = it[0]
    assert counts["v2"] <= 0.7 * counts["v1"], counts


def _chain_inverse(P, a, E, r):
    """script-L_alpha^-1 r by the paper's own route (Sec. 3.2 after eq. (prop-eq)):
    x pencils per l, y pencils per (l, i_x) with the Y_r2 S_y mass (eq. (ops)),
    and the tridiagonal solve in M' with the P-block entries; the z pencils are
    the oracle's."""
    from oracle import physics as ph
    from oracle.wigner import lam, lam_hat_minus, lam_hat_plus
    import scipy.linalg as sla
    d, J = P.desc, P.J
    bz, bx, by = P.bz[a], P.bx[a], P.by[a]
    nz, nx, ny = bz.n, bx.n, by.n
    Sx, D2x, Sy, D2y = bx.matrix(0), bx.matrix(2), by.matrix(0), by.matrix(2)
    Xr2, Yr2 = np.diag(1 / bx.points ** 2), np.diag(1 / by.points ** 2)
    Vx = np.diag(ph.coulomb(d["masses"], d["charges"], a, bx.points))
    Vh = np.diag(ph.v_hat(d, a, by.points))
    Ms = P.Mps
    t = r.reshape(len(Ms), nz, nx, ny).copy()
    zp = [z_pencil(bz, Mp) for Mp in Ms]
    for i in range(len(Ms)):
        t[i] = np.einsum("kq,qxy->kxy", zp[i][0], t[i])
    xs, ys = {}, {}
    for l in range(Ms[0], Ms[-1] + nz):
        lx, Wx = sla.eig(-D2x + l * (l + 1) * Xr2 @ Sx + Vx @ Sx, Sx)
        lx, Wx = lx.real, Wx.real
        xs[l] = (np.linalg.inv(Sx @ Wx), Wx, lx)
        for ix in range(nx):
            ly, Wy = sla.eig(-D2y + Vh @ Sy - E * Sy + lx[ix] * Sy, Yr2 @ Sy)
            ly, Wy = ly.real, Wy.real
            ys[l, ix] = (np.linalg.inv(Yr2 @ Sy @ Wy), Wy, ly)
    for i, Mp in enumerate(Ms):
        for k in range(nz):
            l = Mp + k
            t[i, k] = xs[l][0] @ t[i, k]
            for ix in range(nx):
                t[i, k, ix] = ys[l, ix][0] @ t[i, k, ix]
    for l in range(Ms[0], Ms[-1] + nz):
        idx = [i for i, Mp in enumerate(Ms) if 0 <= l - Mp < nz]
        for ix in range(nx):
            for iy in range(ny):
                T = np.zeros((len(idx), len(idx)))
                for p, i in enumerate(idx):
                    Mp = Ms[i]
                    T[p, p] = ys[l, ix][2][iy] + J * (J + 1) - 2 * Mp * Mp + l * (l + 1)
                    if p + 1 < len(idx):
                        T[p, p + 1] = -lam_hat_plus(J, Mp) * lam(l, Mp)
                    if p >= 1:
                        T[p, p - 1] = -lam_hat_minus(J, Mp) * lam(l, -Mp)
                rhs = np.array([t[i, l - Ms[i], ix, iy] for i in idx])
                sol = np.linalg.solve(T, rhs)
                for p, i in enumerate(idx):
                    t[i, l - Ms[i], ix, iy] = sol[p]
    for i, Mp in enumerate(Ms):
        for k in range(nz):
            l = Mp + k
            for ix in range(nx):
                t[i, k, ix] = ys[l, ix][1] @ t[i, k, ix]
            t[i, k] = xs[l][1] @ t[i, k]
        t[i] = np.einsum("kq,qxy->kxy", zp[i][1], t[i])
    return t.ravel()


@pytest.mark.parametrize("J,tau,deg_z,nz", [(2, 1, 3, 6), (3, -1, 5, 6), (1, 1, 3, 4)])
def test_script_L_inverse_matches_paper_diagonal_chain(J, tau, deg_z, nz):
    desc = W.make_desc(*W.PS_MINUS, 6, nz, J=J, tau=tau, deg_xy=3, deg_z=deg_z, R=20.0)
    P = Problem(desc)
    E = -0.25
    r = W.rhs(5, P.N)
    got = precond_v2_reference(P, E, r, fit_tol=math.inf)      # the paper's matrix: every mode
    o = 0
    for a in range(3):
        n = P.nM * P.block[a]
        want = _chain_inverse(P, a, E, r[o:o + n])
        np.testing.assert_allclose(got[o:o + n], want, rtol=0, atol=1e-9 * np.abs(want).max())
        o += n


def _mode_grid():
    """A quintic z grid of three intervals (n_z = 12) at J = 3: the pencil's
    highest modes of the larger M' do not represent their g_l^{M'}."""
    return W.make_desc(*W.PS_MINUS, 6, 12, J=3, tau=1, deg_xy=3, deg_z=5, R=20.0)


def test_mode_fits_exact_to_the_spline_degree_and_poor_at_the_top():
    from oracle.precond_v2 import DEFAULT_MODE_FIT_TOL, z_modes
    P = Problem(_mode_grid())
    bz = P.bz[0]
    unresolved = 0
    for Mp in P.Mps:
        _, Wz, _, res = z_modes(bz, Mp, DEFAULT_MODE_FIT_TOL)
        vals = bz.matrix(0) @ Wz
        for k in range(6):        # g_{M'+k}^{M'} is a polynomial of degree k <= 5: reproduced
            assert res[k]
            np.testing.assert_allclose(vals[:, k], g_assoc(Mp + k, Mp, bz.points), atol=1e-10)
        unresolved += int((~res).sum())
    assert unresolved > 0


def test_script_L_with_no_mode_resolved_is_block_jacobi():
    P = Problem(_mode_grid())
    E = -0.3
    got = approx_operator(P, E, fit_tol=-1.0)
    want = P.separable(E).toarray()
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_script_L_on_left_out_and_on_resolved_modes():
    """In the z-transformed basis (columns of W_z), script-L with some modes
    left out equals the block-Jacobi operator on a vector of a left-out mode,
    and the paper's matrix on a vector of a resolved mode whose l-chain
    neighbours are resolved too."""
    from oracle.precond_v2 import DEFAULT_MODE_FIT_TOL, approx_block, z_modes
    P = Problem(_mode_grid())
    E = -0.3
    a = 0
    nz, nxy = P.bz[a].n, P.bx[a].n * P.by[a].n
    modes = [z_modes(P.bz[a], Mp, DEFAULT_MODE_FIT_TOL) for Mp in P.Mps]
    Lh, Wbh, Wh = approx_block(P, a, E)
    Lp, Wbp, Wp = approx_block(P, a, E, fit_tol=math.inf)
    hyb = np.linalg.inv(Wbh.toarray()) @ Lh.toarray() @ np.linalg.inv(Wh.toarray())
    pap = np.linalg.inv(Wbp.toarray()) @ Lp.toarray() @ np.linalg.inv(Wp.toarray())
    sep = P.separable(E).toarray()[:P.nM * P.block[a], :P.nM * P.block[a]]
    f = W.rhs(3, nxy)
    checked = {"left_out": 0, "resolved": 0}
    for iM in range(P.nM):
        res = modes[iM][3]
        for k in range(nz):
            e = np.zeros(P.nM * nz)
            e[iM * nz + k] = 1.0
            v = Wh.toarray() @ np.kron(e, f)      # the mode's eigenvector times f
            if not res[k]:
                np.testing.assert_allclose(hyb @ v, sep @ v, atol=1e-9 * np.abs(sep @ v).max())
                checked["left_out"] += 1
            else:
                l = P.Mps[iM] + k
                nb = [(j, l - P.Mps[j]) for j in (iM - 1, iM + 1) if 0 <= j < P.nM and 0 <= l - P.Mps[j] < nz]
                if all(modes[j][3][kk] for j, kk in nb):
                    np.testing.assert_allclose(hyb @ v, pap @ v, atol=1e-9 * np.abs(pap @ v).max())
                    checked["resolved"] += 1
    assert checked["left_out"] > 0 and checked["resolved"] > 0, checked
