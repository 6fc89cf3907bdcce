"""Oracle: the coupled L > 0 preconditioner of Sec. 3.2 (the approximate matrix
script-L of the paper, with the M'+-1 blocks kept).

Test infrastructure only (see oracle/__init__.py).

For a component alpha the separable operator L_alpha of eq. (FM-fin) is
written as W-bar_z^-1 L_alpha^xy W_z^-1 (eq. (z-dec) and the block matrices
after it), where W_z^{M'} diagonalises the z pencil (D_z^{M'}, S_z) and the
blocks of L_alpha^xy are eq. (L-exact) and eq. (L-pm-exact).  The paper then
replaces the computed z eigenvalues by -l(l+1), l = M'+k, and the transformed
M'+-1 blocks W-bar_z^{M'} D_z^{M'+-} W_z^{M'+-1} by the bidiagonal Lambda^{M'+-}
(eq. (prop-eq)); the result is the block script-L_alpha^xy and
script-L_alpha = W-bar_z^-1 script-L_alpha^xy W_z^-1.  Its inverse is the
preconditioner (eqs. (prec-1), (prec-2)).

The paper reaches script-L_alpha^-1 through three more diagonalisations and a
tridiagonal solve in M'; that chain is exact, so the plain definition used
here is the assembled script-L_alpha^xy solved by sparse LU:
    z_alpha = W_z (script-L_alpha^xy)^-1 W-bar_z r_alpha.

The equalities (prop-eq) presuppose that the columns of W_z^{M'} represent the
functions g_l^{M'} of eq. (g-def) (Appendix), including their scale and sign:
the eigenvectors, which a pencil fixes only up to a factor, are ordered by
ascending |lambda~| (column k <-> l = M'+k) and each is scaled by the
least-squares factor that maps its values at the collocation points onto
g_{M'+k}^{M'} there.  W-bar_z^{M'} = (S_z W_z^{M'})^-1 then keeps
W-bar_z S_z W_z = I of eq. (z-dec).

Only the pencil's lower modes are such functions: the spline space
reproduces g_l^{M'} (a polynomial of degree l - M') exactly up to its
polynomial degree, and approximately for a while beyond; the highest modes'
eigenvectors can be nearly orthogonal to their g (a least-squares scale near
zero, which would blow W-bar_z up).  The substitution is therefore made for
the modes whose fit has a relative residual of at most a tolerance (the
description's mode_fit_tol, default DEFAULT_MODE_FIT_TOL); the others keep
their computed eigenvalue and lose the M'+-1 entries that touch them, as in
the block-Jacobi variant.  With every mode resolved this is the paper's
script-L; with none, the block-Jacobi operator.
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as npleg

from . import physics as ph
from .wigner import lam, lam_hat_minus, lam_hat_plus


def g_assoc(l, Mp, z):
    """g_l^{M'}(z) of eq. (g-def): sqrt((2l+1)/2 (l-M')!/(l+M')!) P_l^{M'}(z) /
    (1-z^2)^{M'/2}, with P_l^{M'} the associated Legendre function
    (Condon-Shortley phase), i.e. (-1)^{M'} times the M'-th derivative of the
    Legendre polynomial P_l.  Zero for l < M'."""
    z = np.asarray(z, dtype=np.float64)
    if l < Mp:
        return np.zeros_like(z)
    c = np.zeros(l + 1)
    c[l] = 1.0
    d = npleg.legder(c, Mp) if Mp else c
    norm = math.sqrt((2 * l + 1) / 2.0 * math.factorial(l - Mp) / math.factorial(l + Mp))
    return (-1.0) ** Mp * norm * npleg.legval(z, d)


def lam_z(Mp, nz):
    """Lambda_z^{M'} = diag{-l(l+1)}, l = M', ..., M'+n_z-1 (eq. (prop-eq))."""
    return np.diag([-float((Mp + k) * (Mp + k + 1)) for k in range(nz)])


def lam_z_plus(Mp, nz):
    """Lambda_z^{M'+}: n_z x n_z, row k (k >= 1) holds -lambda^{M'+k, M'} in
    column k-1 (eq. (prop-eq) and the matrix printed after it)."""
    L = np.zeros((nz, nz))
    for k in range(1, nz):
        L[k, k - 1] = -lam(Mp + k, Mp)
    return L


def lam_z_minus(Mp, nz):
    """Lambda_z^{M'-}: n_z x n_z, row k (k <= n_z-2) holds lambda^{M'+k, -M'}
    in column k+1."""
    L = np.zeros((nz, nz))
    for k in range(nz - 1):
        L[k, k + 1] = lam(Mp + k, -Mp)
    return L


def z_operators(bz, Mp):
    """Collocation matrices of d_z^{M'}, d_z^{M'+} and d_z^{M'-} (eq. (d-def))
    on the z basis: rows at the collocation points, columns basis functions."""
    z = bz.points
    Sz, D1z, D2z = bz.matrix(0), bz.matrix(1), bz.matrix(2)
    d0 = np.diag(1 - z * z) @ D2z - 2 * (Mp + 1) * np.diag(z) @ D1z - Mp * (Mp + 1) * Sz
    dp = -np.diag(1 - z * z) @ D1z + 2 * (Mp + 1) * np.diag(z) @ Sz
    dm = -D1z
    return d0, dp, dm


DEFAULT_MODE_FIT_TOL = 0.02


def mode_fit_tol(desc):
    """The description's tolerance of the z-mode fit (the default where it
    gives none or a value <= 0)."""
    t = float(desc.get("mode_fit_tol", 0.0))
    return t if t > 0 else DEFAULT_MODE_FIT_TOL


def z_modes(bz, Mp, fit_tol):
    """(W-bar_z^{M'}, W_z^{M'}, lambda~, resolved) of the z pencil (D_z^{M'},
    S_z) (eq. (z-dec)): eigenvectors ordered by ascending |lambda~| (column k
    <-> l = M'+k).  Column k is fitted to g_{M'+k}^{M'} at the collocation
    points in least squares; where the relative residual of the fit is at most
    fit_tol the mode is resolved and the column takes the fitted scale (the
    functions that eq. (prop-eq) presupposes), otherwise it is left as the
    pencil gave it.  fit_tol None: every mode resolved."""
    Sz = bz.matrix(0)
    d0, _, _ = z_operators(bz, Mp)
    lam_t, W = sla.eig(d0, Sz)
    if np.abs(lam_t.imag).max() > 1e-9 * np.abs(lam_t).max():
        raise ValueError("z pencil with a complex spectrum")
    lam_t, W = lam_t.real, W.real
    order = np.argsort(np.abs(lam_t), kind="stable")
    lam_t, W = lam_t[order], W[:, order]
    vals = Sz @ W
    resolved = np.zeros(W.shape[1], dtype=bool)
    for k in range(W.shape[1]):
        g = g_assoc(Mp + k, Mp, bz.points)
        s = (g @ vals[:, k]) / (vals[:, k] @ vals[:, k])
        if fit_tol is None or np.linalg.norm(s * vals[:, k] - g) <= fit_tol * np.linalg.norm(g):
            resolved[k] = True
            W[:, k] *= s
    Wbar = np.linalg.inv(Sz @ W)
    return Wbar, W, lam_t, resolved


def z_pencil(bz, Mp):
    """(W-bar_z^{M'}, W_z^{M'}, lambda~) = D(D_z^{M'}, S_z) (eq. (z-dec)),
    ordered by ascending |lambda~| and every column scaled to g_{M'+k}^{M'}
    (module docstring)."""
    return z_modes(bz, Mp, None)[:3]


def approx_block(prob, a, E, fit_tol=None):
    """(script-L_alpha^xy, W-bar_z, W_z) for component alpha at energy E: the
    blocks of eq. (L-exact) / (L-pm-exact) after the substitutions of
    eq. (prop-eq), as sparse matrices over the [M'][k][x][y] index.  The
    substitution is made for the resolved z modes (z_modes with the
    description's tolerance, or fit_tol): a mode that is not resolved keeps its
    computed eigenvalue and the M'+-1 entries that touch it are dropped (the
    block-Jacobi treatment of that mode)."""
    d = prob.desc
    J = prob.J
    tol = mode_fit_tol(d) if fit_tol is None else fit_tol
    bz, bx, by = prob.bz[a], prob.bx[a], prob.by[a]
    nz = bz.n
    Sx, D2x = bx.matrix(0), bx.matrix(2)
    Sy, D2y = by.matrix(0), by.matrix(2)
    x, y = bx.points, by.points
    Xr2 = np.diag(1.0 / x ** 2)
    Yr2 = np.diag(1.0 / y ** 2)
    Vx = np.diag(ph.coulomb(d["masses"], d["charges"], a, x))
    Vh = np.diag(ph.v_hat(d, a, y))
    K = sp.kron
    Iz = sp.identity(nz)
    SxYr = K(Sx, Yr2 @ Sy)
    XrSy = K(Xr2 @ Sx, Sy)
    common = -K(Sx, D2y) - K(D2x, Sy) + K(Vx @ Sx, Sy) + K(Sx, Vh @ Sy) - E * K(Sx, Sy)
    modes = [z_modes(bz, Mp, tol) for Mp in prob.Mps]
    blocks = [[None] * prob.nM for _ in range(prob.nM)]
    for iM, Mp in enumerate(prob.Mps):
        _, _, lam_t, res = modes[iM]
        Lz = np.where(res, np.diag(lam_z(Mp, nz)), lam_t)
        blocks[iM][iM] = K(Iz, common + (J * (J + 1) - 2 * Mp * Mp) * SxYr) - K(np.diag(Lz), SxYr + XrSy)
        if iM + 1 < prob.nM:
            Lp = lam_z_plus(Mp, nz) * np.outer(res, modes[iM + 1][3])
            blocks[iM][iM + 1] = lam_hat_plus(J, Mp) * K(Lp, SxYr)
        if iM - 1 >= 0:
            Lm = lam_z_minus(Mp, nz) * np.outer(res, modes[iM - 1][3])
            blocks[iM][iM - 1] = -lam_hat_minus(J, Mp) * K(Lm, SxYr)
    Lxy = sp.bmat(blocks, format="csc")
    nxy = bx.n * by.n
    Wbar_z = sp.block_diag([K(m[0], sp.identity(nxy)) for m in modes], format="csr")
    W_z = sp.block_diag([K(m[1], sp.identity(nxy)) for m in modes], format="csr")
    return Lxy, Wbar_z, W_z


def approx_operator(prob, E, fit_tol=None):
    """script-L = diag{script-L_1, script-L_2, script-L_3} as a dense matrix
    (tiny grids only)."""
    mats = []
    for a in range(3):
        Lxy, Wbar_z, W_z = approx_block(prob, a, E, fit_tol)
        mats.append(np.linalg.inv(Wbar_z.toarray()) @ Lxy.toarray() @ np.linalg.inv(W_z.toarray()))
    return sla.block_diag(*mats)


def precond_v2_factory(prob, E, fit_tol=None):
    """The map r -> script-L(E)^-1 r (eqs. (prec-1), (prec-2)), component by
    component, with each script-L_alpha^xy factorised once."""
    parts = []
    for a in range(3):
        Lxy, Wbar_z, W_z = approx_block(prob, a, E, fit_tol)
        parts.append((prob.nM * prob.block[a], spla.splu(Lxy), Wbar_z, W_z))

    def apply(r):
        r = np.asarray(r, dtype=np.float64)
        out = np.empty_like(r)
        o = 0
        for n, lu, Wbar_z, W_z in parts:
            out[o:o + n] = W_z @ lu.solve(Wbar_z @ r[o:o + n])
            o += n
        return out

    return apply


def precond_v2_reference(prob, E, r, fit_tol=None):
    """z = script-L(E)^-1 r."""
    return precond_v2_factory(prob, E, fit_tol)(r)
