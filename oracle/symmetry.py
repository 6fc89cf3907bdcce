"""Oracle: the exchange-reduced equations for two identical particles (Sec. 2,
"Permutational symmetry", eqs. (2-sym) and (2-sym-part)) and for three
identical particles (eqs. (3-sym) and (3-sym-part)).

Test infrastructure only (see oracle/__init__.py).

With particles 1 and 2 identical and a wave function of parity p under their
exchange, component 2 is p (-1)^{M'} times component 1 at -z (same x, y); the
equations for components 1 and 3 with that substitution are the reduced system
of 2 n_M equations.  Plain definition: E maps the reduced unknowns
(psi_1, psi_3) to the full ones (psi_1, psi_2 = p (-1)^{M'} mirror(psi_1),
psi_3); R keeps the collocation rows of components 1 and 3; then
A_red(E) = R (H - E S) E and S_red = R S E.  mirror takes the coefficients of
f(z) to those of f(-z): interpolation of f(-z_i) at the collocation points,
exact when the nodes and points are symmetric about z = 0.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .eigen import mass_matrix


def mirror_z(bz):
    """Coefficient map f(z) -> f(-z) on the z basis."""
    return np.linalg.solve(bz.matrix(0), bz.matrix(0, t=-bz.points))


def expansion(prob, p):
    """E: reduced unknowns [alpha = 1, 3][M'][z][x][y] -> full unknowns."""
    if p not in (1, -1):
        raise ValueError("p must be +1 or -1")
    rows, cols, vals = [], [], []
    nxy0 = prob.bx[0].n * prob.by[0].n
    Mz = mirror_z(prob.bz[0])
    nz0 = prob.bz[0].n
    red_off = [0, None, prob.nM * prob.block[0]]
    for iM, Mp in enumerate(prob.Mps):
        r0 = red_off[0] + iM * prob.block[0]
        f0 = prob.offsets[0][iM]
        f1 = prob.offsets[1][iM]
        for i in range(prob.block[0]):
            rows.append(f0 + i)
            cols.append(r0 + i)
            vals.append(1.0)
        sign = p * (-1.0) ** Mp
        for k in range(nz0):
            for q in range(nz0):
                w = Mz[k, q]
                if w == 0.0:
                    continue
                for j in range(nxy0):
                    rows.append(f1 + k * nxy0 + j)
                    cols.append(r0 + q * nxy0 + j)
                    vals.append(sign * w)
        r2 = red_off[2] + iM * prob.block[2]
        f2 = prob.offsets[2][iM]
        for i in range(prob.block[2]):
            rows.append(f2 + i)
            cols.append(r2 + i)
            vals.append(1.0)
    nred = prob.nM * (prob.block[0] + prob.block[2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(prob.N, nred))


def kept_rows(prob):
    """Full row indices of components 1 and 3, in the reduced order."""
    idx = []
    for a in (0, 2):
        for iM in range(prob.nM):
            o = prob.offsets[a][iM]
            idx.extend(range(o, o + prob.block[a]))
    return np.array(idx)


def reduced_operator(prob, E, p):
    """A_red(E) = R (H - E S) E."""
    return (prob.assemble(E)[kept_rows(prob)] @ expansion(prob, p)).tocsr()


def reduced_mass(prob, p):
    return (mass_matrix(prob)[kept_rows(prob)] @ expansion(prob, p)).tocsr()


def reduced_shift_invert_eigs(prob, p, sigma, k, tol=1e-13, return_vectors=False):
    """The k energies of the reduced system nearest sigma, nearest first."""
    A = reduced_operator(prob, sigma, p).tocsc()
    S = reduced_mass(prob, p)
    lu = spla.splu(A)
    n = A.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(S @ v), dtype=float)
    v0 = np.ones(n)
    if return_vectors:
        theta, X = spla.eigs(op, k=k, which="LM", tol=tol, v0=v0)
    else:
        theta = spla.eigs(op, k=k, which="LM", tol=tol, v0=v0, return_eigenvectors=False)
    order = np.argsort(-np.abs(theta), kind="stable")
    E = sigma + 1.0 / theta[order]
    return (E, X[:, order]) if return_vectors else E


# -- three identical particles (eq. (3-sym-part)) ------------------------------
# The partial components of all three sets are one function of their own
# coordinates: psi_2 = psi_3 = psi_1 (same bases), so the coefficient vectors
# of components 2 and 3 equal component 1's.  E3 maps component 1's unknowns
# to the full ones, R3 keeps component 1's rows, A_red(E) = R3 (H - E S) E3.
# Both parities p of the full permutations are held by this one equation (its
# solutions split into the parts even and odd under psi_1(x, y, z) ->
# (-1)^{M'} psi_1(x, y, -z)).

def expansion3(prob):
    """E3: component-1 unknowns [M'][z][x][y] -> full unknowns."""
    n1 = prob.nM * prob.block[0]
    if not (prob.block[0] == prob.block[1] == prob.block[2]):
        raise ValueError("three identical particles need identical component bases")
    I = sp.identity(n1, format="csr")
    return sp.vstack([I, I, I], format="csr")


def kept_rows3(prob):
    return np.arange(prob.offsets[0][0], prob.offsets[0][0] + prob.nM * prob.block[0])


def reduced_operator3(prob, E):
    """A_red(E) = R3 (H - E S) E3."""
    return (prob.assemble(E)[kept_rows3(prob)] @ expansion3(prob)).tocsr()


def reduced_mass3(prob):
    return (mass_matrix(prob)[kept_rows3(prob)] @ expansion3(prob)).tocsr()


# -- the symmetric component on z in [0, 1] (the last remark of Sec. 2) ---------
# With two identical particles and n_M = 1, component 3 has the parity
# sigma = p (-1)^{M0} about z = 0 (eq. (2-sym-part)); it is represented by the
# half basis (oracle.basis.half_z_basis) and extended to z < 0 by the parity.
# Plain definition: E_h maps (psi_1, psi_3 on [0, 1]) to the full unknowns
# (psi_1, psi_2 = p (-1)^{M'} mirror(psi_1), psi_3 = extension); R_h keeps the
# rows of component 1 and the rows of component 3 at the half basis's points;
# A_half(E) = R_h (H - E S) E_h.

def half_parity(prob, p):
    return p * (-1) ** prob.M0


def z_extension(bz_full, bz_half, sigma):
    """Full-basis coefficients of f(z) = sigma^[z < 0] g(|z|), g in the half
    basis (exact: the full basis's nodes are the half ones mirrored)."""
    t = bz_full.points
    sign = np.where(t < 0.0, float(sigma), 1.0)
    vals = sign[:, None] * bz_half.matrix(0, t=np.abs(t))
    return np.linalg.solve(bz_full.matrix(0), vals)


def expansion_half(prob, p, bz_half):
    if prob.nM != 1:
        raise ValueError("the halved z-domain needs n_M = 1")
    sigma = half_parity(prob, p)
    Ered = expansion(prob, p).tocsr()              # (psi_1, psi_3 full) -> full unknowns
    n1, n3 = prob.block[0], prob.block[2]
    nxy3 = prob.bx[2].n * prob.by[2].n
    X = z_extension(prob.bz[2], bz_half, sigma)    # nz_full x nz_half
    ext = sp.kron(sp.csr_matrix(X), sp.identity(nxy3), format="csr")
    T = sp.block_diag([sp.identity(n1), ext], format="csr")
    return (Ered @ T).tocsr()


def kept_rows_half(prob, bz_half):
    """Rows of component 1, then rows of component 3 at the half basis's points."""
    o1, o3 = prob.offsets[0][0], prob.offsets[2][0]
    nxy3 = prob.bx[2].n * prob.by[2].n
    full_pts = prob.bz[2].points
    zi = [int(np.argmin(np.abs(full_pts - t))) for t in bz_half.points]
    assert np.allclose(full_pts[zi], bz_half.points, atol=1e-15)
    rows3 = np.concatenate([o3 + k * nxy3 + np.arange(nxy3) for k in zi])
    return np.concatenate([np.arange(o1, o1 + prob.block[0]), rows3])


def reduced_operator_half(prob, E, p, bz_half):
    """A_half(E) = R_h (H - E S) E_h."""
    return (prob.assemble(E)[kept_rows_half(prob, bz_half)] @ expansion_half(prob, p, bz_half)).tocsr()


def separable_half(prob, E, bz_half):
    """The preconditioner's separable operator of the halved system:
    block-diagonal (L_1 on the full grid, L_3 on the half z basis)."""
    import copy
    q = copy.copy(prob)
    q.bz = list(prob.bz)
    q.bz[2] = bz_half
    return sp.block_diag([prob.separable_block(0, E), q.separable_block(2, E)], format="csr")
