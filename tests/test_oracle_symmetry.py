"""Pins for the oracle's exchange-reduced equations (Sec. 2, "Permutational
symmetry", eqs. (2-sym), (2-sym-part)).

P-S1  The z mirror map takes the coefficients of a polynomial f (in the spline
      space) to those of f(-z), and is an involution on the symmetric grids.
P-S2  Helium (identical electrons): the lowest energies of the reduced system
      with p = +1 and p = -1 are the full system's 1 1S and 2 3S levels (the
      para and ortho ground states), and the reduced eigenvectors expanded to
      three components are eigenvectors of the full system.
P-S3  Three identical particles (eqs. (3-sym), (3-sym-part)): the full system
      with the same right-hand side in all three components' rows has the
      same solution in all three components (the cyclic permutation of the
      particles maps each component's equation onto the next one's), and it
      equals the solution of the one-component reduced system; the reduced
      system's energies near a shift are energies of the full system; the
      reduced size of the paper's largest helium-trimer basis is the printed
      1 342 683.
"""
import numpy as np
import pytest

from oracle.assemble import Problem
from oracle.basis import Basis1D
from oracle.eigen import mass_matrix, shift_invert_eigs
from oracle.symmetry import (expansion, mirror_z, reduced_mass3, reduced_operator3,
                             reduced_shift_invert_eigs)
from oracle.solve import lu_solve
from paper_2005_05398_amd import workloads as W


@pytest.mark.parametrize("deg,n", [(3, 8), (3, 16), (5, 12), (5, 24)])
def test_mirror_map(deg, n):
    b = Basis1D(deg, n, "z", 2.0, "sin")
    M = mirror_z(b)
    np.testing.assert_allclose(M @ M, np.eye(n), atol=1e-10)
    c = np.polynomial.Polynomial([0.3, -1.1, 0.7, 2.0])          # degree 3: in every spline space here
    coef = np.linalg.solve(b.matrix(0), c(b.points))
    t = np.linspace(-0.95, 0.95, 17)
    np.testing.assert_allclose(b.matrix(0, t=t) @ (M @ coef), c(-t), atol=1e-10)


def test_helium_para_and_ortho_levels():
    d = W.make_desc((1.0, 1.0, 1e15), (-1.0, -1.0, 2.0), 16, 6, deg_xy=5, deg_z=5, R=15.0,
                    xy_map="quadratic", x0=1.0)
    P = Problem(d)
    full = np.sort(shift_invert_eigs(P, -2.9, 3).real)
    para, X = reduced_shift_invert_eigs(P, +1, -2.9, 1, return_vectors=True)
    ortho = reduced_shift_invert_eigs(P, -1, -2.9, 1)
    assert abs(para[0].real - full[0]) <= 1e-9 * abs(full[0]), (para, full)
    assert abs(ortho[0].real - full[1]) <= 1e-9 * abs(full[1]), (ortho, full)
    x = expansion(P, +1) @ X[:, 0].real
    H = P.assemble(0.0)
    S = mass_matrix(P)
    r = np.linalg.norm(H @ x - para[0].real * (S @ x)) / np.linalg.norm(S @ x)
    assert r <= 1e-8, r


def test_reduced_size_of_the_papers_largest_helium_system():
    """Sec. 4: the largest helium basis (Fig. 4, J = 2, electron symmetry, 2 n_M
    equations) gives a matrix of linear size 4246848."""
    d = W.helium_desc((238, 238, 24), (52, 40, 27), dom1=(45.0, 45.0), dom3=(11.0, 6.0), J=2, tau=1)
    P = Problem(d)
    assert P.nM * (P.block[0] + P.block[2]) == 4246848
    assert W.n_unknowns(dict(d, exchange=1)) == 4246848


THREE = (1.0, 1.0, 1.0), (-1.0, -1.0, -1.0)          # three identical particles


@pytest.mark.parametrize("J,deg_z", [(0, 5), (1, 3), (2, 3)])
def test_three_identical_full_solution_is_threefold(J, deg_z):
    prob = Problem(W.make_desc(*THREE, 7, 6 if deg_z == 5 else 4, J=J, deg_z=deg_z, R=12.0, x0=3.0))
    n1 = prob.nM * prob.block[0]
    E = -0.37
    b = np.random.default_rng(40 + J).standard_normal(n1)
    c_full = lu_solve(prob.assemble(E), np.concatenate([b, b, b]))
    c_red = lu_solve(reduced_operator3(prob, E), b)
    scale = np.linalg.norm(c_red)
    for a in range(3):
        assert np.linalg.norm(c_full[a * n1:(a + 1) * n1] - c_red) <= 1e-10 * scale, (J, a)


def test_three_identical_energies_are_full_system_energies():
    import scipy.sparse.linalg as spla
    prob = Problem(W.make_desc(*THREE, 7, 6, R=12.0, x0=3.0))
    sigma = 0.4
    full = shift_invert_eigs(prob, sigma, 20)
    A = reduced_operator3(prob, sigma).tocsc()
    S = reduced_mass3(prob)
    lu = spla.splu(A)
    n = A.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(S @ v), dtype=float)
    theta = spla.eigs(op, k=3, which="LM", tol=1e-13, v0=np.ones(n), return_eigenvectors=False)
    red = sigma + 1.0 / theta
    for e in red:
        assert np.min(np.abs(full - e)) <= 1e-8 * max(1.0, abs(e)), (e, full)


def test_three_identical_reduced_size_of_the_helium_trimer_basis():
    """The paper's largest helium-trimer system (Sec. 4, J = 0, one equation
    by the permutational symmetry of all three atoms): basis (1: 223, 223, 27)
    gives the printed 1 342 683 unknowns."""
    assert 1 * 223 * 223 * 27 == 1342683
    assert W.n_unknowns(dict(W.make_desc(*THREE, 223, 27, deg_z=5), exchange=3)) == 1342683


# -- component 3 on z in [0, 1] ------------------------------------------------

@pytest.mark.parametrize("deg,n", [(3, 6), (3, 10), (5, 9), (5, 15)])
@pytest.mark.parametrize("parity", [1, -1])
def test_half_z_basis_reproduces_polynomials_of_its_parity(deg, n, parity):
    from oracle.basis import half_z_basis
    b = half_z_basis({"degree": deg, "n": n, "map": "sin"}, parity)
    P = np.polynomial.Polynomial
    powers = [k for k in range(2 * b.q) if (k % 2 == 0) == (parity == 1)]
    rng = np.random.default_rng(deg * 10 + n)
    f = P(np.array([rng.standard_normal() if k in powers else 0.0 for k in range(2 * b.q)]))
    c = np.linalg.solve(b.matrix(0), f(b.points))
    t = np.linspace(0.0, 1.0, 23)
    for d in range(3):
        np.testing.assert_allclose(b.matrix(d, t=t) @ c, f.deriv(d)(t) if d else f(t), atol=1e-9)


@pytest.mark.parametrize("p,deg_z,nz", [(1, 5, 9), (-1, 5, 9), (1, 3, 6), (-1, 3, 10)])
def test_halved_system_solution_is_the_reduced_solution(p, deg_z, nz):
    """With a right-hand side of component 3 of parity sigma the reduced
    system's component 3 has that parity; the halved system (component 3 on
    [0, 1]) has the same solution: its component 1 and the parity extension of
    its component 3."""
    from oracle.basis import half_z_basis
    from oracle.symmetry import (expansion_half, half_parity, kept_rows, kept_rows_half,
                                 reduced_operator, reduced_operator_half, z_extension)
    desc = W.make_desc(*W.H_MINUS, 7, nz, deg_z=deg_z, R=15.0)
    prob = Problem(desc)
    sigma = half_parity(prob, p)
    bh = half_z_basis(desc["z"][2], sigma)
    E = -0.35
    rng = np.random.default_rng(7)
    n1, n3 = prob.block[0], prob.block[2]
    nxy = prob.bx[2].n * prob.by[2].n
    b1 = rng.standard_normal(n1)
    # component 3's rows with parity sigma: b(-z) = sigma b(z) on the symmetric points
    pts = prob.bz[2].points
    b3 = rng.standard_normal((len(pts), nxy))
    for k in range(len(pts)):
        kk = int(np.argmin(np.abs(pts + pts[k])))
        if kk > k:
            b3[kk] = sigma * b3[k]
        elif kk == k:
            b3[k] = 0.0 if sigma == -1 else b3[k]
    c_red = lu_solve(reduced_operator(prob, E, p), np.concatenate([b1, b3.ravel()]))
    zi = [int(np.argmin(np.abs(pts - t))) for t in bh.points]
    b_half = np.concatenate([b1, b3[zi].ravel()])
    c_half = lu_solve(reduced_operator_half(prob, E, p, bh), b_half)
    assert np.linalg.norm(c_half[:n1] - c_red[:n1]) <= 1e-9 * np.linalg.norm(c_red)
    X = z_extension(prob.bz[2], bh, sigma)
    c3 = (X @ c_half[n1:].reshape(bh.n, nxy)).ravel()
    assert np.linalg.norm(c3 - c_red[n1:]) <= 1e-9 * np.linalg.norm(c_red)
    assert W.n_unknowns(dict(desc, exchange=p, zhalf=1)) == n1 + bh.n * nxy
