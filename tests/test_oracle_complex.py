"""Pins of the oracle's complex-energy functions (the linear systems
(H - E S) c = b with E and b complex; H and S are real, Sec. 3.1).

* At a real energy the complex matrix equals the directly assembled A(E).
* The complex LU solution equals the solution of the real block form
  [[A(Re E), Im E S], [-Im E S, A(Re E)]] [c_re; c_im] = [b_re; b_im].
* Conjugation: (conj E, conj b) gives conj c (H, S real).
* The residual-only mode for complex energies (rows of H and S a chunk at a
  time) equals the residual through the assembled complex matrix, across
  chunk boundaries, and is zero at the LU solution.
* The complex separable operator of the preconditioner (Sec. 3.2) with the
  potentials off, inverted through the eigenvectors of the generalized
  eigenproblem of (L(0), S_z (x) S_x (x) S_y) (an independent route: the
  divide by lambda - E itself), equals the oracle's LU solve.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.assemble import Problem
from oracle.solve import complex_matrix, lu_solve, precond_reference_complex, rel_residuals_by_rows_complex
from paper_2005_05398_amd import workloads as W


def _prob(J=0):
    return Problem(W.make_desc(*W.PS_MINUS, 7, 4, J=J, deg_z=3, R=15.0))


def _rhs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_complex_matrix_at_real_energy_equals_assembly():
    O = _prob()
    for E in (-0.3, 0.25):
        A = complex_matrix(O, complex(E, 0.0))
        B = O.assemble(E)
        d = np.abs((A - B).toarray()).max()
        assert d <= 1e-13 * np.abs(B.toarray()).max()


def test_complex_solution_equals_real_block_form():
    for J in (0, 1):
        O = _prob(J)
        E = -0.31 + 0.07j
        b = _rhs(O.N, 3)
        c = lu_solve(complex_matrix(O, E), b)
        Ar = O.assemble(E.real)
        S = O.assemble(0.0) - O.assemble(1.0)
        K = sp.bmat([[Ar, E.imag * S], [-E.imag * S, Ar]], format="csc")
        u = spla.spsolve(K, np.concatenate([b.real, b.imag]))
        cr = u[:O.N] + 1j * u[O.N:]
        assert np.linalg.norm(c - cr) <= 1e-10 * np.linalg.norm(c), J


def test_conjugate_energy_gives_conjugate_solution():
    O = _prob()
    E = -0.27 + 0.11j
    b = _rhs(O.N, 4)
    c = lu_solve(complex_matrix(O, E), b)
    cc = lu_solve(complex_matrix(O, np.conj(E)), np.conj(b))
    assert np.linalg.norm(cc - np.conj(c)) <= 1e-11 * np.linalg.norm(c)


def test_complex_separable_inverse_through_eigenvectors():
    desc = W.make_desc((1.0, 1.0, 1.0), (0.0, 0.0, 0.0), 6, 4, deg_xy=3, deg_z=3, R=10.0)
    O = Problem(desc)
    L0 = O.separable(0.0).toarray()
    M = (O.separable(0.0) - O.separable(1.0)).toarray()     # the mass S_z (x) S_x (x) S_y per component
    lam, V = sla.eig(L0, M)
    E = 0.4 + 0.23j
    r = _rhs(O.N, 5)
    # L(E) = L(0) - E M = M V diag(lam - E) V^-1
    z_eig = V @ (np.linalg.solve(V, np.linalg.solve(M, r)) / (lam - E))
    z = precond_reference_complex(O, E, r)
    assert np.linalg.norm(z - z_eig) <= 1e-9 * np.linalg.norm(z)


def test_complex_residual_by_rows_matches_assembled_matrix():
    O = _prob(1)
    Es = [-0.31 + 0.07j, 0.2 - 0.01j]
    rng = np.random.default_rng(8)
    X = rng.standard_normal((2, 2 * O.N))
    Bm = rng.standard_normal((2, 2 * O.N))
    want = []
    for r, E in enumerate(Es):
        x = X[r, :O.N] + 1j * X[r, O.N:]
        b = Bm[r, :O.N] + 1j * Bm[r, O.N:]
        want.append(np.linalg.norm(b - complex_matrix(O, E) @ x) / np.linalg.norm(b))
    got = rel_residuals_by_rows_complex(O, Es, X, Bm, chunk=997)     # chunks end inside blocks
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # at the LU solution the residual is at rounding level
    b = Bm[0, :O.N] + 1j * Bm[0, O.N:]
    c = lu_solve(complex_matrix(O, Es[0]), b)
    xs = np.concatenate([c.real, c.imag])[None, :]
    assert rel_residuals_by_rows_complex(O, Es[:1], xs, Bm[:1], chunk=997)[0] <= 1e-12
