"""Oracle: bound-state energies, the eigenvalues of H c = E S c (Sec. 3.1,
eq. (FM-lin)).

Test infrastructure only (see oracle/__init__.py).

S is the matrix of the basis products at the collocation points, block
diagonal over (alpha, M'): S_z (x) S_x (x) S_y per block (Sec. 3.1).  The
energies nearest a shift sigma follow from the eigenvalues theta of largest
modulus of (H - sigma S)^-1 S, E = sigma + 1/theta: the paper's Sec. 4 runs
ARPACK's implicitly restarted Arnoldi on S (H - sigma S)^-1, a similar
operator; here ARPACK (SciPy's eigs) runs on (H - sigma S)^-1 S with an LU
factorisation of H - sigma S.  Tiny problems also have the dense generalized
eigenvalue problem solved directly.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def mass_matrix(prob):
    """S: block diagonal over (alpha, M') with blocks S_z (x) S_x (x) S_y."""
    blocks = []
    for a in range(3):
        B = sp.kron(prob.bz[a].matrix(0), sp.kron(prob.bx[a].matrix(0), prob.by[a].matrix(0)))
        blocks += [B] * prob.nM
    return sp.block_diag(blocks, format="csr")


def shift_invert_eigs(prob, sigma, k, tol=1e-13, return_vectors=False):
    """The k energies nearest sigma (complex in general), nearest first; with
    return_vectors also the coefficient vectors (columns)."""
    A = prob.assemble(sigma).tocsc()
    S = mass_matrix(prob)
    lu = spla.splu(A)
    op = spla.LinearOperator((prob.N, prob.N), matvec=lambda v: lu.solve(S @ v), dtype=float)
    v0 = np.ones(prob.N)
    if return_vectors:
        theta, X = spla.eigs(op, k=k, which="LM", tol=tol, v0=v0)
    else:
        theta = spla.eigs(op, k=k, which="LM", tol=tol, v0=v0, return_eigenvectors=False)
    order = np.argsort(-np.abs(theta), kind="stable")
    E = sigma + 1.0 / theta[order]
    return (E, X[:, order]) if return_vectors else E


def dense_eigs(prob):
    """All eigenvalues of the dense pencil (H, S) (tiny problems only)."""
    H = prob.assemble(0.0).toarray()
    S = mass_matrix(prob).toarray()
    return sla.eigvals(H, S)
