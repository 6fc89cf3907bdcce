"""Oracle: direct solves, residuals and the preconditioner reference.

Test infrastructure only (see oracle/__init__.py).

The method reaches c = (H - E S)^{-1} b (Sec. 3.1, eq. (FM-lin): the linear
systems with H - E* S that the Krylov iteration solves).  Its plain definition
is an LU solve of the assembled matrix: dense LU for small systems, SuperLU
otherwise.

The preconditioner (Sec. 3.2) is, for every component alpha, the inverse of
the separable left-hand operator L_alpha of eq. (FM-fin) at E* = E.  Its
reference is that inverse, by dense inversion (tiny grids) or by a sparse LU
solve with L_alpha (any grid that fits the host).  The variant without the
M'+-1 blocks is block-diagonal in M'.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def lu_solve(A, b, method="auto"):
    """Solve A x = b (A sparse).  b may hold several right-hand sides as rows."""
    n = A.shape[0]
    if method == "auto":
        method = "dense" if n <= 20000 else "splu"
    B = np.atleast_2d(b)
    if method == "dense":
        lu = sla.lu_factor(A.toarray())
        X = np.stack([sla.lu_solve(lu, r) for r in B])
    else:
        lu = spla.splu(A.tocsc())
        X = np.stack([lu.solve(r) for r in B])
    return X if np.ndim(b) == 2 else X[0]


def rel_residual(A, x, b):
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def precond_reference(prob, E, r, couple_m=False):
    """z = L(E)^{-1} r with L the block-diagonal separable operator."""
    L = prob.separable(E, couple_m=couple_m).tocsc()
    return spla.splu(L).solve(np.asarray(r, dtype=np.float64))


def precond_dense_inverse(prob, E, couple_m=False):
    """Dense inverse of the separable operator (tiny grids only)."""
    return np.linalg.inv(prob.separable(E, couple_m=couple_m).toarray())
