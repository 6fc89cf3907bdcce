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


def rel_residuals_by_rows(prob, Es, X, B, chunk=16384, progress=None):
    """||b_r - A(E_r) x_r|| / ||b_r|| for several requests without holding the
    matrix: the rows of H = A(0) and of A(1) are assembled a chunk at a time
    (the residual-only mode for systems too large to factor or to store), and
    A(E) x = H x - E S x with S = A(0) - A(1) (Sec. 3.1: A(E) = H - E S).
    Es: energies; X, B: arrays of shape (len(Es), N)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    ss = np.zeros(len(Es))
    for start in range(0, prob.N, chunk):
        idx = np.arange(start, min(prob.N, start + chunk))
        H = prob.rows(0.0, idx)
        S = H - prob.rows(1.0, idx)
        for r, E in enumerate(Es):
            res = B[r, idx] - (H @ X[r] - E * (S @ X[r]))
            ss[r] += float(res @ res)
        if progress is not None:
            progress(idx[-1] + 1, prob.N)
    return np.sqrt(ss) / np.linalg.norm(B, axis=1)


def rel_residuals_by_rows_complex(prob, Es, X, B, chunk=16384, progress=None):
    """||b - A(E) x|| / ||b|| for complex energies E (Sec. 3.1 with H and S
    real) in the residual-only mode: x = x_r + i x_i and b = b_r + i b_i are
    given as the rows [real part, imaginary part] of X and B (shape
    (len(Es), 2N)); A(E) x = H x - E S x splits into
    H x_r - Re E S x_r + Im E S x_i and H x_i - Re E S x_i - Im E S x_r."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    N = prob.N
    ss = np.zeros(len(Es))
    for start in range(0, N, chunk):
        idx = np.arange(start, min(N, start + chunk))
        H = prob.rows(0.0, idx)
        S = H - prob.rows(1.0, idx)
        for r, E in enumerate(Es):
            E = complex(E)
            xr, xi = X[r, :N], X[r, N:]
            sxr, sxi = S @ xr, S @ xi
            rr = B[r, idx] - (H @ xr - E.real * sxr + E.imag * sxi)
            ri = B[r, N + idx] - (H @ xi - E.real * sxi - E.imag * sxr)
            ss[r] += float(rr @ rr) + float(ri @ ri)
        if progress is not None:
            progress(idx[-1] + 1, N)
    return np.sqrt(ss) / np.linalg.norm(B, axis=1)


def complex_matrix(prob, E):
    """A(E) = H - E S for a complex energy E (Sec. 3.1; H, S real): H = A(0),
    S = A(0) - A(1)."""
    H = prob.assemble(0.0)
    S = H - prob.assemble(1.0)
    return (H.astype(np.complex128) - complex(E) * S).tocsr()


def precond_reference_complex(prob, E, r, couple_m=False):
    """z = L(E)^{-1} r with E and r complex (sparse LU of the complex separable
    operator)."""
    L = prob.separable(complex(E), couple_m=couple_m).tocsc()
    return spla.splu(L).solve(np.asarray(r, dtype=np.complex128))


def precond_reference(prob, E, r, couple_m=False):
    """z = L(E)^{-1} r with L the block-diagonal separable operator."""
    L = prob.separable(E, couple_m=couple_m).tocsc()
    return spla.splu(L).solve(np.asarray(r, dtype=np.float64))


def precond_dense_inverse(prob, E, couple_m=False):
    """Dense inverse of the separable operator (tiny grids only)."""
    return np.linalg.inv(prob.separable(E, couple_m=couple_m).toarray())
