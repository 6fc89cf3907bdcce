"""GPU parity of the exchange-reduced equations (Sec. 2, "Permutational
symmetry", eq. (2-sym-part): two identical particles, components 1 and 3
solved, component 2 = p (-1)^{M'} component 1 at -z) against the oracle's
reduced system R (H - E S) E, and of the energies against the full system;
and of the one-component system of three identical particles (eq.
(3-sym-part): component 1 alone, both partners read from it) against
R3 (H - E S) E3.

Tolerances as the full-system parity tests: operator 1e-11, preconditioner
1e-9, solutions 1e-8, energies 1e-8.
"""
import numpy as np
import pytest

from oracle.assemble import Problem as OracleProblem
from oracle.solve import lu_solve, precond_reference, rel_residual
from oracle.symmetry import kept_rows, reduced_operator
from paper_2005_05398_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fm():
    from paper_2005_05398_amd import fm
    return fm


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


HE = ((1.0, 1.0, 1e15), (-1.0, -1.0, 2.0))
CASES = [
    ("hminus_L0_p+1", W.make_desc(*W.H_MINUS, 13, 6, R=40.0, xy_map="quadratic"), 1),
    ("hminus_L0_p-1", W.make_desc(*W.H_MINUS, 13, 6, R=40.0, xy_map="quadratic"), -1),
    ("helium_L2_p+1", W.make_desc(*HE, 7, 4, J=2, deg_z=3, R=15.0, x0=1.0), 1),
    ("hminus_L1_odd_p-1", W.make_desc(*W.H_MINUS, 7, 6, J=1, tau=-1, deg_z=5, R=15.0), -1),
    # more than three M' blocks (the operator kernels that take them one at a time)
    ("helium_L5_p+1", W.make_desc(*HE, 7, 4, J=5, deg_z=3, R=15.0, x0=1.0), 1),
    ("helium_L4_odd_p-1", W.make_desc(*HE, 7, 4, J=4, tau=-1, deg_z=3, R=15.0, x0=1.0), -1),
]


@pytest.mark.parametrize("name,desc,p", CASES, ids=[c[0] for c in CASES])
def test_reduced_operator_parity(device, name, desc, p):
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p))
    O = OracleProblem(desc)
    n = O.nM * (O.block[0] + O.block[2])
    assert P.N == n
    E = -0.35
    A = reduced_operator(O, E, p)
    X = np.random.default_rng(4).standard_normal((2, n))
    Y = to_dev(np.zeros((2, n)), device)
    P.apply_operator([E, E], to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    for r in range(2):
        ref = A @ X[r]
        assert np.abs(Yg[r] - ref).max() <= 1e-11 * np.abs(ref).max(), (name, r)


@pytest.mark.parametrize("name,desc,p", CASES, ids=[c[0] for c in CASES])
def test_reduced_precond_parity(device, name, desc, p):
    """The preconditioner of the reduced system is that of components 1 and 3."""
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p))
    O = OracleProblem(desc)
    keep = kept_rows(O)
    r = np.random.default_rng(6).standard_normal(len(keep))
    z = to_dev(np.zeros((1, len(keep))), device)
    P.apply_precond([-0.35], to_dev(r[None, :], device), z)
    full = np.zeros(O.N)
    full[keep] = r
    ref = precond_reference(O, -0.35, full)[keep]
    assert np.abs(z.cpu().numpy()[0] - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("name,desc,p", [CASES[0], CASES[2]], ids=[CASES[0][0], CASES[2][0]])
def test_reduced_solve_matches_lu(device, name, desc, p):
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p))
    O = OracleProblem(desc)
    E = -0.3
    A = reduced_operator(O, E, p)
    b = W.rhs(11, A.shape[0])
    xref = lu_solve(A, b)
    x = to_dev(np.zeros((1, A.shape[0])), device)
    st, res = P.solve([E], to_dev(b[None, :], device), x, restart=150, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    xg = x.cpu().numpy()[0]
    assert rel_residual(A, xg, b) <= 1e-10
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-8


def test_helium_table1_row1_by_exchange_parity(device):
    """The first basis set of Table 1 (Sec. 4): the full system's four levels nearest -2.095
    are 2 3P, 2 1P, 3 3P, 3 1P; p = +1 keeps the singlets (the paper's
    reduced equations), p = -1 the triplets, with the same energies."""
    fm = _fm()
    g1, g3, printed = W.HE_TABLE1[0]
    desc = dict(W.helium_desc(g1, g3), precond="coupled")
    out = {}
    for p in (0, 1, -1):
        P = fm.Problem(dict(desc, exchange=p))
        nev = 4 if p == 0 else 2
        st, E, res, info = P.eigs(-2.095, nev=nev, ncv=20, tol=1e-10, max_restarts=40, restart=100, rtol=1e-11,
                                  max_iters=4000)
        assert st == fm.FM_OK, (p, info)
        out[p] = sorted(e.real for e in E)
    full = out[0]
    singlets = [full[1], full[3]]
    triplets = [full[0], full[2]]
    np.testing.assert_allclose(out[1], singlets, rtol=1e-8)
    np.testing.assert_allclose(out[-1], triplets, rtol=1e-8)
    for e, want in zip(out[1], printed):
        assert abs(e - want) <= 5.1e-6


# -- three identical particles (eq. (3-sym-part)): component 1 only ----------

THREE_CASES = [
    ("three_L0_quintic", W.make_desc((1.0, 1.0, 1.0), (-1.0, -1.0, -1.0), 10, 6, R=15.0, x0=3.0)),
    ("three_L1_cubicz", W.make_desc((1.0, 1.0, 1.0), (1.0, 1.0, 1.0), 7, 4, J=1, deg_z=3, R=12.0, x0=3.0)),
    ("three_L2_cubicz", W.make_desc((2.0, 2.0, 2.0), (-1.0, -1.0, -1.0), 7, 4, J=2, deg_z=3, R=12.0, x0=3.0)),
    ("three_L4_cubicz", W.make_desc((2.0, 2.0, 2.0), (-1.0, -1.0, -1.0), 7, 4, J=4, deg_z=3, R=12.0, x0=3.0)),
]


@pytest.mark.parametrize("name,desc", THREE_CASES, ids=[c[0] for c in THREE_CASES])
def test_three_identical_operator_parity(device, name, desc):
    from oracle.symmetry import reduced_operator3
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=3))
    O = OracleProblem(desc)
    n = O.nM * O.block[0]
    assert P.N == n
    Es = [-0.35, 0.2]
    X = np.random.default_rng(14).standard_normal((2, n))
    Y = to_dev(np.zeros((2, n)), device)
    P.apply_operator(Es, to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    for r, E in enumerate(Es):
        ref = reduced_operator3(O, E) @ X[r]
        assert np.abs(Yg[r] - ref).max() <= 1e-11 * np.abs(ref).max(), (name, r)


@pytest.mark.parametrize("name,desc", THREE_CASES, ids=[c[0] for c in THREE_CASES])
def test_three_identical_precond_parity(device, name, desc):
    """The preconditioner of the one-component system is component 1's."""
    from oracle.symmetry import kept_rows3
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=3))
    O = OracleProblem(desc)
    keep = kept_rows3(O)
    r = np.random.default_rng(16).standard_normal(len(keep))
    z = to_dev(np.zeros((1, len(keep))), device)
    P.apply_precond([-0.35], to_dev(r[None, :], device), z)
    full = np.zeros(O.N)
    full[keep] = r
    ref = precond_reference(O, -0.35, full)[keep]
    assert np.abs(z.cpu().numpy()[0] - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("name,desc", [THREE_CASES[0], THREE_CASES[2]], ids=[THREE_CASES[0][0], THREE_CASES[2][0]])
def test_three_identical_solve_is_the_full_solution(device, name, desc):
    """The one-component solve equals the oracle's LU of the reduced system,
    and each component of the full system's solution for the right-hand side
    repeated in all three components (1e-8)."""
    from oracle.symmetry import reduced_operator3
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=3))
    O = OracleProblem(desc)
    E = -0.4
    A = reduced_operator3(O, E)
    n = A.shape[0]
    b = W.rhs(12, n)
    x = to_dev(np.zeros((1, n)), device)
    st, res = P.solve([E], to_dev(b[None, :], device), x, restart=100, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    xg = x.cpu().numpy()[0]
    assert rel_residual(A, xg, b) <= 1e-10
    xref = lu_solve(A, b)
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-8
    xfull = lu_solve(O.assemble(E), np.concatenate([b, b, b]))
    for a in range(3):
        assert np.linalg.norm(xfull[a * n:(a + 1) * n] - xg) <= 1e-8 * np.linalg.norm(xg), a


# -- component 3 on z in [0, 1] (zhalf) ---------------------------------------

HALF_CASES = [
    ("hminus_quintic_p+1", W.make_desc(*W.H_MINUS, 10, 9, R=30.0, xy_map="quadratic"), 1),
    ("hminus_quintic_p-1", W.make_desc(*W.H_MINUS, 10, 15, R=30.0, xy_map="quadratic"), -1),
    ("hminus_cubicz_p+1", W.make_desc(*W.H_MINUS, 7, 10, deg_z=3, R=15.0), 1),
    ("hminus_L1_odd_p+1", W.make_desc(*W.H_MINUS, 7, 9, J=1, tau=-1, deg_z=5, R=15.0), 1),
]


def _half(desc, p):
    from oracle.basis import half_z_basis
    from oracle.symmetry import half_parity
    O = OracleProblem(desc)
    return O, half_z_basis(desc["z"][2], half_parity(O, p))


@pytest.mark.parametrize("name,desc,p", HALF_CASES, ids=[c[0] for c in HALF_CASES])
def test_halved_operator_parity(device, name, desc, p):
    from oracle.symmetry import reduced_operator_half
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p, zhalf=1))
    O, bh = _half(desc, p)
    A = reduced_operator_half(O, -0.35, p, bh)
    assert P.N == A.shape[0]
    X = np.random.default_rng(17).standard_normal((2, P.N))
    Y = to_dev(np.zeros((2, P.N)), device)
    P.apply_operator([-0.35, -0.35], to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    for r in range(2):
        ref = A @ X[r]
        assert np.abs(Yg[r] - ref).max() <= 1e-11 * np.abs(ref).max(), (name, r)


@pytest.mark.parametrize("name,desc,p", HALF_CASES, ids=[c[0] for c in HALF_CASES])
def test_halved_precond_parity(device, name, desc, p):
    import scipy.sparse.linalg as spla
    from oracle.symmetry import separable_half
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p, zhalf=1))
    O, bh = _half(desc, p)
    r = np.random.default_rng(18).standard_normal(P.N)
    z = to_dev(np.zeros((1, P.N)), device)
    P.apply_precond([-0.35], to_dev(r[None, :], device), z)
    ref = spla.spsolve(separable_half(O, -0.35, bh).tocsc(), r)
    assert np.abs(z.cpu().numpy()[0] - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("name,desc,p", [HALF_CASES[0], HALF_CASES[2]], ids=[HALF_CASES[0][0], HALF_CASES[2][0]])
def test_halved_solve_matches_lu(device, name, desc, p):
    from oracle.symmetry import reduced_operator_half
    fm = _fm()
    P = fm.Problem(dict(desc, exchange=p, zhalf=1))
    O, bh = _half(desc, p)
    E = -0.3
    A = reduced_operator_half(O, E, p, bh)
    b = W.rhs(13, A.shape[0])
    x = to_dev(np.zeros((1, A.shape[0])), device)
    st, res = P.solve([E], to_dev(b[None, :], device), x, restart=150, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    xg = x.cpu().numpy()[0]
    assert rel_residual(A, xg, b) <= 1e-10
    xref = lu_solve(A, b)
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-8


def test_halved_helium_energies_equal_the_reduced_ones(device):
    """Helium, J = 0: the lowest singlet (p = +1) and triplet (p = -1) levels
    with component 3 on z in [0, 1] equal those of the reduced system on the
    full z grid (the same space of solutions), to 1e-9."""
    fm = _fm()
    desc = W.make_desc(*HE, 13, 9, R=15.0, x0=1.0, xy_map="quadratic")
    for p, sigma in ((1, -2.9), (-1, -2.17)):
        out = []
        for half in (0, 1):
            P = fm.Problem(dict(desc, exchange=p, zhalf=half))
            st, E, res, info = P.eigs(sigma, nev=1, ncv=16, tol=1e-12, max_restarts=40, restart=100, rtol=1e-12,
                                      max_iters=4000)
            assert st == fm.FM_OK, (p, half, info)
            out.append(E[0].real)
        assert abs(out[0] - out[1]) <= 1e-9 * abs(out[0]), (p, out)
