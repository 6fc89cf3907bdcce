"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Operator: y = (H - E S) x from fm_apply_operator against the oracle's
assembled matrix (all rows on small grids, sampled rows at full size).
Preconditioner: fm_apply_precond against the exact inverse of the separable
block of eq. (FM-fin) (sparse LU of the oracle's Kronecker-form L_alpha), and
with all potentials switched off against the dense Kronecker-sum inverse.
Solver: fm_solve against the oracle's LU solution (relative residual 1e-10 and
relative solution error 1e-8), the trivial case P^-1 A = I, and the
identical-particle symmetry of the solution.
Tolerances: operator and preconditioner outputs are compared elementwise
relative to the largest output, at 1e-11 (operator; FP64 with sums of at most
a few hundred terms) and 1e-9 (preconditioner: products with eigenvector
matrices of condition up to ~1e3).
"""
import numpy as np
import pytest

from oracle.assemble import Problem as OracleProblem
from oracle.solve import lu_solve, precond_reference, rel_residual
from paper_2005_05398_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fm():
    from paper_2005_05398_amd import fm
    return fm


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


def small(mc, nxy, nz, J=0, tau=1, dxy=5, dz=5, R=15.0, xy_map="uniform", x0=5.0):
    return W.make_desc(*mc, nxy, nz, J=J, tau=tau, deg_xy=dxy, deg_z=dz, R=R, xy_map=xy_map, x0=x0)


def wide(nx, ny, nz, dz):
    """Slices wider than the fused kernels' 32 (and than 192, a former limit):
    x and y sizes set separately."""
    d = W.make_desc(*W.PS_MINUS, nx, nz, deg_xy=5, deg_z=dz, R=20.0)
    d["y"] = W.make_desc(*W.PS_MINUS, ny, nz, deg_xy=5, deg_z=dz, R=20.0)["y"]
    return d


# 199 x 13: x products of side 199 in 64 x 64 tiles; 10 x 229 with quintic z:
# the operator's stencil tile needs 66 KB of LDS (above the 64 KB default)
WIDE_CASES = [("wide_x199_y13", wide(199, 13, 4, 3)), ("wide_x10_y229", wide(10, 229, 6, 5))]

OP_CASES = [
    ("ps_cubic16", W.ps_cubic16()["desc"]),
    ("quintic_7x7x6", small(W.PS_MINUS, 7, 6)),
    ("hminus_10x13x9_quadratic", dict(small(W.H_MINUS, 10, 9, R=30.0, xy_map="quadratic"),
                                      y=W.make_desc(*W.H_MINUS, 13, 9, R=25.0)["y"])),
    ("L1_tau-1", small(W.H_MINUS, 7, 6, J=1, tau=-1, dz=5)),
    ("L2_tau+1", small(W.PS_MINUS, 7, 4, J=2, tau=1, dz=3)),
    ("cubic_ragged_10x6", small(W.PS_MINUS, 10, 6, dxy=3, dz=3)),
    # finite y0 of the cut-off (eq. (Mcutoff0)): V^(s) and the potential field depend on y
    ("hminus_finite_y0", dict(small(W.H_MINUS, 10, 9, R=30.0, xy_map="quadratic"), y0=6.0)),
    ("L2_finite_y0", dict(small(W.PS_MINUS, 7, 4, J=2, tau=1, dz=3), y0=2.5)),
    # more than three M' blocks (up to 16): the kernels that take the blocks one
    # at a time, every spline-order variant
    ("L5_tau+1", small(W.PS_MINUS, 7, 4, J=5, tau=1, dz=3)),
    ("L10_tau+1", small(W.H_MINUS, 7, 4, J=10, tau=1, dz=3)),
    ("L15_tau+1_most_blocks", small(W.PS_MINUS, 7, 4, J=15, tau=1, dz=3)),
    ("L4_tau-1_quintic", small(W.H_MINUS, 7, 6, J=4, tau=-1, dz=5)),
    ("L5_cubic_xy_quintic_z", small(W.PS_MINUS, 10, 6, J=5, tau=1, dxy=3, dz=5)),
    ("L6_cubic", small(W.PS_MINUS, 10, 4, J=6, tau=1, dxy=3, dz=3)),
    # ... and the generic kernel (x and y of different spline orders)
    ("L5_generic_mixed_xy", dict(small(W.PS_MINUS, 7, 4, J=5, tau=1, dz=3),
                                 y=small(W.PS_MINUS, 10, 4, J=5, tau=1, dxy=3, dz=3)["y"])),
] + WIDE_CASES


@pytest.mark.parametrize("name,desc", OP_CASES, ids=[c[0] for c in OP_CASES])
def test_operator_parity(device, name, desc):
    fm = _fm()
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    assert P.N == O.N
    rng = np.random.default_rng(7)
    Es = [-0.25, -0.61]
    X = rng.standard_normal((2, O.N))
    Y = to_dev(np.zeros((2, O.N)), device)
    P.apply_operator(Es, to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    for r, E in enumerate(Es):
        ref = O.assemble(E) @ X[r]
        err = np.abs(Yg[r] - ref).max() / np.abs(ref).max()
        assert err <= 1e-11, (name, r, err)


@pytest.mark.parametrize("cfg", ["hminus_scan", "ps_q127", "ps_l2_q97"])
def test_operator_parity_full_size_sampled(device, cfg):
    fm = _fm()
    c = W.WORKLOADS[cfg]()
    desc, E = c["desc"], c["E"][0]
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    x = W.rhs(c["seeds"][0] + 17, O.N)
    y = to_dev(np.zeros(O.N), device)
    P.apply_operator([E], to_dev(x, device), y)
    yg = y.cpu().numpy()
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, O.N, 1500), [0, O.N - 1],
                                     [O.offsets[a][0] for a in range(3)]]))
    ref = O.rows(E, rows) @ x
    err = np.abs(yg[rows] - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, err



def test_operator_parity_full_size_sampled_helium_J10(device):
    """The fourth J = 10 basis set of the paper's Table 3 (eleven M' blocks,
    unreduced: N = 3 682 404) on the kernels that take the blocks one at a
    time: sampled rows against the oracle's."""
    fm = _fm()
    g1, g3, _ = W.HE_TABLE3_J10[3]
    desc = W.helium_desc(g1, g3, dom1=W.HE_TABLE3_DOMAINS[0], dom3=W.HE_TABLE3_DOMAINS[1], J=10, tau=1)
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    assert P.N == O.N == 3682404
    E = -2.0045
    x = W.rhs(5, O.N)
    y = to_dev(np.zeros(O.N), device)
    P.apply_operator([E], to_dev(x, device), y)
    yg = y.cpu().numpy()
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, O.N, 600), [0, O.N - 1],
                                     [O.offsets[a][0] for a in range(3)]]))
    ref = O.rows(E, rows) @ x
    err = np.abs(yg[rows] - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, err


# sides of 32 m + 1: the last 32 x 32 tile also computes the leftover row (x)
# or column (y) of the x-y products
EXT_CASES = [("ext_x97_y13", wide(97, 13, 4, 3)), ("ext_x10_y97", wide(10, 97, 4, 3))]

PREC_CASES = [
    ("ps_cubic16", W.ps_cubic16()["desc"]),
    ("quintic_7x7x6", small(W.PS_MINUS, 7, 6)),
    ("hminus_quadratic_22x22x9", small(W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic")),
    ("L2_tau+1", small(W.PS_MINUS, 7, 4, J=2, tau=1, dz=3)),
    ("L5_tau+1", small(W.PS_MINUS, 7, 4, J=5, tau=1, dz=3)),
    # complex pairs in the x and in the y pencil of one slice: the 4 x 4 blocks
    ("x_and_y_pairs_43x19", W.pair_pair_desc()),
] + WIDE_CASES + EXT_CASES


@pytest.mark.parametrize("name,desc", PREC_CASES, ids=[c[0] for c in PREC_CASES])
def test_precond_parity(device, name, desc):
    fm = _fm()
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    rng = np.random.default_rng(5)
    Es = [-0.25, -0.45]
    R = rng.standard_normal((2, O.N))
    Z = to_dev(np.zeros((2, O.N)), device)
    P.apply_precond(Es, to_dev(R, device), Z)
    Zg = Z.cpu().numpy()
    for r, E in enumerate(Es):
        ref = precond_reference(O, E, R[r])
        err = np.abs(Zg[r] - ref).max() / np.abs(ref).max()
        assert err <= 1e-9, (name, r, err)


def test_precond_leftover_corner_backward_error(device):
    """x and y sides 97 = 3 x 32 + 1: the leftover row, column and corner of
    every x-y product.  An LU of the separable operator at this size takes
    half a minute per right-hand side, so the check is the normwise backward
    error of z against that operator, |L z - r| <= 1e-12 |L| |z| (max norms).
    On the oracle's own solve at x 97, y 13 it is 9e-21; zeroing one leftover
    row gives 9e-7 and scaling the corner by 1 + 1e-3 gives 5e-9."""
    fm = _fm()
    desc = wide(97, 97, 4, 3)
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    E = -0.25
    r = np.random.default_rng(11).standard_normal(O.N)
    z = to_dev(np.zeros(O.N), device)
    P.apply_precond([E], to_dev(r, device), z)
    zg = z.cpu().numpy()
    L = O.separable(E).tocsr()
    norm_L = np.abs(L).sum(axis=1).max()
    back = np.abs(L @ zg - r).max() / (norm_L * np.abs(zg).max())
    assert back <= 1e-12, back


def test_precond_equals_kronecker_inverse_without_potentials(device):
    """All charges zero: the separable block is the whole operator and the
    tensor trick must equal the dense inverse of the Kronecker sum."""
    fm = _fm()
    desc = small(((1.0, 1.0, 1.0), (0.0, 0.0, 0.0)), 10, 6, dxy=3, dz=3, R=10.0)
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    E = -0.3
    Ainv = np.linalg.inv(O.assemble(E).toarray())
    r = W.rhs(99, O.N)
    z = to_dev(np.zeros(O.N), device)
    P.apply_precond([E], to_dev(r, device), z)
    ref = Ainv @ r
    assert np.abs(z.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max() * 10


def test_solve_trivial_converges_in_one_step(device):
    fm = _fm()
    desc = small(((1.0, 1.0, 1.0), (0.0, 0.0, 0.0)), 10, 6, dxy=3, dz=3, R=10.0)
    P = fm.Problem(desc)
    b = to_dev(W.rhs(5, P.N), device)
    x = to_dev(np.zeros(P.N), device)
    st, res = P.solve([-0.3], b, x, restart=30, rtol=1e-10)
    assert st == fm.FM_OK
    assert res[0]["iters"] == 1
    assert res[0]["rel_residual"] <= 1e-12


def test_solve_ps_cubic16_matches_lu(device):
    fm = _fm()
    c = W.ps_cubic16()
    desc, E = c["desc"], c["E"][0]
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    b = W.rhs(c["seeds"][0], O.N)
    x = to_dev(np.zeros(O.N), device)
    st, res = P.solve([E], to_dev(b, device), x, restart=30, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    xg = x.cpu().numpy()
    A = O.assemble(E)
    assert rel_residual(A, xg, b) <= 1e-10
    xref = lu_solve(A, b, "dense")
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-8
    assert abs(res[0]["rel_residual"] - rel_residual(A, xg, b)) <= 1e-12


@pytest.mark.parametrize("nxy,nz", [(7, 9), (7, 8), (7, 30)])
def test_solve_odd_and_even_sizes_match_lu(device, nxy, nz):
    """N odd (quintic 7 x 7 x 9: 1323 unknowns) takes the Arnoldi passes one
    element at a time, N even (cubic z 8: 1176) their 16-byte paired loads;
    N = 4410 (quintic z 30) is even but its two dot-pass chunks of 2205 are
    not, so the dot pass reads single elements while the update pass reads
    pairs.  Two requests each, against the oracle's LU."""
    import torch
    fm = _fm()
    desc = W.make_desc(*W.PS_MINUS, nxy, nz, deg_z=5 if nz % 3 == 0 else 3, R=15.0)
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    assert O.N % 2 == (nz % 2) and (nz != 30 or O.N == 4410)
    Es = [-0.3, -0.17]
    B = np.stack([W.rhs(41, O.N), W.rhs(42, O.N)])
    X = torch.zeros(B.shape, dtype=torch.float64, device=device)
    st, res = P.solve(Es, to_dev(B, device), X, restart=40, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    Xg = X.cpu().numpy()
    for r, E in enumerate(Es):
        A = O.assemble(E)
        assert rel_residual(A, Xg[r], B[r]) <= 1e-10
        xref = lu_solve(A, B[r], "dense")
        assert np.linalg.norm(Xg[r] - xref) / np.linalg.norm(xref) <= 1e-8


def test_solve_batched_energies(device):
    fm = _fm()
    desc = small(W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic")
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    Es = [-0.6, -0.35, -0.1]
    B = np.stack([W.rhs(2001 + i, O.N) for i in range(3)])
    X = to_dev(np.zeros_like(B), device)
    st, res = P.solve(Es, to_dev(B, device), X, restart=250, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    Xg = X.cpu().numpy()
    for i, E in enumerate(Es):
        A = O.assemble(E)
        assert rel_residual(A, Xg[i], B[i]) <= 1e-10
        xref = lu_solve(A, B[i], "splu")
        assert np.linalg.norm(Xg[i] - xref) / np.linalg.norm(xref) <= 1e-8


def test_solve_cycle_longer_than_256_steps(device):
    """One FGMRES cycle of more than 256 steps: the cycle's back substitution
    gives each thread of its block several rows of R.  Just below the
    break-up threshold (E -> 0) the block-Jacobi preconditioned iteration on
    this grid needs about 260 steps, which restart = 1000 keeps in one cycle."""
    fm = _fm()
    desc = small(W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic")
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    E = -0.005
    b = W.rhs(2012, O.N)
    x = to_dev(np.zeros((1, O.N)), device)
    st, res = P.solve([E], to_dev(b[None, :], device), x, restart=1000, rtol=1e-10, max_iters=3000)
    assert st == fm.FM_OK, res
    assert res[0]["iters"] > 256, res
    A = O.assemble(E)
    xg = x.cpu().numpy()[0]
    assert rel_residual(A, xg, b) <= 1e-10
    xref = lu_solve(A, b, "splu")
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-7


def test_solve_identical_particle_symmetry(device):
    from tests.test_oracle_operator import permutation_maps
    fm = _fm()
    c = W.ps_cubic16()
    desc, E = c["desc"], c["E"][0]
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    (ci, cs), (ri, rs) = permutation_maps(O, (1, 2))
    b = W.rhs(77, O.N)
    bp = rs * b[ri]
    X = to_dev(np.zeros((2, O.N)), device)
    st, _ = P.solve([E, E], to_dev(np.stack([b, bp]), device), X, restart=30, rtol=1e-12, max_iters=3000)
    assert st == fm.FM_OK
    x, xp = X.cpu().numpy()
    assert np.abs(xp - cs * x[ci]).max() <= 1e-9 * np.abs(x).max()


def test_solve_rejects_nonfinite_rhs(device):
    fm = _fm()
    P = fm.Problem(W.ps_cubic16()["desc"])
    b = W.rhs(1, P.N)
    b[17] = np.nan
    x = to_dev(np.zeros(P.N), device)
    with pytest.raises(fm.FmError) as e:
        P.solve([-0.25], to_dev(b, device), x)
    assert e.value.status == fm.FM_E_NONFINITE


@pytest.mark.parametrize("name,desc", PREC_CASES, ids=[c[0] for c in PREC_CASES])
def test_precond_one_block_per_slice_and_staged_paths(device, name, desc):
    """Slices of side <= 32 run the x-y products with one block per slice,
    wider ones as batched GEMMs over all slices, whatever the batch: a batch
    of 512 slices or more and one of two requests must both match the
    oracle's separable inverse, and each other.  Slices whose sides are not
    multiples of 16 exercise the MFMA output rows that fall outside the slice
    (they must map back inside it)."""
    import torch
    fm = _fm()
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    slices = sum(O.nM * O.bz[a].n for a in range(3))
    nb_big = -(-512 // slices) + 1                      # one block per slice
    rng = np.random.default_rng(9)
    Es = list(np.linspace(-0.6, -0.1, nb_big))
    R = rng.standard_normal((nb_big, O.N))
    Zbig = to_dev(np.zeros((nb_big, O.N)), device)
    P.apply_precond(Es, to_dev(R, device), Zbig)
    Zsmall = to_dev(np.zeros((2, O.N)), device)
    P.apply_precond(Es[:2], to_dev(R[:2], device), Zsmall)
    Zb = Zbig.cpu().numpy()
    for r in (0, 1, nb_big - 1):
        ref = precond_reference(O, Es[r], R[r])
        err = np.abs(Zb[r] - ref).max() / np.abs(ref).max()
        assert err <= 1e-9, (name, r, err)
    d = (torch.linalg.norm(Zsmall - Zbig[:2]) / torch.linalg.norm(Zbig[:2])).item()
    assert d <= 1e-11, d


def test_precond_after_operator_grows_its_buffer(device):
    """fm_apply_operator growing its coupling buffer must leave the
    preconditioner's scratch alone (regression: growing it once freed the
    scratch as well, leaving the preconditioner a dangling buffer)."""
    fm = _fm()
    desc = PREC_CASES[1][1]
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    rng = np.random.default_rng(21)
    r = rng.standard_normal(O.N)
    z = to_dev(np.zeros((1, O.N)), device)
    P.apply_precond([-0.3], to_dev(r[None, :], device), z)
    X = to_dev(rng.standard_normal((3, O.N)), device)
    Y = to_dev(np.zeros((3, O.N)), device)
    P.apply_operator([-0.3] * 3, X, Y)
    z2 = to_dev(np.zeros((1, O.N)), device)
    P.apply_precond([-0.3], to_dev(r[None, :], device), z2)
    ref = precond_reference(O, -0.3, r)
    assert np.abs(z2.cpu().numpy()[0] - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("nxy,nb", [(16, 1), (16, 24), (34, 1)])
def test_solve_reports_the_smallest_denominator(device, nxy, nb):
    """min_abs_denominator of a solve is the smallest |lambda_x + lambda_y - E|
    over every slice of the preconditioner (eq. (prec-2)); on a cubic grid
    every pencil eigenvalue is real.  Side 16 runs the one-block-per-slice
    kernel (one request, and 24 requests), side 34 the staged x-y products
    (divide on the store of the right product).  The host side is the
    library's own slice eigenvalues (fm_host_slice_eigenvalues) with the same
    FP64 sum, so the two agree exactly."""
    import torch
    fm = _fm()
    desc = W.ps_cubic16()["desc"] if nxy == 16 else W.make_desc(*W.PS_MINUS, nxy, 8, deg_xy=3, deg_z=3, R=20.0)
    P = fm.Problem(desc)
    E = -0.3141
    want = np.inf
    for a in range(3):
        for slot in range(desc["z"][a]["n"]):
            lx, lxi, ly, lyi = fm.host_slice_eigenvalues(desc, a, slot)
            assert not lxi.any() and not lyi.any()
            want = min(want, np.abs((lx[:, None] + ly[None, :]) - E).min())
    b = torch.as_tensor(W.rhs_batch([31 + i for i in range(nb)], P.N), device=device)
    x = torch.zeros_like(b)
    st, res = P.solve([E] * nb, b, x, restart=30, rtol=1e-10, max_iters=400)
    assert st == fm.FM_OK
    for r in res:
        assert r["min_abs_denominator"] == want, (r["min_abs_denominator"], want)
