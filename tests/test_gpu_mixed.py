"""Reduced-precision preconditioner products inside the FP64 flexible GMRES.

The FP32-MFMA and BF16x3-MFMA preconditioners must agree with the FP64 one to
their arithmetic's accuracy (FP32: unit roundoff 6e-8 times the conditioning of
the eigenvector products, bounded here by 1e-4; BF16x3 with three products:
about 2^-16 per product, bounded by 1e-3), and the mixed-precision solves must
meet the same FP64 bar as the FP64 path: true relative residual 1e-10 against
the oracle's matrix and relative solution error 1e-8 against the oracle's LU.
"""
import numpy as np
import pytest

from oracle.assemble import Problem as OracleProblem
from oracle.solve import lu_solve, rel_residual
from paper_2005_05398_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fm():
    from paper_2005_05398_amd import fm
    return fm


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


def wide(nx, ny, nz):
    """Quintic x and y of different sizes, cubic z."""
    d = W.make_desc(*W.PS_MINUS, nx, nz, deg_xy=5, deg_z=3, R=20.0)
    d["y"] = W.make_desc(*W.PS_MINUS, ny, nz, deg_xy=5, deg_z=3, R=20.0)["y"]
    return d


# the 97-wide cases (97 = 3 x 32 + 1): the leftover row, column and corner of
# the staged products
CASES = [("ps_cubic16", W.ps_cubic16()["desc"]),
         ("hminus_22x22x9", W.make_desc(*W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic")),
         ("L2_quintic7_cubic4", W.make_desc(*W.PS_MINUS, 7, 4, J=2, deg_z=3, R=15.0)),
         ("ext_x97_y13", wide(97, 13, 4)), ("ext_x10_y97", wide(10, 97, 4)), ("ext_97x97", wide(97, 97, 4)),
         ("x_and_y_pairs_43x19", W.pair_pair_desc()),
         ("L5_quintic7_cubic4", W.make_desc(*W.PS_MINUS, 7, 4, J=5, deg_z=3, R=15.0))]


@pytest.mark.parametrize("name,desc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16x3", 1e-3)])
def test_precond_reduced_precision(device, name, desc, prec, tol):
    import torch
    fm = _fm()
    P = fm.Problem(desc)
    r = to_dev(np.stack([W.rhs(11, P.N), W.rhs(12, P.N)]), device)
    z64 = torch.zeros_like(r)
    zlp = torch.zeros_like(r)
    Es = [-0.25, -0.5]
    P.apply_precond(Es, r, z64, prec="fp64")
    P.apply_precond(Es, r, zlp, prec=prec)
    for i in range(2):
        err = (torch.linalg.norm(zlp[i] - z64[i]) / torch.linalg.norm(z64[i])).item()
        assert err <= tol, (name, prec, err)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name,desc,E,restart", [
    ("ps_cubic16", W.ps_cubic16()["desc"], -0.25, 30),
    ("hminus_22x22x9", W.make_desc(*W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic"), -0.35, 250)])
def test_solve_mixed_precision(device, prec, name, desc, E, restart):
    fm = _fm()
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    b = W.rhs(1001, O.N)
    x = to_dev(np.zeros(O.N), device)
    st, res = P.solve([E], to_dev(b, device), x, restart=restart, rtol=1e-10, max_iters=4000, prec=prec)
    assert st == fm.FM_OK, res
    A = O.assemble(E)
    xg = x.cpu().numpy()
    assert rel_residual(A, xg, b) <= 1e-10
    xref = lu_solve(A, b)
    assert np.linalg.norm(xg - xref) / np.linalg.norm(xref) <= 1e-8


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_long_cycle_reduced_precision_full_size(device, prec):
    """Full-size H- scan energies that take 100+ Arnoldi steps in one cycle of
    300: the newest Krylov direction is rescaled every step, so its size must
    not drift out of the reduced-precision range over the cycle.  Reduced- and
    full-precision solutions agree to the solve's accuracy."""
    import torch
    fm = _fm()
    cfg = W.hminus_scan()
    P = fm.Problem(cfg["desc"])
    Es = [float(e) for e in np.asarray(cfg["E"])[-4:]]
    B = to_dev(np.stack([W.rhs(s, P.N) for s in cfg["seeds"][-4:]]), device)
    x64 = torch.zeros_like(B)
    xlp = torch.zeros_like(B)
    st, res = P.solve(Es, B, x64, restart=300, rtol=1e-10, max_iters=3000, prec="fp64")
    assert st == fm.FM_OK, res
    st, res_lp = P.solve(Es, B, xlp, restart=300, rtol=1e-10, max_iters=3000, prec=prec)
    assert st == fm.FM_OK, res_lp
    assert max(r["iters"] for r in res_lp) >= 100
    for i in range(4):
        assert res_lp[i]["rel_residual"] <= 1e-10
        err = (torch.linalg.norm(xlp[i] - x64[i]) / torch.linalg.norm(x64[i])).item()
        assert err <= 1e-8, (prec, i, err)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16x3", 1e-3)])
@pytest.mark.parametrize("precond", ["block_jacobi", "coupled"])
def test_precond_reduced_precision_wide_batch(device, prec, tol, precond):
    """A batch large enough for the 64 x 64 block tiles of the staged products
    (the energy scan's grid, 16 requests; L = 1 for the coupled variant, whose
    joint z products stay FP64 around the FP32 x-y products)."""
    import torch
    fm = _fm()
    desc = W.hminus_scan()["desc"]
    if precond == "coupled":
        desc = dict(W.make_desc(*W.H_MINUS, 64, 24, J=1, deg_z=5, R=40.0, xy_map="quadratic"), precond="coupled")
    P = fm.Problem(desc)
    nb = 16
    r = to_dev(W.rhs_batch([50 + i for i in range(nb)], P.N), device)
    z64 = torch.zeros_like(r)
    zlp = torch.zeros_like(r)
    Es = list(np.linspace(-0.6, -0.1, nb))
    P.apply_precond(Es, r, z64, prec="fp64")
    P.apply_precond(Es, r, zlp, prec=prec)
    err = (torch.linalg.norm(zlp - z64, dim=1) / torch.linalg.norm(z64, dim=1)).max().item()
    assert err <= tol, (prec, precond, err)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16x3", 1e-3)])
def test_precond_reduced_precision_many_small_slices(device, prec, tol):
    """A batch of 512 slices or more of side 16 (23 requests of the cubic
    16 x 16 x 8 grid, 552 slices): one block per slice for both reduced
    precisions (BF16x3 takes its staged chain only below 512 slices), each
    request against the FP64 preconditioner at its precision's bound."""
    import torch
    fm = _fm()
    desc = W.ps_cubic16()["desc"]
    P = fm.Problem(desc)
    nb = -(-512 // (3 * desc["z"][0]["n"])) + 1
    r = to_dev(W.rhs_batch([70 + i for i in range(nb)], P.N), device)
    z64 = torch.zeros_like(r)
    zlp = torch.zeros_like(r)
    Es = list(np.linspace(-0.6, -0.1, nb))
    P.apply_precond(Es, r, z64, prec="fp64")
    P.apply_precond(Es, r, zlp, prec=prec)
    err = (torch.linalg.norm(zlp - z64, dim=1) / torch.linalg.norm(z64, dim=1)).max().item()
    assert err <= tol, (prec, nb, err)
