"""The benchmark's own path under the oracle, through the C ABI.

* Operator batches wider than one coupling block: the coupling kernel takes
  16 requests per block row, so requests 16-31 and 32-34 of a 35-request
  batch run in its second and third row, and a 12-request batch leaves most
  of one row empty.  Every request is compared elementwise with the oracle's
  assembled matrix (small grids; all spline-order variants of the kernel, and
  the kernel for more than three M' blocks).
* Sampled rows of every request of a 34-request batch at the energy scan's
  full size (the bench's kernel variants: quintic 64 x 64 x 24).
* The 32-energy scan itself, solved as the bench solves it (one batch,
  restart 300, rtol 1e-10): the oracle's residual-only mode (rows of H and of
  A(1) assembled a chunk at a time, no factorisation) gives the true relative
  residual of requests from both coupling block rows, and it must meet 1e-10;
  the same at complex energies E_k + 0.01 i, and for the single large request
  (ps_q127) solved with each precision of the preconditioner products.
Tolerances: operator outputs elementwise relative to the largest, 1e-11 (FP64
sums of a few hundred terms); residuals 1e-10 (the metric's target) and the
GPU's own FP64 residual within 1e-12 of the oracle's.
"""
import sys

import numpy as np
import pytest

from oracle.assemble import Problem as OracleProblem
from oracle.solve import rel_residuals_by_rows, rel_residuals_by_rows_complex
from paper_2005_05398_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fm():
    from paper_2005_05398_amd import fm
    return fm


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


BATCH_CASES = [
    ("quintic_7x7x6", W.make_desc(*W.PS_MINUS, 7, 6, R=15.0)),
    ("hminus_13x13x9_quadratic", W.make_desc(*W.H_MINUS, 13, 9, R=30.0, xy_map="quadratic")),
    # the other spline orders of the one-block coupling kernel
    ("quintic_xy_cubic_z_10x8", W.make_desc(*W.PS_MINUS, 10, 8, deg_z=3, R=15.0)),
    ("cubic_xy_quintic_z_10x6", W.make_desc(*W.PS_MINUS, 10, 6, deg_xy=3, R=15.0)),
    ("cubic_10x6", W.make_desc(*W.PS_MINUS, 10, 6, deg_xy=3, deg_z=3, R=15.0)),
    ("L2_quintic_cubicz", W.make_desc(*W.PS_MINUS, 7, 4, J=2, tau=1, deg_z=3, R=15.0)),
    # six M' blocks: the coupling kernel that takes the blocks one at a time
    ("L5_quintic_cubicz", W.make_desc(*W.PS_MINUS, 7, 4, J=5, tau=1, deg_z=3, R=15.0)),
]


@pytest.mark.parametrize("nb", [35, 12])
@pytest.mark.parametrize("name,desc", BATCH_CASES, ids=[c[0] for c in BATCH_CASES])
def test_operator_parity_many_requests(device, name, desc, nb):
    fm = _fm()
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    rng = np.random.default_rng(21)
    Es = list(np.linspace(-0.6, 0.1, nb))
    X = rng.standard_normal((nb, O.N))
    Y = to_dev(np.zeros((nb, O.N)), device)
    P.apply_operator(Es, to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    H = O.assemble(0.0)
    S = H - O.assemble(1.0)
    for r, E in enumerate(Es):
        ref = H @ X[r] - E * (S @ X[r])
        err = np.abs(Yg[r] - ref).max() / np.abs(ref).max()
        assert err <= 1e-11, (name, r, err)


def test_operator_parity_full_size_34_requests_sampled(device):
    fm = _fm()
    c = W.hminus_scan()
    desc = c["desc"]
    Es = list(c["E"]) + [-0.35, -0.05]
    nb = len(Es)
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    X = W.rhs_batch([c["seeds"][0] + 100 + i for i in range(nb)], O.N)
    Y = to_dev(np.zeros((nb, O.N)), device)
    P.apply_operator(Es, to_dev(X, device), Y)
    Yg = Y.cpu().numpy()
    rng = np.random.default_rng(4)
    rows = np.unique(np.concatenate([rng.integers(0, O.N, 600), [0, O.N - 1],
                                     [O.offsets[a][0] for a in range(3)]]))
    H = O.rows(0.0, rows)
    S = H - O.rows(1.0, rows)
    for r in (0, 15, 16, 17, 30, 31, 32, 33):
        ref = H @ X[r] - Es[r] * (S @ X[r])
        err = np.abs(Yg[r, rows] - ref).max() / np.abs(ref).max()
        assert err <= 1e-11, (r, err)


def test_hminus_scan_batch_oracle_residual(device):
    """The bench's 32-energy scan: oracle residuals of requests 3, 16 and 31."""
    import torch
    fm = _fm()
    c = W.hminus_scan()
    desc, Es, seeds = c["desc"], c["E"], c["seeds"]
    P = fm.Problem(desc)
    B = W.rhs_batch(seeds, P.N)
    X = torch.zeros(B.shape, dtype=torch.float64, device=device)
    st, res = P.solve(Es, to_dev(B, device), X, restart=300, rtol=1e-10, max_iters=20000)
    assert st == fm.FM_OK, res
    Xg = X.cpu().numpy()
    pick = [3, 16, 31]
    O = OracleProblem(desc)

    def progress(done, total):
        print(f"oracle residual rows {done}/{total}", file=sys.stderr, flush=True)

    rel = rel_residuals_by_rows(O, [Es[i] for i in pick], Xg[pick], B[pick], progress=progress)
    for k, i in enumerate(pick):
        assert rel[k] <= 1e-10, (i, rel[k], res[i])
        assert abs(rel[k] - res[i]["rel_residual"]) <= 1e-12, (i, rel[k], res[i])


def test_hminus_scan_complex_oracle_residual(device):
    """The bench's scan at complex energies E_k + 0.01 i (complex seeded
    right-hand sides, two real rows per request): the oracle's complex
    residual-only mode gives the true relative residual of requests 3 and 31
    (the coupling kernel's first and second block rows), which must meet 1e-10
    and equal the GPU's own FP64 residual."""
    import torch
    fm = _fm()
    c = W.hminus_scan()
    desc, seeds = c["desc"], c["seeds"]
    Es = [complex(e, 0.01) for e in c["E"]]
    P = fm.Problem(desc)
    B = np.stack([np.concatenate([W.rhs(s, P.N), W.rhs(s + 500, P.N)]) for s in seeds])
    X = torch.zeros(B.shape, dtype=torch.float64, device=device)
    st, res = P.solve_complex(Es, to_dev(B, device), X, restart=300, rtol=1e-10, max_iters=20000)
    assert st == fm.FM_OK, res
    Xg = X.cpu().numpy()
    pick = [3, 31]
    O = OracleProblem(desc)

    def progress(done, total):
        print(f"oracle complex residual rows {done}/{total}", file=sys.stderr, flush=True)

    rel = rel_residuals_by_rows_complex(O, [Es[i] for i in pick], Xg[pick], B[pick], progress=progress)
    for k, i in enumerate(pick):
        assert rel[k] <= 1e-10, (i, rel[k], res[i])
        assert abs(rel[k] - res[i]["rel_residual"]) <= 1e-12, (i, rel[k], res[i])


def test_ps_q127_solves_oracle_residual_every_precision(device):
    """The single large request (quintic 127 x 127 x cubic 32, N = 1 548 288)
    solved as the bench solves it with FP64, FP32 and BF16x3 preconditioner
    products: the oracle's residual-only mode gives each solution's true
    relative residual, which must meet 1e-10 and equal the GPU's own."""
    import torch
    fm = _fm()
    c = W.ps_q127()
    desc, E = c["desc"], c["E"][0]
    P = fm.Problem(desc)
    b = W.rhs(c["seeds"][0], P.N)
    precs = ("fp64", "fp32", "bf16x3")
    X, res = [], []
    for prec in precs:
        x = torch.zeros((1, P.N), dtype=torch.float64, device=device)
        st, r = P.solve([E], to_dev(b[None, :], device), x, restart=60, rtol=1e-10, max_iters=2000, prec=prec)
        assert st == fm.FM_OK, (prec, r)
        X.append(x.cpu().numpy()[0])
        res.append(r[0])
    O = OracleProblem(desc)

    def progress(done, total):
        print(f"oracle residual rows {done}/{total}", file=sys.stderr, flush=True)

    rel = rel_residuals_by_rows(O, [E] * 3, np.stack(X), np.stack([b] * 3), chunk=65536, progress=progress)
    for k, prec in enumerate(precs):
        assert rel[k] <= 1e-10, (prec, rel[k], res[k])
        assert abs(rel[k] - res[k]["rel_residual"]) <= 1e-12, (prec, rel[k], res[k])


@pytest.mark.parametrize("precond", ["block_jacobi", "coupled"])
def test_ps_l2_q97_solutions_sampled_residual(device, precond):
    """The L = 2 request at full size (three M' blocks, N = 2 709 792; too large
    for the oracle's whole residual in a test) solved as the bench solves it
    with FP64 and FP32 products: at 3000 sampled rows (and the ends of every
    block) each residual component |b_i - (A x)_i| is at most the whole
    residual's bound 1e-10 ||b||, by the oracle's rows."""
    import torch
    fm = _fm()
    c = W.ps_l2_q97()
    desc, E = c["desc"], c["E"][0]
    P = fm.Problem(dict(desc, precond=precond))
    b = W.rhs(c["seeds"][0], P.N)
    O = OracleProblem(desc)
    assert O.N == P.N
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([rng.integers(0, O.N, 3000)] +
                                    [[o, o + O.block[a] - 1] for a in range(3) for o in O.offsets[a]]))
    A = O.rows(E, rows)
    nb = np.linalg.norm(b)
    for prec in ("fp64", "fp32"):
        x = torch.zeros((1, P.N), dtype=torch.float64, device=device)
        st, r = P.solve([E], to_dev(b[None, :], device), x, restart=60, rtol=1e-10, max_iters=2000, prec=prec)
        assert st == fm.FM_OK, (prec, r)
        res = b[rows] - A @ x.cpu().numpy()[0]
        assert np.abs(res).max() <= 1e-10 * nb, (prec, np.abs(res).max() / nb, r)


def test_batched_solve_masks_running_requests(device):
    """Nine energies that converge at different steps: the operator kernels
    skip the requests that have finished, and every solution meets the
    oracle's LU."""
    import torch
    from oracle.solve import lu_solve, rel_residual
    fm = _fm()
    desc = W.make_desc(*W.H_MINUS, 13, 9, R=30.0, xy_map="quadratic")
    P = fm.Problem(desc)
    O = OracleProblem(desc)
    Es = [-0.9, -0.8, -0.7, -0.62, -0.58, -0.48, -0.45, -0.4, -0.35]
    B = W.rhs_batch([5100 + i for i in range(len(Es))], O.N)
    X = torch.zeros(B.shape, dtype=torch.float64, device=device)
    st, res = P.solve(Es, to_dev(B, device), X, restart=100, rtol=1e-10, max_iters=4000)
    assert st == fm.FM_OK, res
    its = [r["iters"] for r in res]
    assert len(set(its)) > 2, its
    Xg = X.cpu().numpy()
    for i, E in enumerate(Es):
        A = O.assemble(E)
        assert rel_residual(A, Xg[i], B[i]) <= 1e-10, (i, res[i])
        xref = lu_solve(A, B[i])
        assert np.linalg.norm(Xg[i] - xref) / np.linalg.norm(xref) <= 1e-8, i
