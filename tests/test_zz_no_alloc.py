"""The allocation-free operator entry point (fm_apply_operator_noalloc)
against fm_apply_operator, through the C ABI.

Two calls in a row share the library's static scratch: the first on a larger
problem and batch, the second on a smaller problem whose coupling slots lie
where the first call left nonzero values (so a slot left uncleared would show
in its output).  Outputs are compared elementwise, relative to the largest
output, at 1e-11 (the operator's parity tolerance: the same kernels run on the
same data).  A batch whose coupling slots exceed the scratch is rejected
before any device work."""
import numpy as np
import pytest

from paper_2005_05398_amd import workloads as W

pytestmark = pytest.mark.gpu


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


def _compare(P, Es, X, device):
    import torch
    y_ref = torch.zeros(X.shape, dtype=torch.float64, device=device)
    y_new = torch.full(X.shape, np.nan, dtype=torch.float64, device=device)
    xd = to_dev(X, device)
    P.apply_operator(Es, xd, y_ref)
    P.apply_operator_noalloc(Es, xd, y_new)
    a, b = y_ref.cpu().numpy(), y_new.cpu().numpy()
    assert np.all(np.isfinite(b))
    return float(np.abs(a - b).max() / np.abs(a).max())


def test_noalloc_operator_matches_apply_operator_twice(device):
    from paper_2005_05398_amd import fm
    rng = np.random.default_rng(8)
    big = fm.Problem(W.make_desc(*W.H_MINUS, 22, 9, R=40.0, xy_map="quadratic"))
    Es = [-0.55, -0.3, -0.12]
    assert _compare(big, Es, rng.standard_normal((3, big.N)), device) <= 1e-11
    small = fm.Problem(W.make_desc(*W.PS_MINUS, 7, 6, R=15.0))
    assert small.N < big.N
    assert _compare(small, [-0.25], rng.standard_normal((1, small.N)), device) <= 1e-11
    # and the larger one again, after the smaller call
    assert _compare(big, Es[:2], rng.standard_normal((2, big.N)), device) <= 1e-11


def test_noalloc_operator_rejects_batches_beyond_its_scratch(device):
    import torch
    from paper_2005_05398_amd import fm
    P = fm.Problem(W.hminus_scan()["desc"])
    cap = ((8 << 20) - 4096) // (2 * P.N)          # requests whose two slots fit
    x = torch.zeros((cap + 1) * P.N, dtype=torch.float64, device=device)
    y = torch.zeros_like(x)
    with pytest.raises(fm.FmError) as e:
        P.apply_operator_noalloc([-0.3] * (cap + 1), x, y)
    assert e.value.status == fm.FM_E_INVALID
    rng = np.random.default_rng(2)
    Es = list(np.linspace(-0.6, -0.1, cap))
    assert _compare(P, Es, rng.standard_normal((cap, P.N)), device) <= 1e-11


def test_noalloc_operator_many_blocks(device):
    """Six M' blocks (the operator kernels that take the blocks one at a time),
    then a one-block problem, then the six-block one again with a smaller batch."""
    from paper_2005_05398_amd import fm
    rng = np.random.default_rng(9)
    many = fm.Problem(W.make_desc(*W.PS_MINUS, 7, 4, J=5, tau=1, deg_z=3, R=15.0))
    Es = [-0.4, -0.2, 0.1]
    assert _compare(many, Es, rng.standard_normal((3, many.N)), device) <= 1e-11
    one = fm.Problem(W.make_desc(*W.PS_MINUS, 7, 6, R=15.0))
    assert _compare(one, [-0.25], rng.standard_normal((1, one.N)), device) <= 1e-11
    assert _compare(many, Es[:1], rng.standard_normal((1, many.N)), device) <= 1e-11
