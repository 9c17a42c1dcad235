"""Plans made with SOFT_INPLACE_OK, through the C-ABI.
Such a plan holds no FFT intermediate of its own: the inverse stages it in
its output grid and the forward in its (overwritten) input grid, each gamma
block in the rows it reads.  The FFT passes do the same arithmetic in the
same order as with the plan-owned intermediate (only the addresses of the
intermediate differ), so every transform must equal a plan without the flag
bit for bit, at every FFT length and tile height (2B = 2 ... 1024, complex128
and complex64), and the oracle to the FP64 bar.
Inputs are seeded synthetic data from paper_1808_00896_amd.inputs.
"""

import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft
from paper_1808_00896_amd.autograd import correlation_grid, soft_forward, soft_inverse

pytestmark = pytest.mark.gpu

CDT = {"fp64": torch.complex128, "fp32": torch.complex64, "fp32_split": torch.complex64}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev, prec="fp64"):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev).to(CDT[prec])


def all_four(plan, c, g):
    """inverse, forward, adjoint and adjoint_inverse of (c, g); the grid
    inputs are copies, since an in-place plan overwrites them."""
    out = (plan.inverse(c), plan.forward(g.clone()), plan.adjoint(c), plan.adjoint_inverse(g.clone()))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64, 128])
def test_inplace_bit_identical(dev, prec, B):
    c = to_dev(inputs.coeffs_decay(B, 80 + B), dev, prec)
    g = to_dev(inputs.grid_random(B, 90 + B), dev, prec)
    with soft.Plan(B, precision=prec) as p0, soft.Plan(B, precision=prec, inplace_ok=True) as p1:
        want = all_four(p0, c, g)
        got = all_four(p1, c, g)
    for name, a, b in zip(("inverse", "forward", "adjoint", "adjoint_inverse"), want, got):
        assert torch.equal(a, b), f"{name}: max rel diff {float((a - b).abs().max() / b.abs().max()):.3e}"


def test_inplace_matches_oracle(oracle, dev):
    B = 16
    c = inputs.coeffs_uniform(B, 0)
    gr = inputs.grid_random(B, 1)
    with soft.Plan(B, inplace_ok=True) as p:
        g = p.inverse(to_dev(c, dev))
        gh = g.cpu().numpy()
        c2 = p.forward(g).cpu().numpy()  # overwrites g
        cr = p.forward(to_dev(gr, dev)).cpu().numpy()
    want = oracle.inverse(B, c)
    assert np.abs(gh - want).max() <= 1e-11 * np.abs(want).max()
    want_c = oracle.forward(B, gr)
    assert np.abs(cr - want_c).max() <= 1e-11 * np.abs(want_c).max()
    assert np.abs(c2 - c).max() <= 1e-11 * np.abs(c).max()


def test_inplace_batched_and_uneven(dev):
    B, n = 8, 3
    c = to_dev(np.stack([inputs.coeffs_decay(B, 100 + f) for f in range(n)]), dev)
    g = to_dev(np.stack([inputs.grid_random(B, 110 + f) for f in range(n)]), dev)
    with soft.Plan(B, n) as p0, soft.Plan(B, n, inplace_ok=True) as p1:
        for a, b in zip(all_four(p0, c, g), all_four(p1, c, g)):
            assert torch.equal(a, b)

    Bs = [4, 16, 8, 16, 64, 2]
    with soft.UnevenPlan(Bs) as u0, soft.UnevenPlan(Bs, inplace_ok=True) as u1:
        cs = np.concatenate([inputs.coeffs_decay(b, 120 + f) for f, b in enumerate(Bs)])
        gs = np.concatenate([inputs.grid_random(b, 130 + f).reshape(-1) for f, b in enumerate(Bs)])
        cu, gu = to_dev(cs, dev), to_dev(gs, dev)
        for a, b in zip(all_four(u0, cu, gu), all_four(u1, cu, gu)):
            assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inplace_workspace(dev, prec):
    B, n = 16, 2
    csize = 16 if prec == "fp64" else 8
    with soft.Plan(B, n, precision=prec) as p0, soft.Plan(B, n, precision=prec, inplace_ok=True) as p1:
        assert p0.workspace_bytes() - p1.workspace_bytes() == n * (2 * B) ** 3 * csize
        assert p1.describe()["inplace_ok"] is True
        assert p0.describe()["inplace_ok"] is False


@pytest.mark.parametrize("B,prec", [(256, "fp64"), (256, "fp32"), (512, "fp64")])
def test_inplace_large_bit_identical(dev, B, prec):
    """2B = 512 and 1024 (the largest tiles, two LDS exchanges at 1024):
    inverse and forward against a plan without the flag."""
    c = to_dev(inputs.coeffs_decay(B, 140 + B), dev, prec)
    with soft.Plan(B, precision=prec) as p0:
        g0 = p0.inverse(c)
        c0 = p0.forward(g0)
        torch.cuda.synchronize()
    torch.cuda.empty_cache()
    with soft.Plan(B, precision=prec, inplace_ok=True) as p1:
        g1 = p1.inverse(c)
        torch.cuda.synchronize()
        assert torch.equal(g0, g1)
        del g0
        c1 = p1.forward(g1)  # overwrites g1
        torch.cuda.synchronize()
        assert torch.equal(c0, c1)
    del g1, c0, c1
    torch.cuda.empty_cache()


def test_inplace_autograd_leaves_inputs(dev):
    """The autograd wrappers hand an in-place plan copies of the grids, so
    neither the caller's grid nor the incoming gradient is overwritten."""
    B = 4
    with soft.Plan(B, inplace_ok=True) as p:
        g = to_dev(inputs.grid_random(B, 150), dev).requires_grad_(True)
        g_before = g.detach().clone()
        y = soft_forward(g, p)
        torch.cuda.synchronize()
        assert torch.equal(g.detach(), g_before)
        c = to_dev(inputs.coeffs_decay(B, 151), dev).requires_grad_(True)
        G = to_dev(inputs.grid_random(B, 152), dev)
        G_before = G.clone()
        out = soft_inverse(c, p)
        out.backward(G)
        torch.cuda.synchronize()
        assert torch.equal(G, G_before)
        assert torch.autograd.gradcheck(lambda x: soft_inverse(x, p), (c.detach().requires_grad_(True),),
                                        eps=1e-6, atol=1e-8)
        assert torch.autograd.gradcheck(lambda x: soft_forward(x, p), (g.detach().requires_grad_(True),),
                                        eps=1e-6, atol=1e-8)
        del y


def test_inplace_match_plan(dev):
    B, n = 16, 4
    a, b = inputs.sh_pair_batch(n, B, seed=160)
    with soft.MatchPlan(B, n) as m0, soft.MatchPlan(B, n, inplace_ok=True) as m1:
        g0, i0 = m0.match(to_dev(a, dev), to_dev(b, dev))
        g1, i1 = m1.match(to_dev(a, dev), to_dev(b, dev))
        torch.cuda.synchronize()
        assert torch.equal(g0, g1) and torch.equal(i0, i1)
        assert m0.plan.workspace_bytes() - m1.plan.workspace_bytes() == n * (2 * B) ** 3 * 16
    a1, b1 = inputs.sh_pair_batch(1, 4, seed=161)
    with soft.MatchPlan(4, 1, inplace_ok=True) as m:
        at = to_dev(a1[0], dev).requires_grad_(True)
        bt = to_dev(b1[0], dev).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x, y: correlation_grid(x, y, m), (at, bt), eps=1e-6, atol=1e-8)
