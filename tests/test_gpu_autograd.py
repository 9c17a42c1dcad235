"""Backward of the transforms = the hand-written adjoints (gradcheck and
dot-product identities through the C-ABI)."""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft
from paper_1808_00896_amd.autograd import soft_forward, soft_inverse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("B", [2, 4])
def test_gradcheck_inverse(dev, B):
    with soft.Plan(B) as p:
        c = torch.from_numpy(inputs.coeffs_uniform(B, 70 + B)).to(dev).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x: soft_inverse(x, p), (c,), eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("B", [2, 4])
def test_gradcheck_forward(dev, B):
    with soft.Plan(B) as p:
        g = torch.from_numpy(inputs.grid_random(B, 80 + B)).to(dev).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x: soft_forward(x, p), (g,), eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("B", [8, 32])
def test_adjoint_dot_products(dev, B):
    """<F g, c> = <g, F^H c> and <I c, g> = <c, I^H g> on the GPU path."""
    c = torch.from_numpy(inputs.coeffs_uniform(B, 90 + B)).to(dev)
    g = torch.from_numpy(inputs.grid_random(B, 95 + B)).to(dev)
    with soft.Plan(B) as p:
        lhs = torch.vdot(c, p.forward(g))
        rhs = torch.vdot(p.adjoint(c).reshape(-1), g.reshape(-1))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        lhs = torch.vdot(g.reshape(-1), p.inverse(c).reshape(-1))
        rhs = torch.vdot(p.adjoint_inverse(g), c)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_backward_through_linear_functional(dev):
    """d/dc Re<I c, G> = I^H G, checked against a central finite difference
    along a random direction at B = 16."""
    B = 16
    c0 = torch.from_numpy(inputs.coeffs_decay(B, 100)).to(dev)
    G = torch.from_numpy(inputs.grid_random(B, 101)).to(dev)
    d = torch.from_numpy(inputs.coeffs_uniform(B, 102)).to(dev)
    with soft.Plan(B) as p:
        c = c0.clone().requires_grad_(True)
        L = torch.real(torch.vdot(G.reshape(-1), soft_inverse(c, p).reshape(-1)))
        L.backward()
        h = 1e-4

        def Lf(x):
            return torch.real(torch.vdot(G.reshape(-1), p.inverse(x).reshape(-1))).item()
        fd = (Lf(c0 + h * d) - Lf(c0 - h * d)) / (2 * h)
        # d L along d = Re<grad, d> with PyTorch's conjugate-Wirtinger gradient
        an = torch.real(torch.vdot(c.grad, d)).item()
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))
