"""torch.autograd Functions over the HIP transforms.

Both transforms are C-linear maps, so under PyTorch's conjugate-Wirtinger
convention the backward of y = A x is grad_x = A^H grad_y:
  SoftForward  (F, the quadrature of eq. "quadrature"):  backward = F^H = W I V
  SoftInverse  (I, eq. "fourier_representation"):        backward = I^H = V^-1 F W^-1
Both adjoints are entry points of the library (soft_adjoint,
soft_adjoint_inverse); nothing here computes on the host.
"""
import torch

from . import soft


class SoftForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, plan):
        ctx.plan = plan
        return plan.forward(grid.contiguous())

    @staticmethod
    def backward(ctx, grad_coeffs):
        return ctx.plan.adjoint(grad_coeffs.contiguous()), None


class SoftInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, plan):
        ctx.plan = plan
        return plan.inverse(coeffs.contiguous())

    @staticmethod
    def backward(ctx, grad_grid):
        return ctx.plan.adjoint_inverse(grad_grid.contiguous()), None


def soft_forward(grid, plan):
    """Differentiable FSOFT of `grid` with `plan` (a soft.Plan)."""
    return SoftForward.apply(grid, plan)


def soft_inverse(coeffs, plan):
    """Differentiable iFSOFT of `coeffs` with `plan` (a soft.Plan)."""
    return SoftInverse.apply(coeffs, plan)
