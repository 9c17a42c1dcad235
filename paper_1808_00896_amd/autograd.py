"""torch.autograd Functions over the HIP transforms.

Both transforms are C-linear maps, so under PyTorch's conjugate-Wirtinger
convention the backward of y = A x is grad_x = A^H grad_y:
  SoftForward  (F, the quadrature of eq. "quadrature"):  backward = F^H = W I V
  SoftInverse  (I, eq. "fourier_representation"):        backward = I^H = V^-1 F W^-1
Both adjoints are entry points of the library (soft_adjoint,
soft_adjoint_inverse); nothing here computes on the host.  With an
``inplace_ok`` plan the forward-type calls overwrite their input grid, so
the grid handed to them here is a copy.

SoftCorrelation forms the correlation coefficients a(l,M) conj(b(l,M')) of
the rotational-matching head; its backward is the library's vector-Jacobian
product (soft_match_coeffs_vjp).
"""
import torch

from . import soft


def _scratch_copy(grid, plan):
    """The grid to hand to a forward-type call: a private copy when the plan
    may overwrite it."""
    return grid.clone(memory_format=torch.contiguous_format) if plan.inplace_ok else grid.contiguous()


class SoftForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, plan):
        ctx.plan = plan
        return plan.forward(_scratch_copy(grid, plan))

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
        return ctx.plan.adjoint_inverse(_scratch_copy(grad_grid, ctx.plan)), None


def soft_forward(grid, plan):
    """Differentiable FSOFT of `grid` with `plan` (a soft.Plan)."""
    return SoftForward.apply(grid, plan)


def soft_inverse(coeffs, plan):
    """Differentiable iFSOFT of `coeffs` with `plan` (a soft.Plan)."""
    return SoftInverse.apply(coeffs, plan)


class SoftCorrelation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, match):
        a, b = a.contiguous(), b.contiguous()
        ctx.match = match
        ctx.save_for_backward(a, b)
        return match.coeffs(a, b)

    @staticmethod
    def backward(ctx, grad_coeffs):
        a, b = ctx.saved_tensors
        ga, gb = ctx.match.coeffs_vjp(a, b, grad_coeffs.contiguous())
        return ga, gb, None


def correlation_coeffs(a, b, match):
    """Differentiable correlation coefficients of the pairs (a, b) (a soft.MatchPlan)."""
    return SoftCorrelation.apply(a, b, match)


def correlation_grid(a, b, match):
    """Differentiable correlation grids: inverse transform of the correlation
    coefficients with the match plan's own soft.Plan."""
    return soft_inverse(correlation_coeffs(a, b, match), match.plan)
