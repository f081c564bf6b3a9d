"""The GLRM objective as differentiable torch functions.

``glrm_loss(X, Y, data)`` is sum_{(i,j) in Omega} L_j(x_i . y_j, A_ij), the loss
part of eq. gpca; ``glrm_objective(X, Y, data)`` is all of eq. gpca, the loss
plus sum_i r(x_i) + sum_j rt(y_j) (Section 3).  Their backward is the
hand-written gradient kernel behind ``glrm_grad`` (Section 7.2: dF/dx_i =
sum_j dL(x_i . y_j, A_ij) y_j and the transposed form for y_j), the same kernel
family that drives the fit; for the objective the library adds, coordinate by
coordinate, the regularizers' subgradient of least magnitude (quadratic 2 w x;
l1 w sign(x), 0 at 0; nonnegative 0; NaN outside their domain).  When gradients
are needed the forward pass already runs that kernel once, returning the value
and keeping both gradients for the backward pass.
"""
import torch

from . import GRAD_WITH_REG, glrm_grad, glrm_objective as _objective

__all__ = ["GLRMLoss", "GLRMObjective", "glrm_loss", "glrm_objective"]


def _forward(ctx, X, Y, data, precision, with_reg):
    if not with_reg and not (data.rx[0] == 0 and data.ry[0] == 0):
        data = data.with_regs((0, 0.0), (0, 0.0))
    Xc, Yc = X.detach().contiguous(), Y.detach().contiguous()
    if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
        dX, dY, val = glrm_grad(data, Xc, Yc, precision, want_objective=True,
                                flags=GRAD_WITH_REG if with_reg else 0)
        ctx.save_for_backward(dX, dY)
    else:
        val = _objective(data, Xc, Yc, precision)
    return torch.tensor(val, dtype=torch.float64, device=X.device)


def _backward(ctx, g):
    dX, dY = ctx.saved_tensors
    if torch.is_tensor(g) and g.numel() == 1 and float(g) == 1.0:
        return dX, dY, None, None
    s = g.to(dX.dtype)
    return dX * s, dY * s, None, None


class GLRMLoss(torch.autograd.Function):
    """The loss part of eq. gpca."""

    @staticmethod
    def forward(ctx, X, Y, data, precision):
        return _forward(ctx, X, Y, data, precision, False)

    @staticmethod
    def backward(ctx, g):
        return _backward(ctx, g)


class GLRMObjective(torch.autograd.Function):
    """All of eq. gpca: the loss and both regularizer sums."""

    @staticmethod
    def forward(ctx, X, Y, data, precision):
        return _forward(ctx, X, Y, data, precision, True)

    @staticmethod
    def backward(ctx, g):
        return _backward(ctx, g)


def glrm_loss(X, Y, data, precision="fp32"):
    """Differentiable loss part of the GLRM objective (float64 scalar)."""
    return GLRMLoss.apply(X, Y, data, precision)


def glrm_objective(X, Y, data, precision="fp32"):
    """Differentiable GLRM objective F(X, Y) of eq. gpca (float64 scalar)."""
    return GLRMObjective.apply(X, Y, data, precision)
