"""The GLRM loss as a differentiable torch function.

``glrm_loss(X, Y, data)`` is sum_{(i,j) in Omega} L_j(x_i . y_j, A_ij), the loss
part of eq. gpca.  Its backward is the hand-written gradient kernel behind
``glrm_grad`` (Section 7.2: dF/dx_i = sum_j dL(x_i . y_j, A_ij) y_j and the
transposed form for y_j), the same kernel family that drives the fit.  When
gradients are needed the forward pass already runs that kernel once, returning
the value and keeping both gradients for the backward pass.
"""
import torch

from . import glrm_grad, glrm_objective

__all__ = ["GLRMLoss", "glrm_loss"]


class GLRMLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, Y, data, precision):
        loss_data = data if (data.rx[0] == 0 and data.ry[0] == 0) else data.with_regs((0, 0.0), (0, 0.0))
        Xc, Yc = X.detach().contiguous(), Y.detach().contiguous()
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            dX, dY, val = glrm_grad(loss_data, Xc, Yc, precision, want_objective=True)
            ctx.save_for_backward(dX, dY)
        else:
            val = glrm_objective(loss_data, Xc, Yc, precision)
        return torch.tensor(val, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, g):
        dX, dY = ctx.saved_tensors
        if torch.is_tensor(g) and g.numel() == 1 and float(g) == 1.0:
            return dX, dY, None, None
        s = g.to(dX.dtype)
        return dX * s, dY * s, None, None


def glrm_loss(X, Y, data, precision="fp32"):
    """Differentiable loss part of the GLRM objective (float64 scalar)."""
    return GLRMLoss.apply(X, Y, data, precision)
