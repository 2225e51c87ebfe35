"""The forward model and the loss as torch.autograd.Functions.

Section 2.2 of the paper describes the forward model as differentiable: the
reconstruction needs the gradient of the loss with respect to the white
noise.  Both functions here route every step through the HIP library of
include/ic_api.h; their backward passes are the hand-written adjoint kernel
chain (CIC readout transposed to paint and back, FFT adjoints, the reversed
kick-drift-kick with the force Jacobian, the 2LPT and whitening adjoints),
not PyTorch's autograd of any PyTorch operation.

* ``ICForward.apply(s, ctx)`` -> delta_s, the redshift-space density
  contrast on the data grid (``ic_forward``); backward: s_bar = J^T delta_bar
  (``ic_vjp``, no prior term).
* ``ICLoss.apply(s, ctx)`` -> L(s) = 1/2 chi^2 + 1/2 w |s|^2 as a 0-dim
  float64 tensor (``ic_loss_and_grad``, which also leaves the gradient);
  backward: that gradient times the incoming scalar cotangent.

``ctx`` is an ``api.Context``; s must be a contiguous tensor of its dtype on
its device with the shape of its particle grid.  Neither function supports
double backward.
"""
import torch

__all__ = ["ICForward", "ICLoss", "forward", "loss"]


class ICForward(torch.autograd.Function):
    """delta_s = forward model(s); backward through ic_vjp."""

    @staticmethod
    def forward(fctx, s, context):
        delta = context.forward(s, delta=True)["delta"]
        fctx.save_for_backward(s)
        fctx.context = context
        return delta

    @staticmethod
    def backward(fctx, delta_bar):
        (s,) = fctx.saved_tensors
        context = fctx.context
        return context.vjp(s, delta_bar.to(context.dtype).contiguous()), None


class ICLoss(torch.autograd.Function):
    """L(s) with its gradient from the same evaluation."""

    @staticmethod
    def forward(fctx, s, context):
        L, g, _ = context.loss_and_grad(s)
        fctx.save_for_backward(g)
        return torch.tensor(L, dtype=torch.float64, device=s.device)

    @staticmethod
    def backward(fctx, L_bar):
        (g,) = fctx.saved_tensors
        # the chain rule's scaling by the incoming scalar (1 for a plain
        # .backward() of the loss itself)
        return g * L_bar.to(g.dtype), None


def forward(s, context):
    """delta_s with autograd through the hand-written adjoint."""
    return ICForward.apply(s, context)


def loss(s, context):
    """L(s) with autograd through the hand-written adjoint."""
    return ICLoss.apply(s, context)
