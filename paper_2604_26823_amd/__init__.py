"""MI355X (gfx950) implementation of the MUJICA reconstruction hot path.

The differentiable forward model (white noise -> BBKS linear field -> 2LPT ->
FastPM kick-drift-kick particle mesh -> redshift-space distortion -> linear
bias and survey response -> masked Gaussian chi^2 + white-noise prior), its
hand-written adjoint, the projection and rank-order matching of the white
noise and the projected L-BFGS step run in hand-written HIP kernels behind
the C ABI of include/ic_api.h.  ``Context`` (api.py) binds it to PyTorch
device memory and streams; ``autograd`` wraps the forward model and the loss
as torch.autograd.Functions (ICForward, ICLoss) whose backward passes are the
hand-written adjoint;
``inputs`` builds the seeded synthetic workloads.
"""
__all__ = ["Context", "ICForward", "ICLoss", "inputs", "build"]


def __getattr__(name):
    if name == "Context":
        from .api import Context
        return Context
    if name in ("ICForward", "ICLoss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
