"""The forward model and the loss as torch.autograd.Functions (GPU).

torch.autograd.grad through ICForward must give the oracle's vector-Jacobian
product, and through ICLoss the oracle's gradient, at c1 (32^3, 5 steps,
plane-parallel RSD, half-box mask) and on the radial 32^3 case, to the
tolerances of the end-to-end parity tests: gradient relative L2 <= 1e-4 in
FP32 and 1e-9 in FP64 against the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import (DEV, cfg_small, context, model, observation, rel_l2, require_gpu,
                        to_dev, to_np, torch)
from paper_2604_26823_amd import inputs
from paper_2604_26823_amd.autograd import ICForward, ICLoss

pytestmark = pytest.mark.gpu

TOL_DENS = {"f32": 1e-5, "f64": 1e-10}
TOL_GRAD = {"f32": 1e-4, "f64": 1e-9}
CASES = {"c1": dict(c=1),
         "radial32": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5, galaxies=2e4)}


def prepared(name, prec):
    kw = dict(CASES[name])
    cfg = dict(cfg_small(kw.pop("c"), **kw))
    cfg["nbar"] = inputs.nbar_for(cfg, inputs.response_field(cfg))
    mdl = model(cfg)
    R, N, s0 = observation(cfg, mdl)
    ctx = context(cfg, prec)
    ctx.set_observation(torch.tensor(N, dtype=torch.int32, device=DEV), to_dev(R, prec))
    return mdl, ctx, R, N, s0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_icforward_grad_is_the_oracle_vjp(prec, name):
    require_gpu()
    mdl, ctx, R, N, s0 = prepared(name, prec)
    w = np.random.default_rng(17).standard_normal(s0.shape).astype(np.float32).astype(np.float64)
    s = to_dev(s0, prec).requires_grad_(True)
    delta = ICForward.apply(s, ctx)
    assert delta.requires_grad
    _, st = mdl.loss(s0, N, R, return_state=True)
    e_d = rel_l2(to_np(delta), st["delta_s"])
    y = torch.sum(delta * to_dev(w, prec))
    (gs,) = torch.autograd.grad(y, s)
    ref = mdl.vjp(s0, w)
    e_g = rel_l2(to_np(gs), ref)
    print("%s %s: delta rel L2 %.3e, autograd J^T w rel L2 %.3e" % (name, prec, e_d, e_g))
    assert e_d <= TOL_DENS[prec]
    assert e_g <= TOL_GRAD[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_icloss_grad_is_the_oracle_gradient(prec, name):
    require_gpu()
    mdl, ctx, R, N, s0 = prepared(name, prec)
    L_ref, g_ref, _ = mdl.loss_and_grad(s0, N, R)
    s = to_dev(s0, prec).requires_grad_(True)
    L = ICLoss.apply(s, ctx)
    assert L.dim() == 0 and L.dtype == torch.float64
    (gs,) = torch.autograd.grad(L, s)
    e_L = abs(float(L.detach()) - L_ref) / abs(L_ref)
    e_g = rel_l2(to_np(gs), g_ref)
    print("%s %s: loss rel %.3e, autograd gradient rel L2 %.3e" % (name, prec, e_L, e_g))
    assert e_L <= TOL_DENS[prec]
    assert e_g <= TOL_GRAD[prec]
    # the incoming cotangent scales the stashed gradient (chain rule through
    # a torch expression of the loss)
    s2 = to_dev(s0, prec).requires_grad_(True)
    (g3,) = torch.autograd.grad(3.0 * ICLoss.apply(s2, ctx) + 1.0, s2)
    assert rel_l2(to_np(g3), 3.0 * g_ref) <= TOL_GRAD[prec]
