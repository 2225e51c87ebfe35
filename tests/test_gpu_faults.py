"""Failure paths through the C ABI (GPU).  Every failure here is detected on
the host, or by a check of the library before the work it would spoil:
non-finite white noise, a line search that cannot decrease the loss (forced
with a step far below the rounding of s), planted extremes that the
projection resets, and argument errors.  After each error the context keeps
working and gives the same result as before."""
import ctypes

import numpy as np
import pytest

from gpu_common import DEV, cfg_small, rel_l2, require_gpu, to_dev, to_np, torch
from paper_2604_26823_amd import _lib, inputs
from paper_2604_26823_amd.api import Context

pytestmark = pytest.mark.gpu

NONFINITE, LINESEARCH, INVALID = -5, -6, -1


def _setup(prec, **kw):
    cfg = cfg_small(1, **kw)
    ctx = Context(cfg, prec, DEV)
    R = inputs.response_field(cfg)
    N = inputs.poisson_counts(np.ones(R.shape), R, cfg["r_min"], 17)
    ctx.set_observation(torch.tensor(N, dtype=torch.int32, device=DEV), to_dev(R, prec))
    s = to_dev(inputs.white_noise(cfg["n_part"], 18), prec)
    ctx.project_rankmatch(s, _lib.IC_PROJECT, event=0)
    return ctx, s


def _code(fn):
    with pytest.raises(_lib.IcError) as e:
        fn()
    return e.value.code


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_non_finite_white_noise_is_refused(prec, bad):
    require_gpu()
    ctx, s = _setup(prec)
    try:
        L0, g0, _ = ctx.loss_and_grad(s)
        g0 = to_np(g0)
        sb = s.clone()
        sb[3, 4, 5] = bad
        assert _code(lambda: ctx.forward(sb, delta=True, loss=True)) == NONFINITE
        assert _code(lambda: ctx.loss_and_grad(sb)) == NONFINITE
        assert _code(lambda: ctx.vjp(sb, s)) == NONFINITE
        assert _code(lambda: ctx.lbfgs_step(sb, to_dev(g0, prec), L0, 0)) == NONFINITE
        assert _code(lambda: ctx.project_rankmatch(sb, _lib.IC_ROM_REAL, event=1)) == NONFINITE
        # the context still works and gives the same loss and gradient
        L1, g1, _ = ctx.loss_and_grad(s)
        assert abs(L1 - L0) <= 1e-6 * abs(L0)
        assert rel_l2(to_np(g1), g0) <= 1e-5
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_line_search_exhaustion_leaves_the_state_unchanged(prec):
    """One trial of a step 1e-30 long changes no element of s, so the loss
    cannot decrease: both the quasi-Newton and the steepest-descent search
    fail, and s, the gradient and the loss come back untouched."""
    require_gpu()
    ctx, s = _setup(prec, max_trials=1, eps_max=1e-30, project_steps=0)
    try:
        L, g, _ = ctx.loss_and_grad(s)
        s0, g0 = s.clone(), g.clone()
        assert _code(lambda: ctx.lbfgs_step(s, g, L, 0)) == LINESEARCH
        assert torch.equal(s, s0) and torch.equal(g, g0)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_planted_extremes_are_reset(prec):
    require_gpu()
    ctx, s = _setup(prec)
    try:
        x = s.clone().reshape(-1)
        where = torch.arange(10, device=DEV) * 997
        x[where] = torch.tensor([50.0, -50.0] * 5, dtype=x.dtype, device=DEV)
        x = x.reshape(s.shape)
        info = ctx.project_rankmatch(x, _lib.IC_PROJECT, event=3)
        out = to_np(x)
        assert info["resets"] >= 10
        assert np.max(np.abs(out)) <= 10.0
        assert abs(out.mean()) < 1e-6 and abs(out.std() - 1.0) < 1e-6
        # the planted values were replaced, the others only z-scored
        assert np.all(np.abs(out.reshape(-1)[to_np(where).astype(int)]) < 10.0)
    finally:
        ctx.close()


def test_argument_errors_through_the_abi():
    require_gpu()
    ctx, s = _setup("f32")
    lib, c = ctx.lib, ctx.ctx
    try:
        L0 = ctx.loss_and_grad(s)[0]
        g = ctx.empty(*ctx.grid)
        P = ctypes.c_void_p
        assert lib.ic_forward(c, None, None, None, None) == INVALID
        assert lib.ic_loss_and_grad(c, P(s.data_ptr()), None, None, None) == INVALID
        assert lib.ic_vjp(c, P(s.data_ptr()), None, P(g.data_ptr())) == INVALID
        assert lib.ic_lbfgs_step(c, P(s.data_ptr()), P(g.data_ptr()), None, 0, None) == INVALID
        assert lib.ic_set_observation(c, None, None) == INVALID
        assert lib.ic_op_rfft(c, 7, P(s.data_ptr()), P(g.data_ptr())) == INVALID
        assert lib.ic_op_sort_desc(c, P(s.data_ptr()), ctx.n ** 3 + 1, P(g.data_ptr())) == INVALID
        assert lib.ic_op_multiplier(c, 2, 3, 0, P(s.data_ptr()), P(g.data_ptr())) == INVALID
        assert lib.ic_loss_and_grad(None, P(s.data_ptr()), P(g.data_ptr()), None, None) == INVALID
        assert lib.ic_last_error(c)
        # still working
        assert abs(ctx.loss_and_grad(s)[0] - L0) <= 1e-6 * abs(L0)
    finally:
        ctx.close()
