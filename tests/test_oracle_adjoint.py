"""Pins of the oracle's loss and its hand-written gradient (CPU only).

The gradient is pinned by central finite differences of the loss (an
independent route to the same derivative) and by the dot-product identity
<J v, w> = <v, J^T w> between the hand JVP and the hand VJP."""
import numpy as np
import pytest

from oracle import cic
from oracle.model import Model, Problem
from paper_2604_26823_amd import inputs

_CACHE = {}


def setup(n=16, rsd="z", nm=None, steps=5, box=None, cone=False):
    key = (n, rsd, nm, steps, box, cone)
    if key in _CACHE:
        return _CACHE[key]
    cfg = inputs.config(2 if cone else 1, n_part=n, n_mesh=nm or n,
                        box=box or 8.0 * n, n_steps=steps, rsd=rsd)
    fields = {k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}
    R = inputs.response_field(cfg)
    fields["nbar"] = 2.0 if cone else 1.0
    mdl = Model(Problem(**fields))
    s_true = inputs.white_noise(n, 11)
    lam = mdl.observe(mdl.forward(s_true), R)
    N = inputs.poisson_counts(lam, R, mdl.p.r_min, 12)
    s0 = inputs.white_noise(n, 13)
    _CACHE[key] = (mdl, R, N, s0)
    return _CACHE[key]


@pytest.mark.parametrize("kw", [dict(rsd="z"), dict(rsd="radial", cone=True),
                                dict(rsd="radial", nm=32, cone=True)])
def test_gradient_central_finite_difference_16(kw):
    mdl, R, N, s0 = setup(**kw)
    L, g, _ = mdl.loss_and_grad(s0, N, R)
    v = np.random.default_rng(14).standard_normal(s0.shape)
    h = 1e-7
    fd = (mdl.loss(s0 + h * v, N, R) - mdl.loss(s0 - h * v, N, R)) / (2 * h)
    an = float(np.sum(g * v))
    assert abs(fd - an) <= 1e-6 * abs(an)


@pytest.mark.parametrize("kw", [dict(rsd="z"), dict(rsd="radial", cone=True),
                                dict(rsd="radial", nm=32, cone=True)])
def test_full_chain_dot_product(kw):
    mdl, R, N, s0 = setup(**kw)
    rng = np.random.default_rng(15)
    v = rng.standard_normal(s0.shape)
    w = rng.standard_normal(s0.shape)
    jv = mdl.jvp(s0, v)
    vj = mdl.vjp(s0, w)
    a, b = float(np.sum(jv * w)), float(np.sum(v * vj))
    assert abs(a - b) <= 1e-10 * abs(a)


def test_force_vjp_dot_product():
    mdl, R, N, s0 = setup()
    d0, _, _ = mdl.lpt(s0)
    d = d0 * 10.0
    rng = np.random.default_rng(16)
    td = rng.standard_normal(d.shape)
    v = rng.standard_normal(d.shape)
    x = mdl.q + d
    g = mdl.force_mesh(d)
    trho = cic.paint_jvp(x, td, mdl.p.n_mesh, mdl.dm) / mdl.nbar_mesh
    tg = [mdl.op("grad", trho, j, mesh=True) for j in range(3)]
    tF = np.stack([cic.readout_jvp(x, td, g[j], tg[j], mdl.dm) for j in range(3)])
    xbar = mdl.force_vjp(d, g, v)
    assert abs(np.sum(tF * v) - np.sum(td * xbar)) <= 1e-11 * abs(np.sum(tF * v))


def test_loss_special_cases():
    """Prior gradient is s itself; counts equal to the rate give chi^2 = 0."""
    mdl, R, N, s0 = setup()
    L, st = mdl.loss(s0, N, R, return_state=True)
    lam = st["lam"]
    L0, g0, st0 = mdl.loss_and_grad(s0, lam, R)
    assert st0["chi2"] == 0.0
    assert np.array_equal(g0, s0)
    assert L0 == 0.5 * np.sum(s0 * s0)
    seed = mdl.loss_seed(lam + 1.0, lam, R)
    m = R >= mdl.p.r_min
    assert np.allclose(seed[m], mdl.p.bias, rtol=1e-14, atol=0)
    assert np.all(seed[~m] == 0)
