"""Pins of the oracle's Poisson observation model (CPU only): the paper's
galaxy bias, lambda = Nbar R (1 + delta)^alpha sigmoid(K (delta - delta_th))
(section 2.2.1, item 4), and the Poisson log-likelihood over the mask
(section 2.2.2), as loss 1/2 D with D = -2 log L.

Pinned by a library routine (scipy's Poisson log-pmf), closed forms of the
bias at the threshold and far above it, central finite differences of the
per-cell data term and of the whole loss, and the stationary point
lambda = N of each cell's term."""
import numpy as np
import pytest
from scipy import stats

from oracle.model import Model, Problem
from paper_2604_26823_amd import inputs

_CACHE = {}


def setup(n=16, rsd="z", cone=False):
    key = (n, rsd, cone)
    if key in _CACHE:
        return _CACHE[key]
    cfg = inputs.config(2 if cone else 1, n_part=n, n_mesh=n, box=8.0 * n, n_steps=5, rsd=rsd)
    fields = {k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}
    fields.update(loss="poisson", nbar=3.0, prior_weight=0.0)
    R = inputs.response_field(cfg)
    mdl = Model(Problem(**fields))
    lam = mdl.observe(mdl.forward(inputs.white_noise(n, 21)), R)
    N = inputs.poisson_counts(lam, R, mdl.p.r_min, 22)
    s0 = inputs.white_noise(n, 23)
    _CACHE[key] = (mdl, R, N, s0)
    return _CACHE[key]


def test_bias_closed_forms():
    mdl, R, N, s0 = setup()
    p = mdl.p
    r = np.array([1.0, 0.5, 0.25])
    # at the threshold the sigmoid is 1/2
    d = np.full(3, p.bias_delta_th)
    assert np.allclose(mdl.observe(d, r), p.nbar * r * (1 + d) ** p.bias_alpha / 2, rtol=1e-14)
    # far above it the sigmoid is 1 to double precision: the plain power law
    d = np.array([30.0, 50.0, 80.0])
    assert np.allclose(mdl.observe(d, r), p.nbar * r * (1 + d) ** p.bias_alpha, rtol=1e-14)
    # the paper's parameters
    assert (p.bias_alpha, p.bias_delta_th, p.bias_k) == (0.7, 1.2, 3.0)


def test_data_term_is_minus_two_poisson_log_likelihood():
    mdl, R, N, s0 = setup(cone=True, rsd="radial")
    L, st = mdl.loss(s0, N, R, return_state=True)
    m = R >= mdl.p.r_min
    ref = -2.0 * np.sum(stats.poisson.logpmf(N[m], st["lam"][m]))
    assert abs(st["chi2"] - ref) <= 1e-12 * abs(ref)
    assert L == 0.5 * st["chi2"]   # prior weight 0: the likelihood-only objective


def test_seed_matches_finite_differences_and_vanishes_at_lambda_equal_n():
    mdl, R, N, s0 = setup()
    rng = np.random.default_rng(24)
    shape = R.shape
    delta = rng.uniform(-0.9, 4.0, shape)
    counts = rng.poisson(2.0, shape).astype(np.int32)
    lam = mdl.observe(delta, R)
    seed = mdl.loss_seed(lam, counts, R, delta)
    m = R >= mdl.p.r_min

    def half_d(dl):
        return 0.5 * mdl.chi2(mdl.observe(dl, R), counts, R)

    idx = np.argwhere(m)[rng.choice(int(m.sum()), 12, replace=False)]
    for c in map(tuple, idx):
        h = 1e-6
        up, dn = delta.copy(), delta.copy()
        up[c] += h
        dn[c] -= h
        fd = (half_d(up) - half_d(dn)) / (2 * h)
        assert abs(fd - seed[c]) <= 1e-6 * max(1.0, abs(seed[c])), (c, fd, seed[c])
    assert np.all(seed[~m] == 0)
    # lambda = N in every masked cell is the stationary point of each term
    lam_c = np.where(m, lam, 0.0)
    seed0 = mdl.loss_seed(lam, np.where(m, lam, 0.0), R, delta)
    assert np.max(np.abs(seed0[m])) <= 1e-12 * np.max(lam_c)


@pytest.mark.parametrize("kw", [dict(rsd="z"), dict(rsd="radial", cone=True)])
def test_poisson_gradient_central_finite_difference_16(kw):
    mdl, R, N, s0 = setup(**kw)
    L, g, _ = mdl.loss_and_grad(s0, N, R)
    v = np.random.default_rng(25).standard_normal(s0.shape)
    h = 1e-6
    fd = (mdl.loss(s0 + h * v, N, R) - mdl.loss(s0 - h * v, N, R)) / (2 * h)
    an = float(np.sum(g * v))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
