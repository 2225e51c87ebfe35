"""Pins of the oracle's lightcone (CPU only): the comoving distance against the
Einstein-de Sitter closed form and adaptive quadrature, its inversion, the
static and single-snapshot limits, the crossing scale factor of straight
trajectories against a root solve, and the hand VJP against finite
differences (the operator alone and the whole loss)."""
import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import lightcone as lc
from oracle.cosmology import hubble_E
from oracle.model import Model, Problem
from paper_2604_26823_amd import inputs

OM = 0.315


def test_comoving_distance_closed_form_and_quadrature():
    a = np.array([0.3, 0.5, 0.8, 0.9, 0.999, 1.0])
    # Einstein-de Sitter: chi = 2 c/H0 (1 - sqrt(a))
    eds = 2.0 * lc.C_OVER_H0 * (1.0 - np.sqrt(a))
    assert np.allclose(lc.comoving_distance(a, 1.0), eds, rtol=1e-13, atol=1e-10)
    for ai in a:
        ref = lc.C_OVER_H0 * integrate.quad(lambda x: 1.0 / (x * x * hubble_E(x, OM)), ai, 1.0,
                                            epsabs=1e-12, epsrel=1e-12)[0]
        assert abs(lc.comoving_distance(ai, OM) - ref) <= 1e-10 * max(ref, 1.0)
    # low redshift: chi ~ c/H0 z
    assert abs(lc.comoving_distance(0.999, OM) / (lc.C_OVER_H0 * (1 / 0.999 - 1)) - 1) < 1e-3


def test_scale_factor_inverts_the_distance_and_clamps():
    d = np.array([0.0, 1.0, 150.0, 400.0, 600.0, 700.0, 5000.0])
    a = lc.scale_factor_at(d, OM, 0.8)
    chi_lo = lc.comoving_distance(0.8, OM)
    for di, ai in zip(d, a):
        if di >= chi_lo:
            assert ai == 0.8
        elif di == 0.0:
            assert ai == 1.0
        else:
            assert abs(lc.comoving_distance(ai, OM) - di) <= 1e-9 * di
    assert np.all(np.diff(a) <= 0)


def _geometry(n=8, box=500.0):
    j = np.arange(n) * (box / n)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()]), box


def test_static_snapshots_reduce_to_the_distance_of_each_particle():
    q, box = _geometry()
    obs = (19.0, 19.0, 19.0)
    rng = np.random.default_rng(0)
    d = rng.normal(0, 3, q.shape)
    p = rng.normal(0, 50, q.shape)
    L = lc.Lightcone(q, box, obs, OM, [0.8, 0.9, 1.0])
    ds, st = L.forward([(d, p)] * 3, "radial")
    x = q + d
    y = x - box * np.floor(x / box)
    u = y - np.asarray(obs)[:, None]
    r = np.sqrt((u * u).sum(0))
    a_ref = lc.scale_factor_at(r, OM, 0.8)
    assert np.array_equal(st["a"][-1], a_ref)
    c = 1.0 / (a_ref ** 2 * hubble_E(a_ref, OM))
    uh = u / r
    assert np.allclose(ds, d + c * (p * uh).sum(0) * uh, rtol=1e-14, atol=1e-12)


def test_straight_trajectories_cross_where_a_root_solve_says():
    q, box = _geometry(6)
    obs = np.array([19.0, 19.0, 19.0])
    rng = np.random.default_rng(1)
    x1 = rng.normal(0, 4, q.shape)          # displacement at a = 1
    v = rng.normal(0, 30, q.shape)          # d x / d a
    a_s = [0.8, 0.9, 1.0]
    snaps = [(x1 + v * (a - 1.0), np.zeros_like(x1)) for a in a_s]
    L = lc.Lightcone(q, box, obs, OM, a_s, iterations=3)
    a3 = L.scale_factors(snaps)[-1]
    a6 = lc.Lightcone(q, box, obs, OM, a_s, iterations=6).scale_factors(snaps)[-1]
    chi_lo = lc.comoving_distance(0.8, OM)
    # the fixed-point map contracts by kappa = max |da/dchi| |dx/da| per iteration
    kappa = hubble_E(1.0, OM) / lc.C_OVER_H0 * np.linalg.norm(v, axis=0)

    def chi(a):
        return lc.C_OVER_H0 * integrate.quad(lambda t: 1.0 / (t * t * hubble_E(t, OM)), a, 1.0,
                                             epsabs=1e-13, epsrel=1e-13)[0]
    checked = 0
    for i in range(q.shape[1]):
        def dist(a):
            x = q[:, i] + x1[:, i] + v[:, i] * (a - 1.0)
            y = x - box * np.floor(x / box)
            return np.linalg.norm(y - obs)
        f = lambda a: chi(a) - dist(a)
        ends = [q[:, i] + x1[:, i] + v[:, i] * (a - 1.0) for a in (0.8, 1.0)]
        if np.any(np.floor(ends[0] / box) != np.floor(ends[1] / box)):
            continue   # crosses a box face: the wrapped distance jumps
        if f(0.8) <= 0 or f(1.0) >= 0 or dist(0.8) >= chi_lo:
            continue   # outside the snapshot range
        try:
            a_star = optimize.brentq(f, 0.8, 1.0, xtol=1e-14)
        except ValueError:
            continue
        assert abs(a3[i] - a_star) <= 0.2 * kappa[i] ** 3 + 1e-12, (i, a3[i], a_star)
        assert abs(a6[i] - a_star) <= 0.2 * kappa[i] ** 6 + 1e-12, (i, a6[i], a_star)
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("rsd", ["radial", "z"])
def test_lightcone_vjp_against_finite_differences(rsd):
    q, box = _geometry(8)
    obs = (19.0, 19.0, 19.0)
    rng = np.random.default_rng(2)
    a_s = [0.8, 0.9, 1.0]
    base = rng.normal(0, 4, q.shape)
    snaps = [(base + rng.normal(0, 1.5, q.shape), rng.normal(0, 40, q.shape)) for _ in a_s]
    L = lc.Lightcone(q, box, obs, OM, a_s)
    ds, st = L.forward(snaps, rsd)
    w = rng.normal(size=ds.shape)
    db, pb = L.vjp(snaps, rsd, st, w)
    tang = [(rng.normal(size=q.shape), rng.normal(size=q.shape)) for _ in a_s]
    h = 1e-5
    plus = [(d + h * td, p + h * tp) for (d, p), (td, tp) in zip(snaps, tang)]
    minus = [(d - h * td, p - h * tp) for (d, p), (td, tp) in zip(snaps, tang)]
    fd = np.sum(w * (L.forward(plus, rsd)[0] - L.forward(minus, rsd)[0])) / (2 * h)
    ad = sum(np.sum(b1 * t1) + np.sum(b2 * t2) for b1, b2, (t1, t2) in zip(db, pb, tang))
    assert abs(fd - ad) <= 1e-7 * abs(ad)


def _small(lightcone, **kw):
    cfg = inputs.config(6, n_part=16, n_mesh=16, n_steps=6, galaxies=4e3, **kw)
    R = inputs.response_field(cfg)
    cfg["nbar"] = inputs.nbar_for(cfg, R)
    fields = {k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}
    fields["lightcone"] = lightcone
    return Model(Problem(**fields)), R, cfg


def test_single_snapshot_is_the_static_model():
    m0, R, cfg = _small(())
    m1, _, _ = _small((1.0,))
    s = inputs.white_noise(16, 5)
    assert np.allclose(m1.forward(s), m0.forward(s), rtol=0, atol=1e-12)


def test_loss_gradient_with_lightcone_against_finite_differences():
    # 6 steps from 0.1 to 1: snapshots at the steps a = 0.7 and 0.85
    m, R, cfg = _small((0.7, 0.85, 1.0))
    assert m.snap_steps == [4, 5]
    s = inputs.white_noise(16, 6)
    lam = m.observe(m.forward(inputs.white_noise(16, 7)), R)
    N = inputs.poisson_counts(lam, R, cfg["r_min"], 8)
    L, g, st = m.loss_and_grad(s, N, R)
    # the lightcone moves particles: the density differs from the static model's
    m0, _, _ = _small(())
    assert np.abs(st["delta_s"] - m0.forward(s)).max() > 1e-3
    a_i = st["lc"]["a"][-1]
    assert a_i.min() >= 0.7 and a_i.max() <= 1.0 and np.any((a_i > 0.7) & (a_i < 0.85))
    v = np.random.default_rng(9).standard_normal(s.shape)
    h = 1e-6
    fd = (m.loss(s + h * v, N, R) - m.loss(s - h * v, N, R)) / (2 * h)
    assert abs(fd - np.sum(g * v)) <= 1e-5 * abs(fd)
