"""Pins of the oracle's CIC, particle-mesh force, 2LPT, KDK and RSD (CPU only)."""
import itertools
import math

import numpy as np
import pytest

from oracle import cic, fourier
from oracle.model import Model, Problem

_MODELS = {}


def model(**kw):
    key = tuple(sorted(kw.items()))
    if key not in _MODELS:
        _MODELS[key] = Model(Problem(**kw))
    return _MODELS[key]


# ----------------------------------------------------------------------- CIC
def brute_paint(pos, n, cell):
    """Pure-Python CIC straight from W(x - c) = prod (1 - |u - c|)_+ ."""
    rho = np.zeros((n, n, n))
    for p in range(pos.shape[1]):
        u = pos[:, p] / cell
        base = [math.floor(v) for v in u]
        for off in itertools.product((0, 1), repeat=3):
            c = [base[a] + off[a] for a in range(3)]
            w = 1.0
            for a in range(3):
                w *= max(0.0, 1.0 - abs(u[a] - c[a]))
            rho[c[0] % n, c[1] % n, c[2] % n] += w
    return rho


def test_paint_matches_brute_force():
    rng = np.random.default_rng(4)
    pos = rng.uniform(-20, 60, size=(3, 40))
    assert np.max(np.abs(cic.paint(pos, 6, 7.0) - brute_paint(pos, 6, 7.0))) <= 1e-13


def test_paint_mass_conservation_and_lattice():
    rng = np.random.default_rng(5)
    n = 16
    pos = rng.uniform(-100, 100, size=(3, n ** 3))
    assert abs(cic.paint(pos, n, 3.0).sum() - n ** 3) <= 1e-9
    j = np.arange(n) * 3.0
    q = np.stack([a.ravel() for a in np.meshgrid(j, j, j, indexing="ij")])
    assert np.max(np.abs(cic.paint(q, n, 3.0) - 1.0)) <= 1e-14


def test_readout_constant_and_transpose():
    rng = np.random.default_rng(6)
    n = 8
    pos = rng.uniform(-10, 30, size=(3, 100))
    assert np.max(np.abs(cic.readout(pos, np.full((n, n, n), 2.5), 2.0) - 2.5)) <= 1e-14
    w = rng.standard_normal(100)
    m = rng.standard_normal((n, n, n))
    lhs = np.sum(cic.paint(pos, n, 2.0, weight=w) * m)
    rhs = np.sum(w * cic.readout(pos, m, 2.0))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_readout_gradient_finite_difference():
    rng = np.random.default_rng(7)
    n = 8
    pos = rng.uniform(0.1, 1.9, size=(3, 30)) + 2.0 * rng.integers(0, n, size=(3, 30))
    m = rng.standard_normal((n, n, n))
    g = cic.readout_gradient(pos, m, 2.0)
    h = 1e-6
    for a in range(3):
        dp = np.zeros_like(pos)
        dp[a] = h
        fd = (cic.readout(pos + dp, m, 2.0) - cic.readout(pos - dp, m, 2.0)) / (2 * h)
        assert np.max(np.abs(fd - g[a])) <= 1e-8


# -------------------------------------------------------------------- force
def _particles_force(mdl, pos):
    """PM force on arbitrary particle positions (q = 0 convention)."""
    n = mdl.p.n_mesh
    rho = cic.paint(pos, n, mdl.dm)
    delta = rho / mdl.nbar_mesh - 1.0
    g = [fourier.apply(mdl.mult("grad", j, True), delta) for j in range(3)]
    return np.stack([cic.readout(pos, g[j], mdl.dm) for j in range(3)])


def test_self_force_vanishes_and_pair_antisymmetry():
    mdl = model(n_part=8, n_mesh=8, box=64.0, n_steps=2)
    rng = np.random.default_rng(8)
    one = rng.uniform(0, 64, size=(3, 1))
    f1 = _particles_force(mdl, one)
    two = np.concatenate([one, rng.uniform(0, 64, size=(3, 1))], axis=1)
    f2 = _particles_force(mdl, two)
    scale = np.max(np.abs(f2))
    assert np.max(np.abs(f1)) <= 1e-12 * scale
    assert np.max(np.abs(f2[:, 0] + f2[:, 1])) <= 1e-12 * scale
    many = rng.uniform(0, 64, size=(3, 50))
    fm = _particles_force(mdl, many)
    assert np.max(np.abs(fm.sum(axis=1))) <= 1e-12 * np.sum(np.abs(fm))


@pytest.mark.parametrize("nm", [8, 16])
def test_unperturbed_lattice_feels_no_force(nm):
    mdl = model(n_part=8, n_mesh=nm, box=64.0, n_steps=2)
    F, _ = mdl.force(np.zeros((3, 8 ** 3)))
    assert np.max(np.abs(F)) <= 1e-13


# --------------------------------------------------------------------- 2LPT
def test_2lpt_orthogonal_waves():
    n, L = 32, 256.0
    mdl = model(n_part=n, n_mesh=n, box=L, n_steps=2)
    A, B = 0.3, 0.2
    k1, k2 = 2 * np.pi * 2 / L, 2 * np.pi * 3 / L
    x = np.arange(n) * L / n
    X, Y, _ = np.meshgrid(x, x, x, indexing="ij")
    dl = A * np.cos(k1 * X) + B * np.cos(k2 * Y)
    _, _, f = mdl.lpt_from_linear(dl)
    psi1 = [-A * np.sin(k1 * X) / k1, -B * np.sin(k2 * Y) / k2, 0 * X]
    c = A * B / (k1 ** 2 + k2 ** 2)
    psi2 = [c * k1 * np.sin(k1 * X) * np.cos(k2 * Y), c * k2 * np.cos(k1 * X) * np.sin(k2 * Y), 0 * X]
    for j in range(3):
        assert np.max(np.abs(f["psi1"][j] - psi1[j].ravel())) <= 1e-12
        assert np.max(np.abs(f["psi2"][j] - psi2[j].ravel())) <= 1e-12
    # a single plane wave has no second-order displacement
    _, _, f = mdl.lpt_from_linear(A * np.cos(k1 * X))
    assert np.max(np.abs(f["psi2"])) <= 1e-13


# ---------------------------------------------------------------------- KDK
def zeldovich_error(n, L=256.0, A=0.1, steps=5):
    mdl = model(n_part=n, n_mesh=n, box=L, n_steps=steps, rsd="z")
    k1 = 2 * np.pi / L
    x = np.arange(n) * L / n
    X, _, _ = np.meshgrid(x, x, x, indexing="ij")
    w = mdl.mult("white")[1, 0, 0].real
    s = A / w * np.cos(k1 * X)
    d0, p0, f = mdl.lpt(s)
    _, pS, tape_d, _ = mdl.evolve(d0, p0)
    psi = -A * np.sin(k1 * X).ravel() / k1
    errs = []
    co = mdl.coef
    from oracle.cosmology import second_order_growth
    grow = second_order_growth(list(co["a"]), 0.3)
    for a, d in zip(co["a"], tape_d):
        errs.append(np.max(np.abs(d[0] - grow[float(a)]["D1"] * psi)))
        assert np.max(np.abs(d[1:])) <= 1e-12
    return max(errs), A / k1, pS, tape_d[-1], grow[1.0]["f1"]


def test_zeldovich_plane_wave_converges_first_order():
    """A plane wave before shell crossing moves exactly as the Zel'dovich
    solution (the FastPM factors carry the growing mode exactly); the only
    error left is the mesh's.  With particles sitting on mesh nodes the CIC
    density of a small displacement is a one-sided difference (half-cell
    offset), so the error is first order in the cell size: below k dq times
    the displacement amplitude and halving with the cell."""
    e32, amp, _, _, _ = zeldovich_error(32)
    e64, _, _, _, _ = zeldovich_error(64)
    kdq = 2 * np.pi / 256.0 * 8.0
    assert e32 <= kdq * amp
    assert 1.8 <= e32 / e64 <= 2.2


def test_rsd_axis_shift_is_growth_rate_times_displacement():
    """In the Zel'dovich limit the momentum at a = 1 is f1 D1 Psi, so the
    plane-parallel redshift-space shift equals f1(1) times the displacement
    along the line of sight (Kaiser)."""
    from oracle.cosmology import G_factor, second_order_growth
    mdl = model(n_part=16, n_mesh=16, box=128.0, n_steps=3, rsd="z")
    psi = np.random.default_rng(12).standard_normal((3, 16 ** 3))
    g = second_order_growth([1.0], 0.3)[1.0]
    d = g["D1"] * psi
    p = G_factor(1.0, 0.3, g["D1"], g["f1"]) * psi
    ds = mdl.rsd(d, p)
    assert np.max(np.abs(ds[2] - d[2] - g["f1"] * d[2])) <= 1e-12
    assert np.array_equal(ds[:2], d[:2])


def test_kdk_time_reversibility():
    mdl = model(n_part=16, n_mesh=16, box=128.0, n_steps=4, rsd="z")
    s = np.random.default_rng(9).standard_normal((16, 16, 16))
    d0, p0, _ = mdl.lpt(s)
    d, p, _, _ = mdl.evolve(d0, p0)
    kc = mdl.kick_coefficients()
    Dr = mdl.coef["Dr"]
    for n in range(mdl.p.n_steps - 1, -1, -1):
        p = p - kc[n + 1] * mdl.force(d)[0]
        d = d - Dr[n] * p
    p = p - kc[0] * mdl.force(d)[0]
    assert np.max(np.abs(d - d0)) <= 1e-11 * np.max(np.abs(d0))
    assert np.max(np.abs(p - p0)) <= 1e-11 * np.max(np.abs(p0))


def test_translation_equivariance():
    """Rolling the white noise by whole cells rolls the data-grid density."""
    mdl = model(n_part=16, n_mesh=16, box=128.0, n_steps=3, rsd="z")
    s = np.random.default_rng(10).standard_normal((16, 16, 16))
    a = mdl.forward(s)
    b = mdl.forward(np.roll(s, (3, -2, 5), axis=(0, 1, 2)))
    assert np.max(np.abs(np.roll(a, (3, -2, 5), axis=(0, 1, 2)) - b)) <= 1e-12


def test_radial_rsd_jacobian_finite_difference():
    mdl = model(n_part=8, n_mesh=8, box=64.0, n_steps=2, rsd="radial",
                observer=(-5.0, 3.0, 70.0))
    rng = np.random.default_rng(11)
    d = rng.normal(0, 2.0, size=(3, 512))
    p = rng.normal(0, 5.0, size=(3, 512))
    xb = rng.standard_normal((3, 512))
    d_bar, p_bar = mdl.rsd_vjp(d, p, xb)
    h = 1e-6
    for a in range(3):
        e = np.zeros_like(d)
        e[a] = h
        fd_d = (mdl.rsd(d + e, p) - mdl.rsd(d - e, p)) / (2 * h)
        fd_p = (mdl.rsd(d, p + e) - mdl.rsd(d, p - e)) / (2 * h)
        assert np.max(np.abs(np.sum(fd_d * xb, axis=0) - d_bar[a])) <= 1e-8
        assert np.max(np.abs(np.sum(fd_p * xb, axis=0) - p_bar[a])) <= 1e-8
