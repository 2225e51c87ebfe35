"""Pins of the oracle's Fourier conventions and cosmology (CPU only).

Each check ties the oracle to something other than itself: a brute-force DFT,
closed forms of single Fourier modes, the Einstein-de Sitter solutions, an
independent quadrature, or a published fitting formula."""
import math

import numpy as np
import pytest

from oracle import cosmology as C
from oracle import fourier as F


def brute_rdft(x):
    """O(N^6) half-spectrum DFT straight from the definition."""
    n = x.shape[0]
    j = np.arange(n)
    out = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n // 2 + 1):
                ph = np.exp(-2j * np.pi * (kx * j[:, None, None] + ky * j[None, :, None]
                                           + kz * j[None, None, :]) / n)
                out[kx, ky, kz] = np.sum(x * ph)
    return out


def test_rfft_matches_brute_force_dft_8():
    x = np.random.default_rng(1).standard_normal((8, 8, 8))
    ref = brute_rdft(x)
    got = F.rfft3(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_dft_modes_match_brute_force_and_full_transform():
    x = np.random.default_rng(11).standard_normal((8, 8, 8))
    modes = [(0, 0, 0), (7, 1, 4), (4, 4, 4), (3, 6, 2), (1, 0, 1)]
    ref = brute_rdft(x)
    got = F.dft_modes(x.astype(np.float32), modes, rows=5)
    x32 = F.rfft3(x.astype(np.float32))
    for m, g in zip(modes, got):
        assert abs(g - x32[m]) <= 1e-12 * np.max(np.abs(x32))
    got = F.dft_modes(x, modes)
    for m, g in zip(modes, got):
        assert abs(g - ref[m]) <= 1e-13 * np.max(np.abs(ref))


def test_parseval_and_roundtrip():
    x = np.random.default_rng(2).standard_normal((16, 16, 16))
    xk = F.rfft3(x)
    wgt = np.full(xk.shape, 2.0)
    wgt[..., 0] = 1.0
    wgt[..., -1] = 1.0
    assert abs(np.sum(wgt * np.abs(xk) ** 2) / x.size - np.sum(x * x)) <= 1e-12 * np.sum(x * x)
    assert np.max(np.abs(F.irfft3(xk, 16) - x)) <= 1e-13


@pytest.mark.parametrize("mode", [(2, -3, 1), (1, 0, 0), (0, 5, 7)])
def test_gradient_and_hessian_of_a_single_mode(mode):
    n, L = 16, 100.0
    k = 2 * np.pi / L * np.array(mode, dtype=np.float64)
    x = np.arange(n) * L / n
    X = np.meshgrid(x, x, x, indexing="ij")
    phase = k[0] * X[0] + k[1] * X[1] + k[2] * X[2]
    delta = np.cos(phase)
    k2 = np.sum(k * k)
    for j in range(3):
        got = F.apply(F.multiplier("grad", n, L, j), delta)
        assert np.max(np.abs(got + k[j] / k2 * np.sin(phase))) <= 1e-13
        for i in range(j, 3):
            got = F.apply(F.multiplier("hess", n, L, (i, j)), delta)
            assert np.max(np.abs(got - k[i] * k[j] / k2 * np.cos(phase))) <= 1e-13


def test_nyquist_mode_has_no_gradient():
    """The derivative wavenumber vanishes at the Nyquist index (Hermitian
    multipliers); the alternating field along x feels no x gradient."""
    n, L = 8, 64.0
    delta = np.broadcast_to(((-1.0) ** np.arange(n))[:, None, None], (n, n, n)).copy()
    got = F.apply(F.multiplier("grad", n, L, 0), delta)
    assert np.max(np.abs(got)) <= 1e-14


@pytest.mark.parametrize("n", [8, 16])
def test_multiplier_adjoint_rule(n):
    """<Op_m x, y> = <x, Op_conj(m) y>: g is antisymmetric, h and w symmetric."""
    L = 50.0
    rng = np.random.default_rng(n)
    x, y = rng.standard_normal((2, n, n, n))
    pk = C.PowerSpectrum(0.3, 0.7, 0.96, 0.8)
    for kind, axis in [("grad", 0), ("grad", 1), ("grad", 2), ("hess", (0, 1)),
                       ("hess", (2, 2)), ("white", None)]:
        m = F.multiplier(kind, n, L, axis, pk)
        lhs = np.sum(F.apply(m, x) * y)
        rhs = np.sum(x * F.apply(np.conj(m), y))
        assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs)) * n ** 1.5


def test_whitening_parseval():
    """|delta_L|^2 = (1/N^3) sum over all k of |s_k|^2 w(k)^2."""
    n, L = 16, 128.0
    pk = C.PowerSpectrum(0.3, 0.7, 0.96, 0.8)
    s = np.random.default_rng(3).standard_normal((n, n, n))
    w = F.multiplier("white", n, L, pk=pk).real
    dl = F.apply(w, s)
    sk = F.rfft3(s)
    wgt = np.full(sk.shape, 2.0)
    wgt[..., 0] = 1.0
    wgt[..., -1] = 1.0
    rhs = np.sum(wgt * np.abs(sk) ** 2 * w ** 2) / n ** 3
    assert abs(np.sum(dl * dl) - rhs) <= 1e-13 * rhs
    # the multiplier itself: sqrt(P(k) / dq^3) on a sample of modes
    k = F.kgrid(n, L)
    assert w[0, 0, 0] == 0.0
    assert abs(w[1, 2, 3] - math.sqrt(pk(k[1, 2, 3]) / (L / n) ** 3)) <= 1e-14 * w[1, 2, 3]


# ---------------------------------------------------------------- cosmology
def test_eds_closed_forms():
    """Omega_m = 1: D1 = a, D2 = -3/7 a^2, f1 = 1, f2 = 2, G = a^(3/2)."""
    g = C.second_order_growth([0.1, 0.37, 1.0], 1.0)
    for a, v in g.items():
        assert abs(v["D1"] - a) <= 1e-10 * a
        assert abs(v["D2"] + 3.0 / 7.0 * a * a) <= 1e-10 * a * a
        assert abs(v["f1"] - 1.0) <= 1e-10
        assert abs(v["f2"] - 2.0) <= 1e-10
        assert abs(C.G_factor(a, 1.0, v["D1"], v["f1"]) - a ** 1.5) <= 1e-10
    co = C.fastpm_coefficients(1.0, 0.1, 1.0, 5)
    a, am = co["a"], co["a_mid"]
    assert np.allclose(co["Dr"], (a[1:] - a[:-1]) / am ** 1.5, rtol=1e-10, atol=0)
    assert np.allclose(co["K1"], (am ** 1.5 - a[:-1] ** 1.5) / a[:-1], rtol=1e-10, atol=0)
    assert np.allclose(co["K2"], (a[1:] ** 1.5 - am ** 1.5) / a[1:], rtol=1e-10, atol=0)
    assert abs(co["E_init"] - 0.1 ** -1.5) <= 1e-12 * co["E_init"]


@pytest.mark.parametrize("a", [0.1, 0.3, 0.55, 0.8, 1.0])
def test_linear_growth_integral_matches_ode(a):
    g = C.second_order_growth([a], 0.3)[a]
    assert abs(C.growth_D1(a, 0.3) - g["D1"]) <= 1e-10
    assert abs(C.growth_f1(a, 0.3) - g["f1"]) <= 1e-10


def test_second_order_growth_fitting_formula():
    """D2 / D1^2 ~ -(3/7) Om(a)^(-1/143) (Bouchet et al. 1995 fit)."""
    for a in [0.1, 0.5, 1.0]:
        g = C.second_order_growth([a], 0.3)[a]
        om_a = 0.3 * a ** -3 / (0.3 * a ** -3 + 0.7)
        fit = -3.0 / 7.0 * om_a ** (-1.0 / 143.0)
        assert abs(g["D2"] / g["D1"] ** 2 - fit) <= 1e-3 * abs(fit)


def test_sigma8_normalisation_independent_quadrature():
    pk = C.PowerSpectrum(0.3, 0.7, 0.96, 0.8)
    lnk = np.linspace(math.log(1e-5), math.log(1e3), 400001)
    k = np.exp(lnk)
    x = 8.0 * k
    W = np.where(x < 1e-2, 1 - x * x / 10 + x ** 4 / 280,
                 3 * (np.sin(x) - x * np.cos(x)) / np.where(x < 1e-2, 1.0, x) ** 3)
    f = k ** 3 * pk(k) * W ** 2
    h = lnk[1] - lnk[0]
    simpson = h / 3 * (f[0] + f[-1] + 4 * np.sum(f[1:-1:2]) + 2 * np.sum(f[2:-1:2]))
    assert abs(math.sqrt(simpson / (2 * math.pi ** 2)) - 0.8) <= 1e-8


def test_bbks_limits():
    assert abs(C.bbks_transfer(1e-8, 0.3, 0.7) - 1.0) <= 1e-6
    # large-q asymptote T ~ ln(2.34 q) / (2.34 q) / (6.71 q)
    q = 1e4
    k = q * 0.3 * 0.7
    asym = math.log(1 + 2.34 * q) / (2.34 * q) / (6.71 * q)
    assert abs(C.bbks_transfer(k, 0.3, 0.7) / asym - 1.0) <= 1e-3
