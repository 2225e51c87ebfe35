"""The study diagnostics (CPU): the cross-correlation coefficient r_c(k) is 1
for a field against itself and -1 against its negative in every k bin, and
of order N^-1/2 per bin for independent fields; the Gaussian smoothing keeps
the mean and damps a single mode by exp(-k^2 sigma^2 / 2); the white-noise
moments of a normal sample."""
import numpy as np

from paper_2604_26823_amd import studies


def test_cross_correlation_limits():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((32, 32, 32))
    b = rng.standard_normal((32, 32, 32))
    same = np.array(studies._cross_correlation(a, a, 100.0))
    neg = np.array(studies._cross_correlation(a, -a, 100.0))
    ind = np.array(studies._cross_correlation(a, b, 100.0))
    assert np.allclose(same[:, 1], 1.0, atol=1e-12)
    assert np.allclose(neg[:, 1], -1.0, atol=1e-12)
    assert np.all(np.abs(ind[:, 1]) < 0.2)
    assert np.all(np.diff(same[:, 0]) > 0)


def test_smoothing_of_a_single_mode():
    n, sig = 32, 2.0
    x = np.arange(n)
    X = np.meshgrid(x, x, x, indexing="ij")[0]
    f = 3.0 + np.cos(2 * np.pi * 4 * X / n)
    out = studies._smooth(f, sig)
    k = 2 * np.pi * 4 / n
    ref = 3.0 + np.exp(-0.5 * k * k * sig * sig) * np.cos(2 * np.pi * 4 * X / n)
    assert np.max(np.abs(out - ref)) < 1e-12


def test_white_noise_moments():
    x = np.random.default_rng(1).standard_normal(1 << 20)
    st = studies._white_noise_stats(x)
    assert abs(st["mean"]) < 5e-3 and abs(st["std"] - 1) < 5e-3
    assert abs(st["excess_kurtosis"]) < 0.02 and st["frac_above_4"] < 2e-4
