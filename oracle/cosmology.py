"""FP64 cosmology for the forward model (test infrastructure only).

Paper section 2.2.1, item 1: the linear field is the white noise scaled by
the square root of the fiducial linear power spectrum.  Item 2: 2LPT brings the
field to a = 0.1, then a FastPM-style leapfrog with constant step in a runs to
a = 1 (FastPM: Feng et al. 2016).  The paper names neither the transfer
function nor the integrator's coefficients; the readings used here are:

* flat LCDM without radiation, E(a) = sqrt(Om a^-3 + 1 - Om);
* BBKS transfer function with shape Gamma = Om h (no baryon term), amplitude
  fixed by sigma8 with a spherical top-hat of radius 8 Mpc/h;
* linear growth D1 from the closed-form integral valid for flat LCDM, second
  order growth D2 from its ODE in ln a, growing modes normalised so that
  D1(1) = 1 and D2 -> -(3/7) D1^2 at early times;
* FastPM factors: with momentum p = a^3 E dx/da and force F = -grad lap^-1
  delta, drift Dr = [D1(a1) - D1(a0)] / G(a_mid), half kicks
  K = [G(a_end) - G(a_start)] / D1(a_force), G = a^3 E dD1/da.  These move
  the linear growing mode exactly.
"""
import math

import numpy as np
from scipy import integrate

__all__ = [
    "hubble_E", "growth_D1", "growth_f1", "second_order_growth", "G_factor",
    "bbks_transfer", "sigma_R", "PowerSpectrum", "fastpm_coefficients",
]


def hubble_E(a, omega_m):
    """E(a) = H(a)/H0 for flat LCDM without radiation."""
    return np.sqrt(omega_m * np.asarray(a, dtype=np.float64) ** -3 + 1.0 - omega_m)


def _heath_integral(a, omega_m):
    """Integral from 0 to a of da' / (a' E(a'))^3."""
    f = lambda x: 1.0 / (x * float(hubble_E(x, omega_m))) ** 3
    val, _ = integrate.quad(f, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def _D_unnormalised(a, omega_m):
    """Growing mode D(a) = (5 Om / 2) E(a) int_0^a da'/(a'E)^3 (-> a early)."""
    return 2.5 * omega_m * float(hubble_E(a, omega_m)) * _heath_integral(a, omega_m)


def growth_D1(a, omega_m):
    """Linear growth factor normalised to D1(1) = 1."""
    return _D_unnormalised(a, omega_m) / _D_unnormalised(1.0, omega_m)


def growth_f1(a, omega_m):
    """f1 = dlnD1/dlna = dlnE/dlna + (5 Om/2) / (a^2 E^2 D_unnorm)."""
    E2 = float(hubble_E(a, omega_m)) ** 2
    return (-1.5 * omega_m * a ** -3 / E2
            + 2.5 * omega_m / (a * a * E2 * _D_unnormalised(a, omega_m)))


def second_order_growth(a_values, omega_m, a_start=1e-6):
    """D1, f1, D2, f2 from the growth ODEs in ln a.

    D'' + (2 + dlnE/dlna) D' - (3/2) Om(a) D = 0,
    D2'' + (2 + dlnE/dlna) D2' - (3/2) Om(a) D2 = -(3/2) Om(a) D1^2,
    with Om(a) = Om a^-3 / E^2 and dlnE/dlna = -(3/2) Om(a).  Growing modes
    start at a_start as D1 = a, D2 = -(3/7) a^2; both are then normalised by
    the unnormalised D1(1) (D2 by its square).
    """
    a_values = np.atleast_1d(np.asarray(a_values, dtype=np.float64))

    def rhs(lna, y):
        a = math.exp(lna)
        E2 = omega_m * a ** -3 + 1.0 - omega_m
        om_a = omega_m * a ** -3 / E2
        damp = 2.0 - 1.5 * om_a
        d1, d1p, d2, d2p = y
        return [d1p, -damp * d1p + 1.5 * om_a * d1,
                d2p, -damp * d2p + 1.5 * om_a * d2 - 1.5 * om_a * d1 * d1]

    y0 = [a_start, a_start, -3.0 / 7.0 * a_start ** 2, -6.0 / 7.0 * a_start ** 2]
    t_eval = np.unique(np.concatenate([np.log(a_values), [0.0]]))
    sol = integrate.solve_ivp(rhs, (math.log(a_start), 0.0), y0, method="DOP853",
                              t_eval=t_eval, rtol=1e-13, atol=1e-300)
    if not sol.success:
        raise RuntimeError(sol.message)
    norm = sol.y[0][-1]
    out = {}
    for a in a_values:
        i = int(np.argmin(np.abs(sol.t - math.log(a))))
        d1, d1p, d2, d2p = sol.y[:, i]
        out[float(a)] = dict(D1=d1 / norm, f1=d1p / d1, D2=d2 / norm ** 2, f2=d2p / d2)
    return out


def G_factor(a, omega_m, D1, f1):
    """G(a) = a^3 E dD1/da = a^2 E f1 D1 (the linear-theory momentum factor)."""
    return a * a * float(hubble_E(a, omega_m)) * f1 * D1


def bbks_transfer(k, omega_m, h):
    """BBKS transfer function, q = k / (Om h), k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (omega_m * h)
    x = 2.34 * q
    with np.errstate(divide="ignore", invalid="ignore"):
        lead = np.where(x > 0, np.log1p(x) / np.where(x > 0, x, 1.0), 1.0)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return lead * poly ** -0.25


def _tophat_window(x):
    """W(x) = 3 (sin x - x cos x) / x^3 (series below x = 1e-2)."""
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-2
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    series = 1.0 - x * x / 10.0 + x ** 4 / 280.0
    return np.where(small, series, full)


def sigma_R(pk, R, lnk_min=math.log(1e-5), lnk_max=math.log(1e3)):
    """sigma^2(R) = (1/2 pi^2) int k^3 P(k) W(kR)^2 dlnk, adaptive quadrature."""
    f = lambda lnk: (math.exp(lnk) ** 3 * float(pk(math.exp(lnk)))
                     * float(_tophat_window(math.exp(lnk) * R)) ** 2)
    edges = np.linspace(lnk_min, lnk_max, 513)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)
        total += v
    return math.sqrt(total / (2.0 * math.pi ** 2))


class PowerSpectrum:
    """P(k) = A k^ns T_BBKS(k)^2 with A set by sigma8 (k in h/Mpc, P in (Mpc/h)^3)."""

    def __init__(self, omega_m, h, n_s, sigma8):
        self.omega_m, self.h, self.n_s, self.sigma8 = omega_m, h, n_s, sigma8
        self.amplitude = 1.0
        s = sigma_R(self, 8.0)
        self.amplitude = (sigma8 / s) ** 2

    def __call__(self, k):
        k = np.asarray(k, dtype=np.float64)
        return self.amplitude * k ** self.n_s * bbks_transfer(k, self.omega_m, self.h) ** 2


def fastpm_coefficients(omega_m, a_init, a_final, n_steps):
    """Per-step FastPM factors for steps linear in a.

    a_n = a_init + n (a_final - a_init)/S, a_{n+1/2} the arithmetic midpoint.
    Dr_n = [D1(a_{n+1}) - D1(a_n)] / G(a_{n+1/2});
    K1_n = [G(a_{n+1/2}) - G(a_n)] / D1(a_n)      (first half kick of step n);
    K2_n = [G(a_{n+1}) - G(a_{n+1/2})] / D1(a_{n+1}) (second half kick).
    Also returns the 2LPT factors at a_init and the RSD factor 1/(a^2 E) at
    a_final.
    """
    S = int(n_steps)
    a = [a_init + n * (a_final - a_init) / S for n in range(S + 1)]
    amid = [0.5 * (a[n] + a[n + 1]) for n in range(S)]
    grow = second_order_growth(a + amid, omega_m)
    D1 = lambda x: grow[float(x)]["D1"]
    G = lambda x: G_factor(x, omega_m, grow[float(x)]["D1"], grow[float(x)]["f1"])
    Dr = np.array([(D1(a[n + 1]) - D1(a[n])) / G(amid[n]) for n in range(S)])
    K1 = np.array([(G(amid[n]) - G(a[n])) / D1(a[n]) for n in range(S)])
    K2 = np.array([(G(a[n + 1]) - G(amid[n])) / D1(a[n + 1]) for n in range(S)])
    g0 = grow[float(a_init)]
    return dict(
        a=np.array(a), a_mid=np.array(amid), Dr=Dr, K1=K1, K2=K2,
        D1_init=g0["D1"], f1_init=g0["f1"], D2_init=g0["D2"], f2_init=g0["f2"],
        E_init=float(hubble_E(a_init, omega_m)),
        rsd_factor=1.0 / (a_final ** 2 * float(hubble_E(a_final, omega_m))),
    )
