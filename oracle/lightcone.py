"""Lightcone of the particle output (test infrastructure only).

Paper section 2.2.1 item 3 and appendix A: snapshots of positions and
velocities are saved at a few scale factors (0.8, 0.9 and 1.0 in the paper);
each particle's trajectory is interpolated between them, and the scale factor
a_i at which it crosses the observer's past lightcone comes from the fixed
point a_i = DistToScaleFactor(|x_i(a_i) - x_obs|), iterated three times from
a_i = 1.  Redshift-space distortions then use the interpolated momentum at
a_i and the factor 1/(a_i^2 E(a_i)).

Readings where the paper is silent: the interpolation is linear in a between
the bracketing snapshots (both displacement and momentum, the snapshot
momentum being the kick-synchronised one); a_i is clamped to the snapshot
range, so particles farther than the comoving distance of the first snapshot
stay on it; the distance uses the box-wrapped position, as the line of sight
does; the comoving distance is chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a')) in
Mpc/h for the flat cosmology of the model.
"""
import numpy as np

from .cosmology import hubble_E

__all__ = ["C_OVER_H0", "comoving_distance", "scale_factor_at", "interp_weights",
           "Lightcone"]

C_OVER_H0 = 2997.92458  # Mpc/h

_GL_X, _GL_W = np.polynomial.legendre.leggauss(64)


def comoving_distance(a, omega_m):
    """chi(a) in Mpc/h by 64-point Gauss-Legendre quadrature over [a, 1]
    (the integrand is smooth there; the rule is exact to rounding)."""
    a = np.asarray(a, dtype=np.float64)
    half = 0.5 * (1.0 - a)
    ap = a[..., None] + half[..., None] * (_GL_X + 1.0)
    f = 1.0 / (ap * ap * hubble_E(ap, omega_m))
    return C_OVER_H0 * half * np.sum(_GL_W * f, axis=-1)


def scale_factor_at(dist, omega_m, a_lo, a_hi=1.0):
    """DistToScaleFactor: a with chi(a) = dist, clamped to [a_lo, a_hi]
    (bisection to rounding; chi decreases with a)."""
    dist = np.asarray(dist, dtype=np.float64)
    lo = np.full(dist.shape, a_lo)
    hi = np.full(dist.shape, a_hi)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        far = comoving_distance(mid, omega_m) > dist
        lo = np.where(far, mid, lo)
        hi = np.where(far, hi, mid)
    a = 0.5 * (lo + hi)
    a = np.where(dist >= comoving_distance(np.float64(a_lo), omega_m), a_lo, a)
    return np.where(dist <= comoving_distance(np.float64(a_hi), omega_m), a_hi, a)


def interp_weights(a, a_snap):
    """Index j of the lower snapshot and the weight t of the upper one,
    x(a) = (1 - t) x_j + t x_{j+1}; a inside [a_snap[0], a_snap[-1]]."""
    a_snap = np.asarray(a_snap, dtype=np.float64)
    if a_snap.size == 1:
        return np.zeros(np.shape(a), dtype=np.int64), np.zeros(np.shape(a))
    j = np.clip(np.searchsorted(a_snap, a, side="right") - 1, 0, a_snap.size - 2)
    t = (a - a_snap[j]) / (a_snap[j + 1] - a_snap[j])
    return j, t


class Lightcone:
    """Forward map and hand VJP of the lightcone for one model geometry.

    q: lattice positions (3, n); box, observer, omega_m; a_snap ascending
    (the last is a_final); iterations of the fixed point."""

    def __init__(self, q, box, observer, omega_m, a_snap, iterations=3):
        self.q = q
        self.box = float(box)
        self.obs = np.asarray(observer, dtype=np.float64)[:, None]
        self.om = omega_m
        self.a_snap = np.asarray(a_snap, dtype=np.float64)
        self.iterations = iterations
        self.a_lo, self.a_hi = float(self.a_snap[0]), float(self.a_snap[-1])

    def _interp(self, snaps, a):
        j, t = interp_weights(a, self.a_snap)
        if len(snaps) == 1:
            return snaps[0][0].copy(), snaps[0][1].copy(), np.zeros_like(snaps[0][0]), \
                np.zeros_like(snaps[0][1])
        D = np.stack([s[0] for s in snaps])   # (J, 3, n)
        P = np.stack([s[1] for s in snaps])
        cols = np.arange(a.size)
        d0, d1 = D[j, :, cols].T, D[j + 1, :, cols].T
        p0, p1 = P[j, :, cols].T, P[j + 1, :, cols].T
        span = self.a_snap[j + 1] - self.a_snap[j]
        d = (1.0 - t) * d0 + t * d1
        p = (1.0 - t) * p0 + t * p1
        return d, p, (d1 - d0) / span, (p1 - p0) / span

    def _sight(self, d):
        x = self.q + d
        y = x - self.box * np.floor(x / self.box)
        u = y - self.obs
        r = np.sqrt(np.sum(u * u, axis=0))
        safe = np.where(r > 0, r, 1.0)
        return np.where(r > 0, u / safe, 0.0), r

    def dadchi(self, a):
        """da/dchi = -a^2 E(a) / (c/H0); zero where a is clamped."""
        return -a * a * hubble_E(a, self.om) / C_OVER_H0

    def scale_factors(self, snaps):
        """a^(0) = a_hi, a^(k) = DistToScaleFactor(|x(a^(k-1)) - x_obs|)."""
        n = snaps[0][0].shape[1]
        a = [np.full(n, self.a_hi)]
        for _ in range(self.iterations):
            d, _, _, _ = self._interp(snaps, a[-1])
            _, r = self._sight(d)
            a.append(scale_factor_at(r, self.om, self.a_lo, self.a_hi))
        return a

    def forward(self, snaps, rsd):
        """Redshift-space displacement ds of every particle (and the state).

        snaps: list of (d, p) at a_snap, each (3, n); rsd 'none'|'z'|'radial'."""
        a = self.scale_factors(snaps)
        ai = a[-1]
        d, p, _, _ = self._interp(snaps, ai)
        c = 1.0 / (ai * ai * hubble_E(ai, self.om))
        if rsd == "none":
            ds = d.copy()
        elif rsd == "z":
            ds = d.copy()
            ds[2] += c * p[2]
        else:
            u, _ = self._sight(d)
            ds = d + c * np.sum(p * u, axis=0) * u
        return ds, dict(a=a, d=d, p=p, c=c)

    def vjp(self, snaps, rsd, st, ds_bar):
        """Cotangents (d_bar_j, p_bar_j) of every snapshot from ds_bar."""
        dbar = [np.zeros_like(s[0]) for s in snaps]
        pbar = [np.zeros_like(s[1]) for s in snaps]
        a = st["a"]
        ai, c = a[-1], st["c"]
        d, p, dd, dp = self._interp(snaps, ai)
        # s = d + c(a) * shift(d, p): cotangents of d, p and a at fixed a
        E = hubble_E(ai, self.om)
        # c(a) = 1/(a^2 E): dc/da = -c (2/a + dlnE/da), dlnE/da = -3 om a^-4 / (2 E^2)
        dlnE = -1.5 * self.om * ai ** -4 / (E * E)
        dc = -c * (2.0 / ai + dlnE)
        if rsd == "none":
            d_bar, p_bar, a_bar = ds_bar.copy(), np.zeros_like(ds_bar), np.zeros(ai.shape)
        elif rsd == "z":
            d_bar = ds_bar.copy()
            p_bar = np.zeros_like(ds_bar)
            p_bar[2] = c * ds_bar[2]
            a_bar = dc * p[2] * ds_bar[2]
        else:
            u, r = self._sight(d)
            inv_r = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
            ux = np.sum(u * ds_bar, axis=0)
            pu = np.sum(u * p, axis=0)
            d_bar = ds_bar + c * inv_r * (ux * (p - pu * u) + pu * (ds_bar - ux * u))
            p_bar = c * ux * u
            a_bar = dc * pu * ux
        # interpolation at a_i: d(a), p(a) depend on a through the slopes
        a_bar = a_bar + np.sum(d_bar * dd, axis=0) + np.sum(p_bar * dp, axis=0)
        self._scatter(dbar, pbar, ai, d_bar, p_bar)
        # back through the fixed point: a^(k) = A(r(a^(k-1)))
        for k in range(self.iterations, 0, -1):
            ak, aprev = a[k], a[k - 1]
            free = (ak > self.a_lo) & (ak < self.a_hi)
            g = np.where(free, a_bar * self.dadchi(ak), 0.0)    # r_bar
            dk, _, ddk, _ = self._interp(snaps, aprev)
            u, _ = self._sight(dk)
            r_d = g * u                                       # d r / d d = u
            self._scatter(dbar, pbar, aprev, r_d, np.zeros_like(r_d))
            a_bar = np.sum(r_d * ddk, axis=0) if k > 1 else np.zeros_like(a_bar)
        return dbar, pbar

    def _scatter(self, dbar, pbar, a, d_bar, p_bar):
        J = len(dbar)
        if J == 1:
            dbar[0] += d_bar
            pbar[0] += p_bar
            return
        j, t = interp_weights(a, self.a_snap)
        for jj in range(J - 1):
            lo = j == jj
            dbar[jj] += np.where(lo, 1.0 - t, 0.0) * d_bar
            pbar[jj] += np.where(lo, 1.0 - t, 0.0) * p_bar
            dbar[jj + 1] += np.where(lo, t, 0.0) * d_bar
            pbar[jj + 1] += np.where(lo, t, 0.0) * p_bar
