"""Differentiable forward model, its hand VJP and JVP (test infrastructure only).

Follows paper section 2.2.1 (items 1-5) with the workload readings of the
synthetic configurations:

1. s (real white noise, N_p^3) -> delta_L = Op_w[s]                    (item 1)
2. 2LPT at a_init: Psi1 = Op_g[delta_L], phi_ij = Op_h_ij[delta_L],
   mu2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2), Psi2 = -Op_g[mu2];
   d0 = D1 Psi1 + D2 Psi2, p0 = a^2 E (f1 D1 Psi1 + f2 D2 Psi2)         (item 2)
3. FastPM kick-drift-kick steps linear in a with CIC paint, Poisson
   force F = -grad lap^-1 delta_m on the mesh and CIC readout           (item 2)
4. RSD at a_final: shift c (p . d) d with d the line of sight from the
   observer (radial) or the z axis (plane parallel); c = 1/(a^2 E)       (item 3)
   -- or, with snapshot scale factors given, at each particle's lightcone
   crossing a_i (item 3, appendix A; ``oracle.lightcone``), the snapshots
   being the kick-synchronised states at those steps.
5. CIC of the shifted particles on the data grid -> delta_s; bias and
   response (items 4-5): linear, lambda = Nbar R (1 + b delta_s), or the
   paper's power law times a sigmoid (item 4, eq. of the galaxy bias),
   lambda = Nbar R u^alpha sigmoid(K (delta_s - delta_th)), u = 1 + delta_s
   floored at 1e-6 (the paper leaves lambda = 0 in empty cells, where
   log lambda diverges; below the floor u is constant).
6. Loss L = 1/2 D + 1/2 w_prior sum s^2 over the mask M = [R >= r_min], with
   the data term D = sum_M (N - lambda)^2 / sigma^2, sigma^2 = Nbar R (the
   Gaussian chi^2 of the benchmarked reconstructions), or D = -2 log L_P with
   the paper's Poisson log-likelihood (section 2.2.2), log L_P =
   sum_M (-lambda + N log lambda - log N!).

Particles carry a displacement d from their lattice point q_n = n dq and a
momentum p = a^3 E dx/da, stored as (3, N_p^3) arrays in C order of n.
"""
from dataclasses import dataclass, field

import numpy as np

from . import cic, cosmology, fourier
from .lightcone import Lightcone

__all__ = ["Problem", "Model"]


@dataclass
class Problem:
    """Plain statement of one reconstruction problem."""
    n_part: int
    n_mesh: int
    box: float
    n_steps: int = 10
    a_init: float = 0.1
    a_final: float = 1.0
    omega_m: float = 0.3
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    rsd: str = "radial"            # 'none' | 'z' | 'radial'
    observer: tuple = (0.0, 0.0, 0.0)
    bias: float = 1.5
    nbar: float = 1.0
    r_min: float = 1e-3
    prior_weight: float = 1.0
    loss: str = "gauss"            # 'gauss' (linear bias, chi^2) | 'poisson' (paper's model)
    bias_alpha: float = 0.7        # power-law index alpha (section 2.2.1, item 4)
    bias_delta_th: float = 1.2     # sigmoid threshold delta_th
    bias_k: float = 3.0            # sigmoid steepness K
    lightcone: tuple = ()          # snapshot scale factors, ascending, last a_final; () = off
    lc_iterations: int = 3         # fixed-point iterations of the crossing scale factor


class Model:
    """FP64 forward model for one Problem (coefficients computed once)."""

    def __init__(self, prob: Problem):
        self.p = prob
        n, nm = prob.n_part, prob.n_mesh
        self.dq = prob.box / n
        self.dm = prob.box / nm
        self.nbar_mesh = (n / nm) ** 3
        self.coef = cosmology.fastpm_coefficients(prob.omega_m, prob.a_init,
                                                  prob.a_final, prob.n_steps)
        self.pk = cosmology.PowerSpectrum(prob.omega_m, prob.h, prob.n_s, prob.sigma8)
        j = np.arange(n, dtype=np.float64) * self.dq
        qx, qy, qz = np.meshgrid(j, j, j, indexing="ij")
        self.q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()])
        self._mult = {}
        self.snap_steps = []
        self.lc = None
        if prob.lightcone:
            S = prob.n_steps
            a_n = prob.a_init + np.arange(S + 1) * (prob.a_final - prob.a_init) / S
            la = list(prob.lightcone)
            if abs(la[-1] - prob.a_final) > 1e-9 or any(b <= a for a, b in zip(la, la[1:])):
                raise ValueError("snapshots must ascend and end at a_final")
            for a in la[:-1]:
                m = int(np.argmin(np.abs(a_n - a)))
                if abs(a_n[m] - a) > 1e-9 or m < 1 or m >= S:
                    raise ValueError("snapshot a = %g is not an interior step" % a)
                self.snap_steps.append(m)
            self.lc = Lightcone(self.q, prob.box, prob.observer, prob.omega_m,
                                [a_n[m] for m in self.snap_steps] + [prob.a_final],
                                prob.lc_iterations)

    # ------------------------------------------------------------ multipliers
    def mult(self, kind, axis=None, mesh=False):
        key = (kind, axis, mesh)
        if key not in self._mult:
            n = self.p.n_mesh if mesh else self.p.n_part
            self._mult[key] = fourier.multiplier(kind, n, self.p.box, axis, self.pk)
        return self._mult[key]

    def op(self, kind, x, axis=None, mesh=False):
        return fourier.apply(self.mult(kind, axis, mesh), x)

    def _field(self, v):
        n = self.p.n_part
        return v.reshape(n, n, n)

    # ------------------------------------------------------------------- 2LPT
    def lpt(self, s):
        """White noise -> (d0, p0) plus the fields the adjoint needs."""
        return self.lpt_from_linear(self.op("white", s))

    def lpt_from_linear(self, delta_L):
        """Linear field at a = 1 -> 2LPT displacement and momentum at a_init."""
        c = self.coef
        psi1 = np.stack([self.op("grad", delta_L, j).ravel() for j in range(3)])
        phi = {ij: self.op("hess", delta_L, ij) for ij in
               [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]}
        mu2 = (phi[0, 0] * phi[1, 1] + phi[0, 0] * phi[2, 2] + phi[1, 1] * phi[2, 2]
               - phi[0, 1] ** 2 - phi[0, 2] ** 2 - phi[1, 2] ** 2)
        psi2 = np.stack([-self.op("grad", mu2, j).ravel() for j in range(3)])
        a2E = self.p.a_init ** 2 * c["E_init"]
        d0 = c["D1_init"] * psi1 + c["D2_init"] * psi2
        p0 = a2E * (c["f1_init"] * c["D1_init"] * psi1 + c["f2_init"] * c["D2_init"] * psi2)
        return d0, p0, dict(delta_L=delta_L, psi1=psi1, psi2=psi2, phi=phi, mu2=mu2)

    # ------------------------------------------------------------------ force
    def density_mesh(self, d):
        """delta_m = rho / nbar - 1 on the PM mesh for displacements d."""
        rho = cic.paint(self.q + d, self.p.n_mesh, self.dm)
        return rho / self.nbar_mesh - 1.0

    def force_mesh(self, d):
        """g_j = Op_g_j[delta_m], the force field -grad lap^-1 delta_m."""
        delta = self.density_mesh(d)
        return [self.op("grad", delta, j, mesh=True) for j in range(3)]

    def force(self, d, g=None):
        if g is None:
            g = self.force_mesh(d)
        x = self.q + d
        return np.stack([cic.readout(x, g[j], self.dm) for j in range(3)]), g

    def kick_coefficients(self):
        """c_0 = K1_0, c_n = K2_{n-1} + K1_n (1 <= n < S), c_S = K2_{S-1}."""
        K1, K2, S = self.coef["K1"], self.coef["K2"], self.p.n_steps
        return [K1[0]] + [K2[n - 1] + K1[n] for n in range(1, S)] + [K2[S - 1]]

    # -------------------------------------------------------------------- KDK
    def evolve(self, d0, p0, snaps=None):
        """Kick-drift-kick with merged half kicks; returns the tape of
        displacements d_0..d_S, force meshes g_0..g_S and final momentum.
        With a list snaps, the synchronised states (d_m, p_m) of the snapshot
        steps m are appended to it (p_m = p_{m-1/2} + K2_{m-1} F(d_m))."""
        kc = self.kick_coefficients()
        Dr, K2 = self.coef["Dr"], self.coef["K2"]
        d, p = d0.copy(), p0.copy()
        F, g = self.force(d)
        p = p + kc[0] * F
        tape_d, tape_g = [d], [g]
        for n in range(self.p.n_steps):
            d = d + Dr[n] * p
            F, g = self.force(d)
            if snaps is not None and n + 1 in self.snap_steps:
                snaps.append((d.copy(), p + K2[n] * F))
            p = p + kc[n + 1] * F
            tape_d.append(d)
            tape_g.append(g)
        return d, p, tape_d, tape_g

    def redshift_space(self, dS, pS, snaps):
        """Redshift-space displacements: at a_final, or on the lightcone."""
        if self.lc is None:
            return self.rsd(dS, pS), None
        ds, lc_state = self.lc.forward(list(snaps) + [(dS, pS)], self.p.rsd)
        return ds, lc_state

    # -------------------------------------------------------------------- RSD
    def line_of_sight(self, d):
        """Unit vector from the observer to the wrapped position, and r."""
        L = self.p.box
        x = self.q + d
        y = x - L * np.floor(x / L)
        u = y - np.asarray(self.p.observer, dtype=np.float64)[:, None]
        r = np.sqrt(np.sum(u * u, axis=0))
        safe = np.where(r > 0, r, 1.0)
        return np.where(r > 0, u / safe, 0.0), r

    def rsd(self, d, p):
        c = self.coef["rsd_factor"]
        if self.p.rsd == "none":
            return d.copy()
        if self.p.rsd == "z":
            out = d.copy()
            out[2] += c * p[2]
            return out
        dhat, _ = self.line_of_sight(d)
        return d + c * np.sum(p * dhat, axis=0) * dhat

    # ------------------------------------------------------------ observation
    def data_density(self, ds):
        """delta_s on the data grid (N_d = N_p, nbar_d = 1)."""
        n = self.p.n_part
        return cic.paint(self.q + ds, n, self.dq) - 1.0

    U_FLOOR = 1e-6   # floor of 1 + delta_s in the power-law bias

    def observe(self, delta_s, response):
        """lambda = Nbar R (1 + b delta_s), or Nbar R u^alpha sigmoid(K (delta_s - delta_th))."""
        if self.p.loss == "poisson":
            u = np.maximum(1.0 + delta_s, self.U_FLOOR)
            sig = 1.0 / (1.0 + np.exp(-self.p.bias_k * (delta_s - self.p.bias_delta_th)))
            return self.p.nbar * response * u ** self.p.bias_alpha * sig
        return self.p.nbar * response * (1.0 + self.p.bias * delta_s)

    def chi2(self, lam, counts, response):
        """Data term D: Gaussian chi^2, or -2 log L_P of the Poisson model."""
        m = response >= self.p.r_min
        if self.p.loss == "poisson":
            from scipy.special import gammaln
            n = counts[m].astype(np.float64)
            return float(2.0 * np.sum(lam[m] - n * np.log(lam[m]) + gammaln(n + 1.0)))
        var = self.p.nbar * response[m]
        return float(np.sum((counts[m] - lam[m]) ** 2 / var))

    def loss(self, s, counts, response, return_state=False):
        """L(s) = 1/2 chi^2 + 1/2 w_prior |s|^2, with everything the adjoint needs."""
        s = np.asarray(s, dtype=np.float64)
        d0, p0, lpt = self.lpt(s)
        snaps = []
        dS, pS, tape_d, tape_g = self.evolve(d0, p0, snaps)
        ds, lc_state = self.redshift_space(dS, pS, snaps)
        delta_s = self.data_density(ds)
        lam = self.observe(delta_s, response)
        chi2 = self.chi2(lam, counts, response)
        prior = float(np.sum(s * s))
        L = 0.5 * chi2 + 0.5 * self.p.prior_weight * prior
        if not return_state:
            return L
        return L, dict(lpt=lpt, d0=d0, p0=p0, dS=dS, pS=pS, tape_d=tape_d,
                       tape_g=tape_g, ds=ds, delta_s=delta_s, lam=lam,
                       chi2=chi2, prior=prior, snaps=snaps, lc=lc_state)

    def forward(self, s):
        """s -> delta_s (the redshift-space data-grid overdensity)."""
        d0, p0, _ = self.lpt(np.asarray(s, dtype=np.float64))
        snaps = []
        dS, pS, _, _ = self.evolve(d0, p0, snaps)
        return self.data_density(self.redshift_space(dS, pS, snaps)[0])

    # ---------------------------------------------------------------- adjoint
    def loss_seed(self, lam, counts, response, delta_s=None):
        """dL/d delta_s = 1/2 dD/d delta_s: M b Nbar R (lambda - N) / sigma^2 (Gaussian), or
        M (1 - N / lambda) dlambda/d delta_s (Poisson, delta_s needed)."""
        m = response >= self.p.r_min
        out = np.zeros_like(lam)
        if self.p.loss == "poisson":
            d = delta_s[m]
            a, k = self.p.bias_alpha, self.p.bias_k
            u = np.maximum(1.0 + d, self.U_FLOOR)
            sig = 1.0 / (1.0 + np.exp(-k * (d - self.p.bias_delta_th)))
            du = np.where(1.0 + d > self.U_FLOOR, a * u ** (a - 1.0), 0.0)
            dlam = self.p.nbar * response[m] * (du * sig + u ** a * k * sig * (1.0 - sig))
            out[m] = (1.0 - counts[m] / lam[m]) * dlam
            return out
        var = self.p.nbar * response[m]
        out[m] = self.p.bias * self.p.nbar * response[m] * (lam[m] - counts[m]) / var
        return out

    def rsd_vjp(self, d, p, xs_bar):
        c = self.coef["rsd_factor"]
        if self.p.rsd == "none":
            return xs_bar.copy(), np.zeros_like(xs_bar)
        if self.p.rsd == "z":
            p_bar = np.zeros_like(xs_bar)
            p_bar[2] = c * xs_bar[2]
            return xs_bar.copy(), p_bar
        dhat, r = self.line_of_sight(d)
        inv_r = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
        dx = np.sum(dhat * xs_bar, axis=0)
        pd = np.sum(dhat * p, axis=0)
        perp_p = p - pd * dhat
        perp_x = xs_bar - dx * dhat
        d_bar = xs_bar + c * inv_r * (dx * perp_p + pd * perp_x)
        p_bar = c * dx * dhat
        return d_bar, p_bar

    def force_vjp(self, d, g, v):
        """Cotangent of positions for F(d) = readout(q + d, g(d)) given dF = v."""
        x = self.q + d
        gbar = [cic.paint(x, self.p.n_mesh, self.dm, weight=v[j]) for j in range(3)]
        delta_bar = -fourier.apply_sum([(self.mult("grad", j, True), gbar[j])
                                        for j in range(3)])
        rho_bar = delta_bar / self.nbar_mesh
        xbar = cic.readout_gradient(x, rho_bar, self.dm)
        for j in range(3):
            xbar += v[j] * cic.readout_gradient(x, g[j], self.dm)
        return xbar

    def vjp_state(self, st, delta_bar):
        """s_bar = J^T delta_bar for s -> delta_s (no prior term)."""
        c = self.coef
        Dr = c["Dr"]
        kc = self.kick_coefficients()
        xs_bar = cic.readout_gradient(self.q + st["ds"], delta_bar, self.dq)
        snap_bar = {}
        if self.lc is None:
            d_bar, p_bar = self.rsd_vjp(st["dS"], st["pS"], xs_bar)
        else:
            snaps = list(st["snaps"]) + [(st["dS"], st["pS"])]
            db, pb = self.lc.vjp(snaps, self.p.rsd, st["lc"], xs_bar)
            d_bar, p_bar = db[-1], pb[-1]
            snap_bar = {m: (db[j], pb[j]) for j, m in enumerate(self.snap_steps)}
        S = self.p.n_steps
        K2 = c["K2"]
        for n in range(S - 1, -1, -1):
            m = n + 1
            v = kc[m] * p_bar
            if m in snap_bar:
                # snapshot (d_m, p_{m-1/2} + K2_{m-1} F(d_m))
                sd, sp = snap_bar[m]
                d_bar = d_bar + sd
                v = v + K2[m - 1] * sp
            d_bar = d_bar + self.force_vjp(st["tape_d"][m], st["tape_g"][m], v)
            if m in snap_bar:
                p_bar = p_bar + snap_bar[m][1]
            p_bar = p_bar + Dr[n] * d_bar
        d_bar = d_bar + self.force_vjp(st["tape_d"][0], st["tape_g"][0], kc[0] * p_bar)
        return self.lpt_vjp(st["lpt"], d_bar, p_bar)

    def lpt_vjp(self, lpt, d_bar, p_bar):
        c = self.coef
        a2E = self.p.a_init ** 2 * c["E_init"]
        psi1_bar = c["D1_init"] * d_bar + a2E * c["f1_init"] * c["D1_init"] * p_bar
        psi2_bar = c["D2_init"] * d_bar + a2E * c["f2_init"] * c["D2_init"] * p_bar
        F = self._field
        mu2_bar = fourier.apply_sum([(self.mult("grad", j), F(psi2_bar[j])) for j in range(3)])
        phi = lpt["phi"]
        phi_bar = {
            (0, 0): mu2_bar * (phi[1, 1] + phi[2, 2]),
            (1, 1): mu2_bar * (phi[0, 0] + phi[2, 2]),
            (2, 2): mu2_bar * (phi[0, 0] + phi[1, 1]),
            (0, 1): -2.0 * mu2_bar * phi[0, 1],
            (0, 2): -2.0 * mu2_bar * phi[0, 2],
            (1, 2): -2.0 * mu2_bar * phi[1, 2],
        }
        pairs = [(-self.mult("grad", j), F(psi1_bar[j])) for j in range(3)]
        pairs += [(self.mult("hess", ij), phi_bar[ij]) for ij in phi_bar]
        deltaL_bar = fourier.apply_sum(pairs)
        return self.op("white", deltaL_bar)

    def loss_and_grad(self, s, counts, response):
        """(L, grad L, state)."""
        s = np.asarray(s, dtype=np.float64)
        L, st = self.loss(s, counts, response, return_state=True)
        seed = self.loss_seed(st["lam"], counts, response, st["delta_s"])
        grad = self.vjp_state(st, seed) + self.p.prior_weight * s
        return L, grad, st

    def vjp(self, s, delta_bar):
        _, st = self.loss(s, np.zeros(s.shape), np.zeros(s.shape), return_state=True)
        return self.vjp_state(st, delta_bar)

    # -------------------------------------------------------------------- JVP
    def jvp(self, s, ds):
        """Tangent of delta_s along the white-noise tangent ds (no lightcone)."""
        if self.lc is not None:
            raise NotImplementedError("the tangent model has no lightcone")
        c = self.coef
        s = np.asarray(s, dtype=np.float64)
        d0, p0, lpt = self.lpt(s)
        phi = lpt["phi"]
        tdL = self.op("white", ds)
        tpsi1 = np.stack([self.op("grad", tdL, j).ravel() for j in range(3)])
        tphi = {ij: self.op("hess", tdL, ij) for ij in phi}
        tmu2 = (tphi[0, 0] * phi[1, 1] + phi[0, 0] * tphi[1, 1]
                + tphi[0, 0] * phi[2, 2] + phi[0, 0] * tphi[2, 2]
                + tphi[1, 1] * phi[2, 2] + phi[1, 1] * tphi[2, 2]
                - 2 * phi[0, 1] * tphi[0, 1] - 2 * phi[0, 2] * tphi[0, 2]
                - 2 * phi[1, 2] * tphi[1, 2])
        tpsi2 = np.stack([-self.op("grad", tmu2, j).ravel() for j in range(3)])
        a2E = self.p.a_init ** 2 * c["E_init"]
        td = c["D1_init"] * tpsi1 + c["D2_init"] * tpsi2
        tp = a2E * (c["f1_init"] * c["D1_init"] * tpsi1 + c["f2_init"] * c["D2_init"] * tpsi2)

        def force_jvp(d, td):
            x = self.q + d
            g = self.force_mesh(d)
            trho = cic.paint_jvp(x, td, self.p.n_mesh, self.dm) / self.nbar_mesh
            tg = [self.op("grad", trho, j, mesh=True) for j in range(3)]
            return np.stack([cic.readout_jvp(x, td, g[j], tg[j], self.dm) for j in range(3)])

        kc = self.kick_coefficients()
        Dr = c["Dr"]
        d, p = d0.copy(), p0.copy()
        F, _ = self.force(d)
        tF = force_jvp(d, td)
        p, tp = p + kc[0] * F, tp + kc[0] * tF
        for n in range(self.p.n_steps):
            d, td = d + Dr[n] * p, td + Dr[n] * tp
            F, _ = self.force(d)
            tF = force_jvp(d, td)
            p, tp = p + kc[n + 1] * F, tp + kc[n + 1] * tF
        crsd = c["rsd_factor"]
        if self.p.rsd == "none":
            ds_, tds = d, td
        elif self.p.rsd == "z":
            ds_, tds = d.copy(), td.copy()
            ds_[2] += crsd * p[2]
            tds[2] += crsd * tp[2]
        else:
            dhat, r = self.line_of_sight(d)
            inv_r = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
            tdhat = (td - np.sum(dhat * td, axis=0) * dhat) * inv_r
            pd = np.sum(p * dhat, axis=0)
            ds_ = d + crsd * pd * dhat
            tds = td + crsd * (np.sum(tp * dhat, axis=0) * dhat
                               + np.sum(p * tdhat, axis=0) * dhat + pd * tdhat)
        return cic.paint_jvp(self.q + ds_, tds, self.p.n_part, self.dq)
