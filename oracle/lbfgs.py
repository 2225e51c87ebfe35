"""Projected L-BFGS (test infrastructure only).

Paper section 2.3.1: L-BFGS (limited-memory quasi-Newton, Nocedal & Wright
two-loop recursion) whose line search moves along s' = P(s + eps p) instead of
s + eps p, P being the projection of ``oracle.projection``.  Appendix B sets
the maximum step eps_max = 1 for the method.

Readings where the paper is silent: backtracking from eps_max, halving, up to
30 trials, with the sufficient-decrease (Armijo) test taken along the
projection arc, L(s') <= L(s) + c1 g.(s' - s) with c1 = 1e-4,
g.(s' - s) < 0 and L(s') < L(s) (the last rejects steps the projection
undoes, whose predicted decrease is rounding noise) (Bertsekas' rule for projected line searches: the projection
rescales long steps, so the unprojected eps g.p would demand far more
decrease than any projected step can give); initial inverse Hessian gamma I
with gamma = S.Y / Y.Y of the newest pair, and 1/|g| with an empty history,
so that the first step from a fresh history, -g/|g|, has unit length (the
direction is written with a hat in section 2.3.1; the gradient's scale says
nothing about the step's, above all without the prior term, where |g| grows
with the galaxy count); a pair is stored only when
S.Y > 1e-10 |S| |Y|; the history holds m = 10 pairs; a non-descent direction
resets the history and falls back to -g/|g|, and so does a quasi-Newton
direction whose line search fails (trials then continue numbering from
max_trials).  All dot products are FP64.
"""
import numpy as np

from .projection import project

__all__ = ["ProjectedLBFGS", "LineSearchError"]


class LineSearchError(RuntimeError):
    pass


class ProjectedLBFGS:
    def __init__(self, m=10, eps_max=1.0, c1=1e-4, max_trials=30, s_th=10.0,
                 seed=0, curvature_eps=1e-10, project_steps=True):
        self.m, self.eps_max, self.c1 = m, eps_max, c1
        self.max_trials, self.s_th, self.seed = max_trials, s_th, seed
        self.curvature_eps = curvature_eps
        # False: plain L-BFGS trial points s + eps p (the ablation baseline of
        # appendix B, table 1) instead of P(s + eps p)
        self.project_steps = project_steps
        self.S, self.Y = [], []

    def reset(self):
        self.S, self.Y = [], []

    def direction(self, g):
        """p = -H g by the two-loop recursion."""
        q = np.array(g, dtype=np.float64)
        alpha = []
        for S, Y in zip(reversed(self.S), reversed(self.Y)):
            rho = 1.0 / np.dot(S, Y)
            a = rho * np.dot(S, q)
            q = q - a * Y
            alpha.append(a)
        gamma = 1.0 / np.linalg.norm(g)
        if self.S:
            gamma = np.dot(self.S[-1], self.Y[-1]) / np.dot(self.Y[-1], self.Y[-1])
        r = gamma * q
        for (S, Y), a in zip(zip(self.S, self.Y), reversed(alpha)):
            rho = 1.0 / np.dot(S, Y)
            b = rho * np.dot(Y, r)
            r = r + (a - b) * S
        return -r

    def _search(self, s, g, L, p, fun, iteration, first_trial):
        """Backtracking along the projection arc; returns (accepted, trial,
        eps, s', g', L', resets)."""
        eps = self.eps_max
        for k in range(self.max_trials):
            trial = first_trial + k
            if self.project_steps:
                s_t, resets = project(s + eps * p, self.s_th, self.seed, iteration, trial)
            else:
                s_t, resets = s + eps * p, 0
            L_t, g_t = fun(s_t)
            g_t = np.asarray(g_t, dtype=np.float64).reshape(-1)
            s_t = s_t.reshape(-1)
            self._evals += 1
            decrease = float(np.dot(g, s_t - s))
            if decrease < 0 and L_t < L and L_t <= L + self.c1 * decrease:
                return True, trial, eps, s_t, g_t, L_t, resets
            eps *= 0.5
        return False, trial, eps, None, None, None, resets

    def step(self, s, g, L, fun, iteration):
        """One projected L-BFGS iteration.

        fun(s) -> (L, g).  Returns (s', g', L', info)."""
        s = np.asarray(s, dtype=np.float64).reshape(-1)
        g = np.asarray(g, dtype=np.float64).reshape(-1)
        self._evals = 0
        p = self.direction(g)
        gp = float(np.dot(g, p))
        restarted = False
        if not gp < 0:
            self.reset()
            p = -g / np.linalg.norm(g)
            gp = float(np.dot(g, p))
            restarted = True
        accepted, trial, eps, s_t, g_t, L_t, resets = self._search(s, g, L, p, fun,
                                                                    iteration, 0)
        if not accepted and self.S:
            self.reset()
            p = -g / np.linalg.norm(g)
            gp = float(np.dot(g, p))
            restarted = True
            accepted, trial, eps, s_t, g_t, L_t, resets = self._search(
                s, g, L, p, fun, iteration, self.max_trials)
        if not accepted:
            raise LineSearchError("no acceptable step in %d trials" % self.max_trials)
        S = s_t - s
        Y = g_t - g
        sy = float(np.dot(S, Y))
        stored = sy > self.curvature_eps * np.sqrt(np.dot(S, S) * np.dot(Y, Y))
        if stored:
            self.S.append(S)
            self.Y.append(Y)
            if len(self.S) > self.m:
                self.S.pop(0)
                self.Y.pop(0)
        info = dict(eps=eps, trials=trial + 1, evaluations=self._evals, resets=resets,
                    stored=bool(stored),
                    restarted=restarted, history=len(self.S), gp=gp)
        return s_t, g_t, L_t, info
