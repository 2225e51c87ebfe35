"""The projected L-BFGS path amplifies tiny input differences (CPU, oracle).

This is the property that bounds how closely any finite-precision
implementation can follow the FP64 oracle's loss trajectory: a 1e-7
relative perturbation of the start field grows by orders of magnitude within
a dozen iterations on c1 (32^3, 8 Mpc/h cells, half-box mask)."""
import numpy as np

from oracle import lbfgs, projection
from oracle.model import Model, Problem
from paper_2604_26823_amd import inputs


def test_oracle_trajectory_sensitivity():
    cfg = inputs.config(1)
    R = inputs.response_field(cfg)
    mdl = Model(Problem(**{k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}))
    sd = inputs.seeds(1)
    s_true = inputs.white_noise(32, sd["truth"])
    N = inputs.poisson_counts(mdl.observe(mdl.forward(s_true), R), R, cfg["r_min"], sd["counts"])
    s0 = inputs.white_noise(32, sd["start"])

    def fun(x):
        L, g, _ = mdl.loss_and_grad(x.reshape(32, 32, 32), N, R)
        return L, g.reshape(-1)

    def run(start, iters=12):
        s, _ = projection.project(start, 10.0, cfg["seed"], 0, 0)
        L, g = fun(s)
        s = s.reshape(-1)
        opt = lbfgs.ProjectedLBFGS(seed=cfg["seed"])
        out = [L]
        for it in range(iters):
            s, g, L, _ = opt.step(s, g, L, fun, it)
            out.append(L)
        return np.array(out)

    a = run(s0)
    b = run(s0 * (1 + 1e-7 * np.random.default_rng(1).standard_normal(s0.shape)))
    rel = np.abs(a - b) / np.abs(a)
    assert rel[0] < 1e-7
    assert rel[-1] > 1000 * rel[0]
