"""Writes the oracle's expected values for the 128^3 survey-shaped problem
(512 Mpc/h, 4 Mpc/h cells, 10 steps, radial RSD, the 40 x 40 degree
footprint with the r^2 exp(-(r/300)^1.5) selection, ~1e6 galaxies), the
scale of the paper's first (4 Mpc/h) reconstruction level (section 3):

* c2_density_grad.txt (part "eval"): delta_s and the loss gradient at 8192
  sampled cells each, at the configuration's seeded start field, with the
  loss, the data term and the full-field norms;
* c2_trajectory.txt (part "trajectory"): the loss after each of 50 projected
  L-BFGS iterations (section 2.3.1) from the projected start, with the
  rank-order matching event (real space, Fourier space, projection, history
  reset) every 20 iterations (section 2.3.2), and the evaluations each
  iteration made;
* c2_trajectory_perturbed_<eps>.txt (part "trajectory --perturb eps"): the
  same run from the start field times (1 + eps xi), xi white noise of seed 1
  - how far a rounding-level difference in the input carries along the path;
* c2_counts.npz (part "counts"): the mock galaxy counts all parts use, so
  that a test can set the same observation without the oracle's forward.

Truth and counts come from the oracle's own forward model (seeds of the
configuration: truth 2001, counts 2002, start 2003, generator key 2004).

Run from the repository root, one part per process (each part takes one to
three hours on 8 cores):
    python tests/golden/make_c2_golden.py eval
    python tests/golden/make_c2_golden.py trajectory
    python tests/golden/make_c2_golden.py trajectory --perturb 1e-14
    python tests/golden/make_c2_golden.py trajectory --perturb 1e-7
    python tests/golden/make_c2_golden.py counts
Calls only the oracle and the seeded input generators."""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbfgs, projection, rom  # noqa: E402
from oracle.model import Model, Problem  # noqa: E402
from paper_2604_26823_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLES = 8192
ITERATIONS = 50


def problem():
    cfg = inputs.config(2)
    R = inputs.response_field(cfg)
    cfg["nbar"] = inputs.nbar_for(cfg, R)
    mdl = Model(Problem(**{k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}))
    sd = inputs.seeds(2)
    s_true = inputs.white_noise(cfg["n_part"], sd["truth"])
    N = inputs.poisson_counts(mdl.observe(mdl.forward(s_true), R), R, cfg["r_min"], sd["counts"])
    s0 = inputs.white_noise(cfg["n_part"], sd["start"])
    return cfg, mdl, R, N, s0


def part_eval():
    cfg, mdl, R, N, s0 = problem()
    L, g, st = mdl.loss_and_grad(s0, N, R)
    delta, g = st["delta_s"].ravel(), g.ravel()
    rng = np.random.default_rng(8193)
    i_d = np.sort(rng.choice(delta.size, SAMPLES, replace=False))
    i_g = np.sort(rng.choice(g.size, SAMPLES, replace=False))
    with open(os.path.join(HERE, "c2_density_grad.txt"), "w") as fh:
        fh.write("# oracle, 128^3 particles and mesh, 512 Mpc/h, 10 steps, radial RSD, cone;\n")
        fh.write("# written by make_c2_golden.py at the seeded start field (seed 2003)\n")
        fh.write("# loss %.17g chi2 %.17g prior %.17g\n" % (L, st["chi2"], st["prior"]))
        fh.write("# delta_s full-field L2 %.17g; gradient full-field L2 %.17g\n"
                 % (np.linalg.norm(delta), np.linalg.norm(g)))
        fh.write("# kind (0 delta_s, 1 gradient) linear_index value\n")
        for i in i_d:
            fh.write("0 %d %.17g\n" % (i, delta[i]))
        for i in i_g:
            fh.write("1 %d %.17g\n" % (i, g[i]))


def part_trajectory(perturb):
    cfg, mdl, R, N, s0 = problem()
    n, seed, every = cfg["n_part"], cfg["seed"], cfg["rom_every"]
    if perturb:
        s0 = s0 * (1.0 + perturb * np.random.default_rng(1).standard_normal(s0.shape))
        name = "c2_trajectory_perturbed_%g.txt" % perturb
    else:
        name = "c2_trajectory.txt"

    def fun(x):
        L, g, _ = mdl.loss_and_grad(x.reshape(n, n, n), N, R)
        return L, g.reshape(-1)

    t0 = time.time()
    s, _ = projection.project(s0, 10.0, seed, 0, 0)
    L, g = fun(s)
    s = s.reshape(-1)
    opt = lbfgs.ProjectedLBFGS(seed=seed)
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        fh.write("# oracle, 128^3 projected L-BFGS from the projected start field (seed 2003)")
        fh.write(" times (1 + %g xi)\n" % perturb if perturb else "\n")
        fh.write("# rank-order matching every %d iterations; written by make_c2_golden.py\n"
                 % every)
        fh.write("# iteration loss evaluations (iteration 0: the start)\n")
        fh.write("0 %.17g 1\n" % L)
        fh.flush()
        for it in range(ITERATIONS):
            s, g, L, info = opt.step(s, g, L, fun, it)
            ev = info["evaluations"]
            if (it + 1) % every == 0:
                x, _ = rom.rom_real(s.reshape(n, n, n), R, cfg["r_min"], seed, it + 1)
                x, _ = rom.rom_fourier(x, cfg["box"], seed, it + 1)
                x, _ = projection.project(x, 10.0, seed, it + 1, 0)
                s = x.reshape(-1)
                opt.reset()
                L, g = fun(s)
                ev += 1
            fh.write("%d %.17g %d\n" % (it + 1, L, ev))
            fh.flush()
            print("iteration %d loss %.12e (%.0f s)" % (it + 1, L, time.time() - t0), flush=True)


def part_counts():
    _, _, _, N, _ = problem()
    np.savez_compressed(os.path.join(HERE, "c2_counts.npz"), counts=N)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("part", choices=["eval", "trajectory", "counts"])
    ap.add_argument("--perturb", type=float, default=0.0)
    a = ap.parse_args()
    if a.part == "eval":
        part_eval()
    elif a.part == "counts":
        part_counts()
    else:
        part_trajectory(a.perturb)
