"""Seeded synthetic workloads (shared by the tests, the benchmark and the oracle
side of the parity checks).

This module only builds inputs: problem sizes and parameters, white-noise
fields, the survey response (selection) field and Poisson counts drawn from a
given rate field.  It holds none of the method's arithmetic; the rate field
of the truth is computed by whichever forward model the caller trusts.

The paper reconstructs a mock lightcone catalogue (section 2.1) that is not
available here; synthetic survey-shaped volumes stand in for it:

* c1 - 32^3 particles and mesh, 256 Mpc/h, 5 steps, plane-parallel RSD along
  z, response 1 on the half box x < L/2, mean one galaxy per cell;
* c2 - 128^3, 512 Mpc/h (4 Mpc/h cells), 10 steps, observer at the box
  corner, radial RSD, a 40 x 40 degree gnomonic square footprint centred on
  the box diagonal and radial selection R(r) = exp(-(r/300)^1.5) (the r^2 of
  n(r) being the volume factor), about 1e6 galaxies;
* c3 - 256^3, 1000 Mpc/h, 10 steps, same geometry, about 8e6 galaxies;
* c4 - 256^3 particles on a 512^3 force mesh, 1000 Mpc/h, 20 steps;
* c5 - 512^3 particles on a 1024^3 mesh, 2000 Mpc/h, 20 steps, c3's
  selection density;
* c6 - the paper's own scale (sections 2.1 and 2.2.1): Planck13 parameters,
  256^3 particles and mesh in a 500 Mpc/h box whose centre lies 400 Mpc/h
  from the observer along the box diagonal, 18 steps of 0.05 in a, a disk
  footprint of 20 degrees half-opening between comoving distances 200 and
  625 Mpc/h with the same radial selection shape, 1.06e6 galaxies, and the
  Poisson likelihood of the power-law x sigmoid bias without the prior
  term.  coarsen() gives its 4 Mpc/h data for the first level of the
  resolution schedule.

Seeds for configuration c: truth white noise 1000c+1, counts 1000c+2, start
1000c+3, counter-generator key 1000c+4.  White noise is drawn in FP64,
rounded to FP32 and widened back, so FP32 and FP64 consumers see the same
values.
"""
import math

import numpy as np

__all__ = ["CONFIGS", "config", "white_noise", "response_field", "nbar_for",
           "poisson_counts", "seeds", "coarsen"]

_COMMON = dict(a_init=0.1, a_final=1.0, omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8,
               bias=1.5, r_min=1e-3, prior_weight=1.0, observer=(0.0, 0.0, 0.0),
               lbfgs_m=10, eps_max=1.0, armijo_c1=1e-4, max_trials=30, s_th=10.0,
               rom_nbins=100, rom_kmin=0.1)

# c6 observer: the box centre (250, 250, 250) lies 400 Mpc/h away along (1,1,1)/sqrt(3)
_OBS6 = 250.0 - 400.0 / math.sqrt(3.0)

CONFIGS = {
    1: dict(_COMMON, n_part=32, n_mesh=32, box=256.0, n_steps=5, rsd="z",
            geometry="halfbox", galaxies=None, nbar=1.0, rom_every=5, iterations=20),
    2: dict(_COMMON, n_part=128, n_mesh=128, box=512.0, n_steps=10, rsd="radial",
            geometry="cone", galaxies=1.0e6, rom_every=20, iterations=50),
    3: dict(_COMMON, n_part=256, n_mesh=256, box=1000.0, n_steps=10, rsd="radial",
            geometry="cone", galaxies=8.0e6, rom_every=20, iterations=200),
    4: dict(_COMMON, n_part=256, n_mesh=512, box=1000.0, n_steps=20, rsd="radial",
            geometry="cone", galaxies=8.0e6, rom_every=20, iterations=20),
    5: dict(_COMMON, n_part=512, n_mesh=1024, box=2000.0, n_steps=20, rsd="radial",
            geometry="cone", galaxies=None, nbar_from=3, rom_every=20, iterations=50),
    6: dict(_COMMON, n_part=256, n_mesh=256, box=500.0, n_steps=18, omega_m=0.315, h=0.673,
            sigma8=0.829, rsd="radial", geometry="disk", galaxies=1.06e6, loss="poisson",
            prior_weight=0.0, observer=(_OBS6, _OBS6, _OBS6), rom_every=20, iterations=3600,
            low_rom_every=5, low_iterations=250),
}


def config(c, **overrides):
    """A copy of configuration c with overrides applied."""
    cfg = dict(CONFIGS[c])
    cfg["id"] = c
    cfg["seed"] = seeds(c)["key"]
    cfg.update(overrides)
    return cfg


def seeds(c):
    return dict(truth=1000 * c + 1, counts=1000 * c + 2, start=1000 * c + 3,
                key=1000 * c + 4)


def white_noise(n, seed):
    """N(0,1) field of shape (n, n, n) from PCG64(seed), FP32-representable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)


def _cone_inside(y):
    """40 x 40 degree gnomonic square centred on (1,1,1)/sqrt(3)."""
    n0 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    e1 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
    e2 = np.array([1.0, 1.0, -2.0]) / math.sqrt(6.0)
    t = math.tan(math.radians(20.0))
    c0 = np.tensordot(n0, y, axes=1)
    c1 = np.tensordot(e1, y, axes=1)
    c2 = np.tensordot(e2, y, axes=1)
    return (c0 > 0) & (np.abs(c1) <= t * c0) & (np.abs(c2) <= t * c0)


def _disk_inside(y, r):
    """Circular footprint of 20 degrees half-opening around (1,1,1)/sqrt(3),
    comoving distance between 200 and 625 Mpc/h."""
    c0 = np.tensordot(np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0), y, axes=1)
    return (c0 >= math.cos(math.radians(20.0)) * r) & (r >= 200.0) & (r <= 625.0)


def response_field(cfg):
    """Survey response R on the data grid (N_p^3), FP32-representable.

    Nodes sit at c * (L / N_p).  'halfbox': R = 1 where x < L/2.  'cone' and
    'disk': R = exp(-(r/300)^1.5) inside the footprint seen from the observer
    (nodes of the box only: no periodic images)."""
    n, L = cfg["n_part"], cfg["box"]
    x = np.arange(n, dtype=np.float64) * (L / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    if cfg["geometry"] == "halfbox":
        R = (X < 0.5 * L).astype(np.float64)
    else:
        obs = np.asarray(cfg["observer"], dtype=np.float64)
        y = np.stack([X - obs[0], Y - obs[1], Z - obs[2]])
        r = np.sqrt(np.sum(y * y, axis=0))
        inside = _cone_inside(y) if cfg["geometry"] == "cone" else _disk_inside(y, r)
        R = np.where(inside, np.exp(-(r / 300.0) ** 1.5), 0.0)
    return R.astype(np.float32).astype(np.float64)


def coarsen(counts, R):
    """Data of a grid of half the side: counts summed and the response
    averaged over each 2 x 2 x 2 group of cells (cells 2c and 2c+1 along each
    axis), FP32-representable.  Integer counts stay integers; the coarse node
    2c sits half a fine cell below the centre of its group."""
    n = counts.shape[0] // 2
    c = np.asarray(counts, dtype=np.int64).reshape(n, 2, n, 2, n, 2).sum(axis=(1, 3, 5))
    r = np.asarray(R, dtype=np.float64).reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))
    return c.astype(np.int32), r.astype(np.float32).astype(np.float64)


def nbar_for(cfg, R=None):
    """Mean galaxies per cell so that sum over masked cells of Nbar R equals
    the target count (1 for the half box)."""
    if cfg.get("galaxies") is None and "nbar_from" in cfg:
        return nbar_for(config(cfg["nbar_from"]))
    if cfg.get("galaxies") is None:
        return float(cfg.get("nbar", 1.0))
    if R is None:
        R = response_field(cfg)
    m = R >= cfg["r_min"]
    return float(cfg["galaxies"] / np.sum(R[m]))


def poisson_counts(lam, R, r_min, seed):
    """N ~ Poisson(max(lambda, 0)) on masked cells, 0 elsewhere, int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
    counts = rng.poisson(lam)
    counts[np.asarray(R) < r_min] = 0
    return counts.astype(np.int32)
