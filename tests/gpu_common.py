"""Shared helpers of the GPU parity tests: contexts on cuda:0 and oracle models
built from the same seeded synthetic inputs."""
import functools

import numpy as np
import pytest

from oracle.model import Model, Problem
from paper_2604_26823_amd import inputs

torch = pytest.importorskip("torch")

DEV = "cuda:0"


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dt(prec):
    return torch.float32 if prec == "f32" else torch.float64


def np_dt(prec):
    return np.float32 if prec == "f32" else np.float64


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cfg_small(c=1, **kw):
    return inputs.config(c, **kw)


@functools.lru_cache(maxsize=None)
def _context(key, prec):
    from paper_2604_26823_amd.api import Context
    cfg = dict(key)
    cfg["observer"] = tuple(cfg.get("observer", (0.0, 0.0, 0.0)))
    return Context(cfg, prec, DEV)


def context(cfg, prec):
    key = tuple(sorted((k, v) for k, v in cfg.items() if not isinstance(v, (dict, list))))
    return _context(key, prec)


@functools.lru_cache(maxsize=None)
def _model(key):
    cfg = dict(key)
    fields = {k: cfg[k] for k in Problem.__dataclass_fields__ if k in cfg}
    return Model(Problem(**fields))


def model(cfg):
    key = tuple(sorted((k, v) for k, v in cfg.items() if not isinstance(v, (dict, list))))
    return _model(key)


def observation(cfg, mdl):
    """Response, counts (truth from the oracle) and the start field."""
    sd = inputs.seeds(cfg["id"])
    R = inputs.response_field(cfg)
    s_true = inputs.white_noise(cfg["n_part"], sd["truth"])
    lam = mdl.observe(mdl.forward(s_true), R)
    N = inputs.poisson_counts(lam, R, cfg["r_min"], sd["counts"])
    s0 = inputs.white_noise(cfg["n_part"], sd["start"])
    return R, N, s0


def to_dev(x, prec):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt(prec), device=DEV)


def to_np(t):
    return t.detach().double().cpu().numpy()
