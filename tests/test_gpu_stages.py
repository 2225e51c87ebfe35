"""Stage-by-stage parity of the HIP path against the FP64 oracle (GPU).

Every check calls the library through its C ABI (via the ctypes binding) on
seeded inputs and compares element by element with the oracle on the same
values.  Tolerances: FP64 near machine precision; FP32 a few units of the
FP32 rounding of the stage (derived in the test names' comments)."""
import numpy as np
import pytest

from gpu_common import (DEV, cfg_small, context, model, np_dt, rel_l2, require_gpu, to_dev,
                        to_np, torch)
from oracle import cic, fourier, philox, projection, rom

pytestmark = pytest.mark.gpu

PRECS = ["f32", "f64"]
# FP32: an FFT of length N accumulates ~log2(N) roundings of 6e-8 per axis.
TOL_FFT = {"f32": 3e-6, "f64": 1e-13}


def small(n, nm=None, steps=2, rsd="z", c=1, box=None):
    return cfg_small(c, n_part=n, n_mesh=nm or n, n_steps=steps, rsd=rsd, box=box or 8.0 * n)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256])
def test_rfft_matches_oracle(prec, n):
    require_gpu()
    ctx = context(small(n), prec)
    x = np.random.default_rng(n).standard_normal((n, n, n)).astype(np_dt(prec))
    got = ctx.rfft(to_dev(x, prec)).cpu().numpy()
    ref = fourier.rfft3(x.astype(np.float64))
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= TOL_FFT[prec], err


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [8, 32, 64])
def test_irfft_matches_oracle(prec, n):
    require_gpu()
    ctx = context(small(n), prec)
    x = np.random.default_rng(100 + n).standard_normal((n, n, n))
    xk = fourier.rfft3(x)
    ctype = np.complex64 if prec == "f32" else np.complex128
    got = to_np(ctx.irfft(torch.tensor(xk.astype(ctype), device=DEV)))
    ref = fourier.irfft3(xk.astype(ctype).astype(np.complex128), n)
    assert np.max(np.abs(got - ref)) <= TOL_FFT[prec] * np.max(np.abs(ref)) * 4


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", [("grad", 0), ("grad", 2), ("hess", (0, 1)), ("hess", (2, 2)),
                                  ("white", None)])
@pytest.mark.parametrize("n", [32, 256])
def test_multiplier_operators(prec, kind, n):
    """Op_m[x] = irfft(m rfft(x)) through one scatter chain; at n = 256 the
    FP32 chain runs the fused z+y passes (the packed kz = 0 / n/2 column,
    the hand radix-2 step along y)."""
    require_gpu()
    cfg = small(n)
    ctx = context(cfg, prec)
    mdl = model(cfg)
    x = np.random.default_rng(7).standard_normal((n, n, n)).astype(np_dt(prec)).astype(np.float64)
    name, axis = kind
    if name == "grad":
        bits, a, b = 2, axis, 0
    elif name == "hess":
        bits, (a, b) = 4, axis
    else:
        bits, a, b = 1, 0, 0
    got = to_np(ctx.multiplier(to_dev(x, prec), bits, a, b))
    ref = fourier.apply(mdl.mult(name, axis), x)
    assert rel_l2(got, ref) <= (5e-6 if prec == "f32" else 1e-12)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("ratio", [1, 2])
def test_paint_matches_oracle(prec, ratio):
    require_gpu()
    n = 32
    cfg = small(n, nm=ratio * n)
    ctx = context(cfg, prec)
    mdl = model(cfg)
    d = np.random.default_rng(8).normal(0, 6.0, (3, n ** 3)).astype(np_dt(prec)).astype(np.float64)
    for grid, cells, cell in [(0, n, mdl.dq), (1, ratio * n, mdl.dm)]:
        got = to_np(ctx.paint(to_dev(d, prec), grid))
        ref = cic.paint(mdl.q + d, cells, cell)
        assert abs(got.sum() - n ** 3) <= (2e-6 if prec == "f32" else 1e-10) * n ** 3
        assert np.max(np.abs(got - ref)) <= (2e-5 if prec == "f32" else 1e-11)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("ratio", [1, 2])
def test_force_matches_oracle(prec, ratio):
    require_gpu()
    n = 32
    cfg = small(n, nm=ratio * n)
    ctx = context(cfg, prec)
    mdl = model(cfg)
    d = np.random.default_rng(9).normal(0, 4.0, (3, n ** 3)).astype(np_dt(prec)).astype(np.float64)
    got = to_np(ctx.force(to_dev(d, prec)))
    ref, _ = mdl.force(d)
    assert rel_l2(got, ref) <= (2e-5 if prec == "f32" else 1e-11)


@pytest.mark.parametrize("prec", PRECS)
def test_lpt_matches_oracle(prec):
    require_gpu()
    n = 32
    cfg = small(n)
    ctx = context(cfg, prec)
    mdl = model(cfg)
    s = np.random.default_rng(10).standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    d, p = ctx.lpt(to_dev(s, prec))
    d0, p0, _ = mdl.lpt(s)
    tol = 5e-6 if prec == "f32" else 1e-12
    assert rel_l2(to_np(d), d0) <= tol
    assert rel_l2(to_np(p), p0) <= tol


@pytest.mark.parametrize("prec", PRECS)
def test_philox_draws_match_oracle(prec):
    require_gpu()
    ctx = context(small(16), prec)
    seed = ctx.problem.seed
    n = 5000
    j = np.arange(n, dtype=np.uint64)
    for kind, fn in [(0, philox.normal), (1, philox.rayleigh)]:
        got = to_np(ctx.philox(kind, 3, 2, 11, n))
        ref = fn(j, 3, 2, 11, seed)
        tol = 2e-7 if prec == "f32" else 1e-14
        assert np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))) <= tol


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 7, 4096, 4097, 100000])
def test_sort_desc_is_stable_argsort(prec, n):
    require_gpu()
    ctx = context(small(64), prec)
    rng = np.random.default_rng(n)
    v = rng.integers(-20, 20, n).astype(np_dt(prec)) * np_dt(prec)(0.25)
    v[rng.integers(0, n, max(1, n // 10))] = -0.0
    order = ctx.sort_desc(torch.tensor(v, device=DEV)).cpu().numpy()
    assert np.array_equal(order, rom.descending_order(v.astype(np.float64)))


@pytest.mark.parametrize("prec", PRECS)
def test_projection_matches_oracle(prec):
    require_gpu()
    n = 16
    ctx = context(small(n), prec)
    seed = ctx.problem.seed
    s = np.random.default_rng(11).normal(0.2, 1.7, (n, n, n)).astype(np_dt(prec))
    s[1, 2, 3] = 60.0
    s[5, 5, 5] = -55.0
    t = to_dev(s, prec)
    info = ctx.project_rankmatch(t, 1, event=4, trial=2)
    ref, nres = projection.project(s.astype(np.float64), 10.0, seed, 4, 2)
    assert info["resets"] == nres == 2
    assert np.max(np.abs(to_np(t) - ref)) <= (4e-7 if prec == "f32" else 1e-14)
