"""White-noise upsampling between the levels of the resolution schedule (GPU)
against the oracle: every element of the fine field on the same coarse input,
seed and event, from 16^3 -> 32^3 up to the schedule's 128^3 -> 256^3, plus
the argument checks of the entry point.

Tolerance: relative L2 over the fine field.  The fresh draws are Philox
normals rounded to the working precision and the field goes through one
forward and one inverse 3D transform (~log2(N^3) roundings each), so FP32
sits near 1e-7 and FP64 near 1e-15."""
import functools

import numpy as np
import pytest

from gpu_common import DEV, rel_l2, require_gpu, to_np, torch
from oracle import upsample
from paper_2604_26823_amd import _lib, inputs
from paper_2604_26823_amd.api import Context

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-6, "f64": 1e-12}
BOX = 500.0


def _cfg(n):
    return inputs.config(1, n_part=n, n_mesh=n, box=BOX, n_steps=1, tape_forces=0, lbfgs_m=1)


@functools.lru_cache(maxsize=None)
def _reference(n_low, event):
    s_low = inputs.white_noise(n_low, 100 + n_low)
    seed = _cfg(2 * n_low)["seed"]
    return s_low, upsample.upsample(s_low.astype(np.float64), 2 * n_low, seed, event)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n_low,event", [(16, 0), (32, 3), (64, 1), (128, 2)])
def test_upsampled_field_matches_oracle(n_low, event, prec):
    require_gpu()
    s_low, ref = _reference(n_low, event)
    low = Context(_cfg(n_low), prec, DEV)
    high = Context(_cfg(2 * n_low), prec, DEV)
    try:
        sl = torch.tensor(s_low, dtype=low.dtype, device=DEV)
        got = to_np(high.upsample_from(low, sl, event))
        # the coarse field is read only
        assert torch.equal(sl, torch.tensor(s_low, dtype=low.dtype, device=DEV))
    finally:
        high.close()
        low.close()
    err = rel_l2(got, ref)
    print("upsample %d -> %d %s: rel L2 %.3e, std %.4f" % (n_low, 2 * n_low, prec, err,
                                                          got.std()))
    assert err <= TOL[prec]
    assert abs(got.std() - 1.0) < 0.05


def test_upsample_argument_checks():
    require_gpu()
    a32 = Context(_cfg(16), "f32", DEV)
    b32 = Context(_cfg(32), "f32", DEV)
    b64 = Context(_cfg(32), "f64", DEV)
    other_box = Context(dict(_cfg(32), box=2 * BOX), "f32", DEV)
    try:
        s = torch.zeros(a32.grid, dtype=torch.float32, device=DEV)
        with pytest.raises(_lib.IcError):
            b64.upsample_from(a32, s, 0)           # precision differs
        with pytest.raises(_lib.IcError):
            a32.upsample_from(a32, s, 0)           # same context
        with pytest.raises(_lib.IcError):
            other_box.upsample_from(a32, s, 0)     # box differs
        s32 = torch.zeros(b32.grid, dtype=torch.float32, device=DEV)
        with pytest.raises(_lib.IcError):
            a32.upsample_from(b32, s32, 0)         # coarse grid larger
        out = b32.upsample_from(a32, s, 5)         # zero coarse field: fresh noise, band cleared
        z = torch.fft.rfftn(out.double())
        assert float(z[:7, :7, :7].abs().max()) < 1e-3
        assert float(z[9:, 9:, 9:].abs().max()) > 1.0
    finally:
        for c in (a32, b32, b64, other_box):
            c.close()
