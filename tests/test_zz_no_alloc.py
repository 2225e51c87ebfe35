"""The sort entry point for callers that cannot allocate (ic_op_sort_desc_noalloc)
against the context's own sort (ic_op_sort_desc) and the oracle's stable
descending order (GPU).

Three calls in a row on the same device, so the second and third find the
previous call's contents in the shared array: the largest accepted length
(2^21), then two shorter ones, each with ties and signed zeros.  The orders
must be identical (bit-exact integer output); an oversized length and a NaN
are refused with their error codes and leave the output untouched."""
import ctypes

import numpy as np
import pytest

from gpu_common import DEV, cfg_small, context, require_gpu, torch
from oracle import rom
from paper_2604_26823_amd import _lib

pytestmark = pytest.mark.gpu

MAX_N = 1 << 21


def _values(n, seed, prec):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v[::7] = np.round(v[::7], 1)  # ties
    v[3::11] = 0.0
    v[5::13] = -0.0
    dt = torch.float32 if prec == "f32" else torch.float64
    return torch.tensor(v, dtype=dt, device=DEV)


def _sort(lib, prec, x, n=None):
    n = x.numel() if n is None else n
    out = torch.full((max(n, 1),), -7, dtype=torch.int32, device=DEV)
    code = _lib.IC_F32 if prec == "f32" else _lib.IC_F64
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.ic_op_sort_desc_noalloc(code, ctypes.c_void_p(x.data_ptr()), ctypes.c_int64(n),
                                     ctypes.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    return rc, out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_sort_matches_the_context_sort(prec):
    require_gpu()
    lib = _lib.load()
    ctx = context(cfg_small(1, n_part=64, n_mesh=64, box=512.0), prec)  # sorts up to 64^3
    x = _values(MAX_N, 1, prec)
    rc, got = _sort(lib, prec, x)
    assert rc == _lib.IC_OK
    ref = rom.descending_order(x.double().cpu().numpy())
    assert np.array_equal(got.cpu().numpy(), ref)
    for n, seed in ((200_003, 2), (50_001, 3)):
        x = _values(n, seed, prec)
        rc, got = _sort(lib, prec, x)
        assert rc == _lib.IC_OK
        assert torch.equal(got, ctx.sort_desc(x))
        assert np.array_equal(got.cpu().numpy(), rom.descending_order(x.double().cpu().numpy()))
    # refused: longer than the array holds; a NaN (output untouched)
    big = torch.zeros(MAX_N + 1, dtype=x.dtype, device=DEV)
    rc, out = _sort(lib, prec, big)
    assert rc == -1 and bool((out == -7).all())
    assert b"IC_NOALLOC_SORT_MAX" in lib.ic_last_error(None)
    x[17] = float("nan")
    rc, out = _sort(lib, prec, x)
    assert rc == -5 and bool((out == -7).all())
    rc, _ = _sort(lib, prec, x, n=0)
    assert rc == _lib.IC_OK
