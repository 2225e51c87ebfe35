"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
validates problems, sizes workspaces and computes the same FP64 cosmology
coefficients as the oracle.  No device work is started here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import cosmology
from paper_2604_26823_amd import _lib, api, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2604_26823_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    names = []
    for h in ("ic_api.h", "ic_ops.h"):
        with open(os.path.join(ROOT, "include", h)) as f:
            text = f.read()
        names += re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(ic_\w+)\s*\(", text, re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_abi_version_and_defaults(lib):
    assert lib.ic_abi_version() == 6
    p = _lib.IcProblem()
    lib.ic_problem_defaults(ctypes.byref(p))
    assert p.s_th == 10.0 and p.rom_nbins == 100 and p.rom_kmin == 0.1
    assert p.eps_max == 1.0 and p.a_init == 0.1 and p.lbfgs_m == 10


def _size(lib, cfg, prec=_lib.IC_F32):
    p = api.make_problem(cfg)
    size = ctypes.c_size_t()
    rc = lib.ic_workspace_size(ctypes.byref(p), prec, ctypes.byref(size))
    return rc, size.value


def test_workspace_sizes_and_validation(lib):
    rc, b32 = _size(lib, inputs.config(3))
    assert rc == 0
    rc, b64 = _size(lib, inputs.config(3), _lib.IC_F64)
    # field buffers double; the 32-bit particle orders (ids, destinations,
    # block keys) do not
    assert rc == 0 and 1.6 < b64 / b32 < 2.1
    # 256^3 FP32 fits comfortably in one MI355X's 288 GB
    assert 4e9 < b32 < 2e10
    for bad in [dict(n_part=48), dict(n_part=1024, n_mesh=1024), dict(n_mesh=96)]:
        cfg = inputs.config(1, **bad)
        rc, _ = _size(lib, cfg)
        assert rc == -2, bad
        assert b"n_" in lib.ic_last_error(None)
    rc, _ = _size(lib, inputs.config(1, n_steps=0))
    assert rc == -1
    rc, _ = _size(lib, inputs.config(1), 7)
    assert rc == -1
    rc, _ = _size(lib, inputs.config(1, ckpt_every=-1))
    assert rc == -1
    p = api.make_problem(inputs.config(1))
    assert p.loss_kind == 0 and (p.bias_alpha, p.bias_delta_th, p.bias_k) == (0.7, 1.2, 3.0)
    assert p.project_steps == 1
    p.loss_kind = 2
    size = ctypes.c_size_t()
    assert lib.ic_workspace_size(ctypes.byref(p), _lib.IC_F32, ctypes.byref(size)) == -1
    p.loss_kind = 1
    p.bias_k = 0.0
    assert lib.ic_workspace_size(ctypes.byref(p), _lib.IC_F32, ctypes.byref(size)) == -1
    # lightcone: snapshots ascend, sit on interior steps and end at a_final
    assert p.lc_n == 0 and p.lc_iterations == 3
    ok = dict(n_steps=18, lightcone=(0.8, 0.9, 1.0))
    for lc, rc in [((0.8, 0.9, 1.0), 0), ((1.0,), 0), ((0.9, 0.8, 1.0), -1), ((0.8, 0.9), -1),
                   ((0.82, 1.0), -1), ((0.1, 1.0), -1), ((0.4, 0.6, 0.8, 0.9, 1.0), None)]:
        cfg = inputs.config(1, **dict(ok, lightcone=lc))
        if rc is None:
            with pytest.raises(ValueError):
                api.make_problem(cfg)
            continue
        assert _size(lib, cfg)[0] == rc, lc
    assert _size(lib, inputs.config(1, **ok, lc_iterations=0))[0] == -1
    # snapshot states and their cotangents (2 x 2 x 6 fields of 4 bytes per
    # particle), the snapshot slots of the final order (2 x 4 bytes) and the table
    base = _size(lib, inputs.config(1, n_steps=18))[1]
    assert (_size(lib, inputs.config(1, **ok))[1] - base
            == (2 * 2 * 6 * 4 + 2 * 4) * 32 ** 3 + 2 * 1024 * 8)


def test_checkpoints_and_recomputed_forces_shrink_the_workspace(lib):
    # 512^3 particles on a 1024^3 mesh, 20 steps: every state and force mesh
    # taped does not fit one GPU; states every 5 steps with recomputed forces do
    full = _size(lib, inputs.config(5, tape_forces=1, ckpt_every=0))[1]
    forces = _size(lib, inputs.config(5, tape_forces=0, ckpt_every=0))[1]
    both = _size(lib, inputs.config(5, tape_forces=0, ckpt_every=5))[1]
    assert full > 288e9 > forces > both
    # one position slot (3 fields) per state dropped, one momentum slot per
    # checkpoint added: 21 states -> 5 checkpoints + 4 segment slots
    P = 512 ** 3
    assert forces - both == (21 - 9 - 5) * 3 * P * 4
    # a spacing beyond the last step keeps state 0 and replays all the others
    rc, far = _size(lib, inputs.config(1, ckpt_every=100))
    assert rc == 0 and far == _size(lib, inputs.config(1, ckpt_every=6))[1]


@pytest.mark.parametrize("om,steps", [(0.3, 5), (0.3, 10), (1.0, 4)])
def test_host_coefficients_match_oracle(lib, om, steps):
    cfg = inputs.config(1, omega_m=om, n_steps=steps)
    p = api.make_problem(cfg)
    out = (ctypes.c_double * (7 + 3 * steps))()
    assert lib.ic_host_coefficients(ctypes.byref(p), out, len(out)) == 0
    got = np.array(out[:])
    co = cosmology.fastpm_coefficients(om, 0.1, 1.0, steps)
    pk = cosmology.PowerSpectrum(om, 0.7, 0.96, 0.8)
    ref = np.concatenate([[co["D1_init"], co["f1_init"], co["D2_init"], co["f2_init"],
                           co["E_init"], co["rsd_factor"], pk.amplitude],
                          co["Dr"], co["K1"], co["K2"]])
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-10


def test_product_path_fails_loudly_without_library(tmp_path):
    with pytest.raises(_lib.NativeLibraryMissing):
        _lib.load(str(tmp_path / "missing.so"))


def test_deterministic_mode_field(lib):
    """ic_problem.deterministic: 0 by default, 0 or 1 accepted, and the mode
    adds to the workspace its integer paint fields (three mesh fields of 8
    bytes per cell), their z halo (one value per 8 cells), their x/y halo
    staging (153 cells of three fields per work item of the mesh orders,
    items = ceil(n^3 / 1024) + (n / 8)^3) and eight doubles (a 256-byte
    block)."""
    p = api.make_problem(inputs.config(1))
    assert p.deterministic == 0
    n = 32
    items = -(-n ** 3 // 1024) + (n // 8) ** 3
    base = _size(lib, inputs.config(1))[1]
    rc, det = _size(lib, inputs.config(1, deterministic=1))
    assert rc == 0
    assert det - base == 3 * 8 * n ** 3 + 3 * n ** 3 + 3 * items * 153 * 8 + 256
    p.deterministic = 2
    size = ctypes.c_size_t()
    assert lib.ic_workspace_size(ctypes.byref(p), _lib.IC_F32, ctypes.byref(size)) == -1
    assert b"deterministic" in lib.ic_last_error(None)
