"""The parameters the paper fixes are the defaults of the oracle, the synthetic
workloads and the library header (golden values in tests/golden/)."""
import inspect
import os
import re

from oracle import lbfgs, rom
from paper_2604_26823_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def golden():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_parameters.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, value = line.split()[:2]
                out[name] = float(value)
    return out


def test_oracle_and_workload_defaults():
    g = golden()
    sig = inspect.signature(lbfgs.ProjectedLBFGS.__init__).parameters
    assert sig["s_th"].default == g["s_th"]
    assert sig["eps_max"].default == g["eps_max"]
    fsig = inspect.signature(rom.rom_fourier).parameters
    assert fsig["k_min"].default == g["rom_kmin"]
    assert fsig["n_bins"].default == g["rom_nbins"]
    for c in (2, 3, 5):
        cfg = inputs.config(c)
        assert cfg["rom_every"] == g["rom_every"]
        assert cfg["a_init"] == g["a_init"] and cfg["a_final"] == g["a_final"]
        assert cfg["s_th"] == g["s_th"] and cfg["eps_max"] == g["eps_max"]
        assert cfg["rom_nbins"] == g["rom_nbins"] and cfg["rom_kmin"] == g["rom_kmin"]
    assert inputs.config(1)["rom_every"] == g["rom_every_lowres"]


def test_library_header_defaults():
    g = golden()
    with open(os.path.join(ROOT, "include", "ic_api.h")) as f:
        text = f.read()
    def define(name):
        m = re.search(r"#define\s+%s\s+([0-9.eE+-]+)" % name, text)
        assert m, name
        return float(m.group(1))
    assert define("IC_DEFAULT_S_TH") == g["s_th"]
    assert define("IC_DEFAULT_ROM_NBINS") == g["rom_nbins"]
    assert define("IC_DEFAULT_ROM_KMIN") == g["rom_kmin"]
    assert define("IC_DEFAULT_A_INIT") == g["a_init"]
    assert define("IC_DEFAULT_EPS_MAX") == g["eps_max"]
