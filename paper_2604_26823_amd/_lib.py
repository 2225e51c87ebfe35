"""ctypes declarations of the C ABI in include/ic_api.h and include/ic_ops.h.

Argument marshalling only: every computation happens in libic_mi355x.so.
Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libic_mi355x.so")

IC_OK = 0
IC_ERR = {
    -1: "IC_ERR_INVALID_ARG", -2: "IC_ERR_UNSUPPORTED", -3: "IC_ERR_WORKSPACE",
    -4: "IC_ERR_HIP", -5: "IC_ERR_NONFINITE", -6: "IC_ERR_LINESEARCH", -7: "IC_ERR_STATE",
}
IC_F32, IC_F64 = 0, 1
IC_RSD = {"none": 0, "z": 1, "radial": 2}
IC_PROJECT, IC_ROM_REAL, IC_ROM_FOURIER, IC_ROM_FOURIER_REIM = 1, 2, 4, 8
IC_GRID_PART, IC_GRID_MESH = 0, 1
IC_MULT_WHITE, IC_MULT_GRAD, IC_MULT_HESS = 1, 2, 4

EXPORTS = [
    "ic_abi_version", "ic_problem_defaults", "ic_workspace_size", "ic_create", "ic_destroy",
    "ic_last_error", "ic_set_stream", "ic_set_observation", "ic_forward", "ic_loss_and_grad",
    "ic_vjp", "ic_project_rankmatch", "ic_lbfgs_step", "ic_lbfgs_reset", "ic_upsample_noise",
    "ic_op_rfft", "ic_op_irfft", "ic_op_multiplier", "ic_op_paint", "ic_op_force", "ic_op_lpt",
    "ic_op_evolve", "ic_op_sort_desc", "ic_op_sort_desc_noalloc", "ic_op_philox", "ic_debug_rom_order", "ic_timing",
    "ic_timing_only", "ic_timing_report", "ic_host_coefficients",
]


class IcProblem(ctypes.Structure):
    _fields_ = [
        ("n_part", ctypes.c_int32), ("n_mesh", ctypes.c_int32), ("n_steps", ctypes.c_int32),
        ("rsd_mode", ctypes.c_int32), ("box", ctypes.c_double), ("a_init", ctypes.c_double),
        ("a_final", ctypes.c_double), ("omega_m", ctypes.c_double), ("h", ctypes.c_double),
        ("n_s", ctypes.c_double), ("sigma8", ctypes.c_double),
        ("observer", ctypes.c_double * 3), ("bias", ctypes.c_double),
        ("nbar", ctypes.c_double), ("r_min", ctypes.c_double),
        ("prior_weight", ctypes.c_double), ("lbfgs_m", ctypes.c_int32),
        ("max_trials", ctypes.c_int32), ("eps_max", ctypes.c_double),
        ("armijo_c1", ctypes.c_double), ("s_th", ctypes.c_double),
        ("rom_nbins", ctypes.c_int32), ("tape_forces", ctypes.c_int32),
        ("ckpt_every", ctypes.c_int32),
        ("rom_kmin", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("bias_alpha", ctypes.c_double), ("bias_delta_th", ctypes.c_double),
        ("bias_k", ctypes.c_double), ("loss_kind", ctypes.c_int32),
        ("project_steps", ctypes.c_int32), ("lc_n", ctypes.c_int32),
        ("lc_iterations", ctypes.c_int32), ("lc_a", ctypes.c_double * 4),
        ("deterministic", ctypes.c_int32),
    ]


class IcLossTerms(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("chi2", ctypes.c_double),
                ("prior", ctypes.c_double), ("n_masked", ctypes.c_int64)]


class IcLbfgsInfo(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("gp", ctypes.c_double),
                ("trials", ctypes.c_int32), ("evaluations", ctypes.c_int32),
                ("stored", ctypes.c_int32), ("history", ctypes.c_int32),
                ("restarted", ctypes.c_int32), ("resets", ctypes.c_int32)]


class IcRomInfo(ctypes.Structure):
    _fields_ = [("n_real", ctypes.c_int64), ("n_fourier", ctypes.c_int64),
                ("resets", ctypes.c_int32), ("bins_used", ctypes.c_int32)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "ic_abi_version": (ctypes.c_int32, []),
    "ic_problem_defaults": (None, [ctypes.POINTER(IcProblem)]),
    "ic_workspace_size": (_I, [ctypes.POINTER(IcProblem), _I, ctypes.POINTER(ctypes.c_size_t)]),
    "ic_create": (_I, [ctypes.POINTER(IcProblem), _I, _P, ctypes.c_size_t, _P,
                       ctypes.POINTER(_P)]),
    "ic_destroy": (None, [_P]),
    "ic_last_error": (ctypes.c_char_p, [_P]),
    "ic_set_stream": (_I, [_P, _P]),
    "ic_set_observation": (_I, [_P, _P, _P]),
    "ic_forward": (_I, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "ic_loss_and_grad": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(IcLossTerms)]),
    "ic_vjp": (_I, [_P, _P, _P, _P]),
    "ic_project_rankmatch": (_I, [_P, _P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                  ctypes.POINTER(IcRomInfo)]),
    "ic_lbfgs_step": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                           ctypes.POINTER(IcLbfgsInfo)]),
    "ic_lbfgs_reset": (_I, [_P]),
    "ic_upsample_noise": (_I, [_P, _P, _P, _P, ctypes.c_uint64]),
    "ic_op_rfft": (_I, [_P, _I, _P, _P]),
    "ic_op_irfft": (_I, [_P, _I, _P, _P]),
    "ic_op_multiplier": (_I, [_P, _I, _I, _I, _P, _P]),
    "ic_op_paint": (_I, [_P, _I, _P, _P]),
    "ic_op_force": (_I, [_P, _P, _P]),
    "ic_op_lpt": (_I, [_P, _P, _P, _P]),
    "ic_op_evolve": (_I, [_P, _P, _P, _P]),
    "ic_op_sort_desc": (_I, [_P, _P, ctypes.c_int64, _P]),
    "ic_op_sort_desc_noalloc": (_I, [_I, _P, ctypes.c_int64, _P, _P]),
    "ic_op_philox": (_I, [_P, _I, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_int64, _P]),
    "ic_debug_rom_order": (_I, [_P, _I, _P, _P, _P, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64)]),
    "ic_host_coefficients": (_I, [ctypes.POINTER(IcProblem), ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_size_t]),
    "ic_timing": (_I, [_P, _I]),
    "ic_timing_only": (_I, [_P, ctypes.c_char_p]),
    "ic_timing_report": (_I, [_P, ctypes.c_char_p, ctypes.c_size_t]),
}

_LIB = None


class NativeLibraryMissing(RuntimeError):
    pass


def load(path=None):
    """Loads the HIP library (no fallback: raises when it is missing)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise NativeLibraryMissing(
            "libic_mi355x.so not built; run `python -m paper_2604_26823_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


class IcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (IC_ERR.get(code, "IC_ERR"), code, msg))
        self.code = code
