"""Python binding of the hot-path library with PyTorch device memory.

``Context`` owns one library context and its workspace (a torch uint8
tensor); every method marshals tensor pointers into the C ABI of
include/ic_api.h and include/ic_ops.h on the current torch stream.  No step
of the path runs in Python or PyTorch.
"""
import ctypes

import torch

from . import _lib
from ._lib import IcLbfgsInfo, IcLossTerms, IcProblem, IcRomInfo

PROBLEM_KEYS = ["n_part", "n_mesh", "n_steps", "box", "a_init", "a_final", "omega_m", "h",
                "n_s", "sigma8", "bias", "nbar", "r_min", "prior_weight", "lbfgs_m",
                "max_trials", "eps_max", "armijo_c1", "s_th", "rom_nbins", "tape_forces", "ckpt_every",
                "rom_kmin", "seed", "bias_alpha", "bias_delta_th", "bias_k", "project_steps",
                "deterministic"]


def make_problem(cfg):
    """ic_problem from a dict (keys of ic_problem; rsd as 'none'|'z'|'radial')."""
    lib = _lib.load()
    p = IcProblem()
    lib.ic_problem_defaults(ctypes.byref(p))
    for k in PROBLEM_KEYS:
        if k in cfg and cfg[k] is not None:
            setattr(p, k, type(getattr(p, k))(cfg[k]))
    if "rsd" in cfg:
        p.rsd_mode = _lib.IC_RSD[cfg["rsd"]]
    if "loss" in cfg:
        p.loss_kind = {"gauss": 0, "poisson": 1}[cfg["loss"]]
    if "observer" in cfg:
        for a in range(3):
            p.observer[a] = float(cfg["observer"][a])
    lc = cfg.get("lightcone") or ()
    if len(lc) > 4:
        raise ValueError("at most 4 lightcone snapshots")
    p.lc_n = len(lc)
    for j, a in enumerate(lc):
        p.lc_a[j] = float(a)
    if cfg.get("lc_iterations") is not None:
        p.lc_iterations = int(cfg["lc_iterations"])
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """One library context on one device, FP32 or FP64."""

    def __init__(self, cfg, precision="f32", device="cuda"):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the hot-path library needs a GPU")
        self.cfg = dict(cfg)
        self.device = torch.device(device)
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self.prec = _lib.IC_F32 if precision == "f32" else _lib.IC_F64
        self.problem = make_problem(cfg)
        self.n = self.problem.n_part
        self.nm = self.problem.n_mesh
        size = ctypes.c_size_t()
        self._check(self.lib.ic_workspace_size(ctypes.byref(self.problem), self.prec,
                                               ctypes.byref(size)), None)
        self.ws_bytes = size.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        ctx = ctypes.c_void_p()
        self._check(self.lib.ic_create(ctypes.byref(self.problem), self.prec,
                                       ctypes.c_void_p(aligned), ctypes.c_size_t(self.ws_bytes),
                                       self._stream(), ctypes.byref(ctx)), None)
        self.ctx = ctx
        self._obs = None

    # --------------------------------------------------------------- plumbing
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc, ctx="self"):
        if rc != _lib.IC_OK:
            c = self.ctx if ctx == "self" else None
            msg = self.lib.ic_last_error(c)
            raise _lib.IcError(rc, msg.decode() if msg else "")

    def _sync_stream(self):
        self._check(self.lib.ic_set_stream(self.ctx, self._stream()))

    def _field(self, t, shape=None, dtype=None):
        dtype = dtype or self.dtype
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous():
            raise ValueError("expected a contiguous %s tensor on %s" % (dtype, self.device))
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
        return t

    def empty(self, *shape, dtype=None):
        return torch.empty(*shape, dtype=dtype or self.dtype, device=self.device)

    @property
    def grid(self):
        return (self.n, self.n, self.n)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ API
    def set_observation(self, counts, response):
        self._field(counts, self.grid, torch.int32)
        self._field(response, self.grid)
        self._obs = (counts, response)  # keep alive
        self._check(self.lib.ic_set_observation(self.ctx, _ptr(counts), _ptr(response)))

    def forward(self, s, delta=True, lam=False, loss=False):
        self._sync_stream()
        self._field(s, self.grid)
        d = self.empty(*self.grid) if delta else None
        l = self.empty(*self.grid) if lam else None
        L = ctypes.c_double()
        self._check(self.lib.ic_forward(self.ctx, _ptr(s), _ptr(d), _ptr(l),
                                        ctypes.byref(L) if loss else None))
        out = {}
        if delta:
            out["delta"] = d
        if lam:
            out["lambda"] = l
        if loss:
            out["loss"] = L.value
        return out

    def loss_and_grad(self, s, grad=None):
        self._sync_stream()
        self._field(s, self.grid)
        g = grad if grad is not None else self.empty(*self.grid)
        L = ctypes.c_double()
        t = IcLossTerms()
        self._check(self.lib.ic_loss_and_grad(self.ctx, _ptr(s), _ptr(g), ctypes.byref(L),
                                              ctypes.byref(t)))
        return L.value, g, dict(loss=t.loss, chi2=t.chi2, prior=t.prior, n_masked=t.n_masked)

    def vjp(self, s, delta_bar):
        self._sync_stream()
        self._field(s, self.grid)
        self._field(delta_bar, self.grid)
        out = self.empty(*self.grid)
        self._check(self.lib.ic_vjp(self.ctx, _ptr(s), _ptr(delta_bar), _ptr(out)))
        return out

    def project_rankmatch(self, s, flags, event, trial=0):
        self._sync_stream()
        self._field(s, self.grid)
        info = IcRomInfo()
        self._check(self.lib.ic_project_rankmatch(self.ctx, _ptr(s), ctypes.c_uint32(flags),
                                                  ctypes.c_uint64(event), ctypes.c_int32(trial),
                                                  ctypes.byref(info)))
        return dict(n_real=info.n_real, n_fourier=info.n_fourier, resets=info.resets,
                    bins_used=info.bins_used)

    def lbfgs_step(self, s, grad, loss, iteration):
        self._sync_stream()
        self._field(s, self.grid)
        self._field(grad, self.grid)
        L = ctypes.c_double(loss)
        info = IcLbfgsInfo()
        rc = self.lib.ic_lbfgs_step(self.ctx, _ptr(s), _ptr(grad), ctypes.byref(L),
                                    ctypes.c_int64(iteration), ctypes.byref(info))
        self._check(rc)
        return L.value, dict(eps=info.eps, gp=info.gp, trials=info.trials,
                             evaluations=info.evaluations, stored=info.stored,
                             history=info.history, restarted=info.restarted, resets=info.resets)

    def lbfgs_reset(self):
        self._check(self.lib.ic_lbfgs_reset(self.ctx))

    def upsample_from(self, low, s_low, event):
        """White noise on this context's grid carrying the large-scale modes of
        s_low, a field of the coarse context low (half the grid side)."""
        self._sync_stream()
        low._field(s_low, low.grid)
        out = self.empty(*self.grid)
        self._check(self.lib.ic_upsample_noise(self.ctx, low.ctx, _ptr(s_low), _ptr(out),
                                               ctypes.c_uint64(event)))
        return out

    # ---------------------------------------------------------- single stages
    def rfft(self, x, grid=_lib.IC_GRID_PART):
        self._sync_stream()
        n = self.n if grid == _lib.IC_GRID_PART else self.nm
        self._field(x, (n, n, n))
        ctype = torch.complex64 if self.dtype == torch.float32 else torch.complex128
        out = torch.empty((n, n, n // 2 + 1), dtype=ctype, device=self.device)
        self._check(self.lib.ic_op_rfft(self.ctx, grid, _ptr(x), _ptr(out)))
        return out

    def irfft(self, xk, grid=_lib.IC_GRID_PART):
        self._sync_stream()
        n = self.n if grid == _lib.IC_GRID_PART else self.nm
        if not xk.is_contiguous() or tuple(xk.shape) != (n, n, n // 2 + 1):
            raise ValueError("bad half spectrum")
        out = self.empty(n, n, n)
        self._check(self.lib.ic_op_irfft(self.ctx, grid, _ptr(xk), _ptr(out)))
        return out

    def multiplier(self, x, kinds, a=0, b=0):
        self._sync_stream()
        self._field(x, self.grid)
        out = self.empty(*self.grid)
        self._check(self.lib.ic_op_multiplier(self.ctx, kinds, a, b, _ptr(x), _ptr(out)))
        return out

    def paint(self, disp, grid=_lib.IC_GRID_PART):
        self._sync_stream()
        self._field(disp, (3, self.n ** 3))
        n = self.n if grid == _lib.IC_GRID_PART else self.nm
        out = self.empty(n, n, n)
        self._check(self.lib.ic_op_paint(self.ctx, grid, _ptr(disp), _ptr(out)))
        return out

    def force(self, disp):
        self._sync_stream()
        self._field(disp, (3, self.n ** 3))
        out = self.empty(3, self.n ** 3)
        self._check(self.lib.ic_op_force(self.ctx, _ptr(disp), _ptr(out)))
        return out

    def lpt(self, s):
        self._sync_stream()
        self._field(s, self.grid)
        d = self.empty(3, self.n ** 3)
        p = self.empty(3, self.n ** 3)
        self._check(self.lib.ic_op_lpt(self.ctx, _ptr(s), _ptr(d), _ptr(p)))
        return d, p

    def evolve(self, s):
        self._sync_stream()
        self._field(s, self.grid)
        d = self.empty(3, self.n ** 3)
        p = self.empty(3, self.n ** 3)
        self._check(self.lib.ic_op_evolve(self.ctx, _ptr(s), _ptr(d), _ptr(p)))
        return d, p

    def sort_desc(self, values):
        self._sync_stream()
        if values.dtype != self.dtype or not values.is_contiguous() or values.dim() != 1:
            raise ValueError("expected a contiguous 1-D tensor of the context dtype")
        order = torch.empty(values.numel(), dtype=torch.int32, device=self.device)
        self._check(self.lib.ic_op_sort_desc(self.ctx, _ptr(values), values.numel(),
                                             _ptr(order)))
        return order

    def philox(self, kind, sub, stream, event, n):
        self._sync_stream()
        out = self.empty(n)
        self._check(self.lib.ic_op_philox(self.ctx, kind, sub, stream, event, n, _ptr(out)))
        return out

    def rom_order(self, space):
        """(flat indices, keys, bins) of the last matching pass, in rank order."""
        import numpy as np
        n = ctypes.c_int64()
        self._check(self.lib.ic_debug_rom_order(self.ctx, space, None, None, None, 0,
                                                ctypes.byref(n)))
        cnt = n.value
        idx = np.empty(cnt, dtype=np.int32)
        keys = np.empty(cnt, dtype=np.float32 if self.dtype == torch.float32 else np.float64)
        bins = np.empty(cnt, dtype=np.int32)
        self._check(self.lib.ic_debug_rom_order(
            self.ctx, space, idx.ctypes.data_as(ctypes.c_void_p),
            keys.ctypes.data_as(ctypes.c_void_p), bins.ctypes.data_as(ctypes.c_void_p), cnt,
            ctypes.byref(n)))
        return idx, keys, bins

    def timing(self, enable):
        self._check(self.lib.ic_timing(self.ctx, 1 if enable else 0))

    def timing_only(self, kernel):
        """Record only the launches of one kernel (stop with timing(False))."""
        self._check(self.lib.ic_timing_only(self.ctx, kernel.encode()))

    def timing_report(self):
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self.lib.ic_timing_report(self.ctx, buf, len(buf)))
        rows = []
        for line in buf.value.decode().splitlines():
            name, count, ms, nbytes = line.split()
            rows.append(dict(name=name, count=int(count), ms=float(ms), bytes=float(nbytes)))
        return rows
