"""Precision and scale studies of the hot path on one GPU (this library only).

  python -m paper_2604_26823_amd.studies precision [--steps 1,2,...] [--out F]
      256^3 particles on a 512^3 force mesh, 1000 Mpc/h, 20 KDK steps, radial
      RSD and the 40x40 degree selection.  For each k the model is cut after
      step k (the same linear-in-a time grid ending at a_k, so its first k
      steps are the full run's); mock counts come from the FP64 model at a_k.
      FP32 and FP64 instantiations of the same kernels evaluate density,
      chi^2, loss and gradient at the same white noise; each record gives the
      FP32 errors relative to FP64.
  python -m paper_2604_26823_amd.studies scale [--iterations 50] [--ckpt-every 5]
          [--tape-forces 0] [--profile] [--skip-f64] [--out F]
      512^3 particles on a 1024^3 mesh, 2000 Mpc/h, 20 steps; particle states
      kept every 5 steps and replayed in the adjoint, force meshes recomputed.
      FP32: time per loss+gradient evaluation, peak device memory, then
      projected L-BFGS iterations with rank-order matching every 20.  FP64:
      one evaluation at the same start, compared with FP32.

  python -m paper_2604_26823_amd.studies ablation [--iterations 200]
          [--objective c2|paper] [--restarts] [--out F]
      The optimiser ablation of appendix B (table 1) on synthetic data of
      the 128^3, 512 Mpc/h radial-selection configuration: the method
      (projected steps, eps_max = 1, rank-order matching every 20) against
      plain L-BFGS (trial points s + eps p, no matching) with eps_max = 1,
      0.1, 0.01, 0.001.  Per run: the loss every 10 iterations, the loss of
      the homogeneous start s = 0 for reference, moments of the final white
      noise, its cross-correlation coefficient r_c(k) with the truth over the
      box, and the correlation with the truth of both fields smoothed over 4
      cells, on the cells under the mask; the losses of s = 0 and of the
      truth for reference.  --objective paper: the paper's own objective on
      its coarse level instead (c6 geometry on 128^3, 18 steps, lightcone,
      Poisson likelihood without the prior term).  --restarts adds table 1's
      last rows: plain L-BFGS (eps_max = 1) from the method's checkpoints 5,
      10 and 15 (after 100, 200, 300 iterations), run to the same total.

  python -m paper_2604_26823_amd.studies schedule [--iterations 3600]
          [--low-iterations 250] [--runs annealed,cold] [--lightcone] [--out F]
      The resolution schedule of section 3 at the paper's own scale (c6:
      Planck13, 256^3 in 500 Mpc/h, 18 steps, disk footprint, 1.06e6
      galaxies, Poisson likelihood of the power-law x sigmoid bias, no prior
      term).  'annealed': projected L-BFGS on the 4 Mpc/h data (counts
      summed over 2^3 cells) with rank-order matching every 5 iterations,
      the result upsampled to 256^3 (large-scale modes kept, fresh small
      scales), then full resolution with matching every 20.  'cold': full
      resolution from a random start.  Per run: the loss every 50
      iterations, evaluations, time, moments of the final noise, r_c(k) with
      the truth and the masked correlation of both fields smoothed over 4
      cells; the losses of s = 0 and of the truth for reference.  With
      --lightcone, both levels use the paper's snapshots (a = 0.8, 0.9, 1.0).

  python -m paper_2604_26823_amd.studies lightcone [--repeats 3] [--out F]
      c6 with the paper's snapshots (a = 0.8, 0.9, 1.0; section 2.2.1 item 3,
      appendix A) against c6 with RSD at a = 1, FP32 and FP64: time per
      loss+gradient evaluation and of the lightcone kernels, FP32 errors
      relative to FP64, and how far the lightcone moves the density.

Every output line is one JSON record (also appended to --out)."""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2604_26823_amd import _lib, inputs  # noqa: E402


def _emit(rec, out):
    line = json.dumps(rec)
    print(line, flush=True)
    if out:
        with open(out, "a") as fh:
            fh.write(line + "\n")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _timed_eval(ctx, s, g, repeats=1):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(repeats):
        L, g, terms = ctx.loss_and_grad(s, g)
    torch.cuda.synchronize()
    return L, g, terms, 1e3 * (time.perf_counter() - t) / repeats


def _observe(ctx, R, counts):
    import torch
    ctx.set_observation(torch.tensor(counts, dtype=torch.int32, device=ctx.device),
                        torch.tensor(R, dtype=ctx.dtype, device=ctx.device))


def _mock_counts(ctx, cfg, R, seed_cfg):
    """Poisson counts of the truth white noise through ctx's forward model."""
    import torch
    sd = inputs.seeds(seed_cfg)
    s_true = torch.tensor(inputs.white_noise(cfg["n_part"], sd["truth"]), dtype=ctx.dtype,
                          device=ctx.device)
    _observe(ctx, R, np.zeros(R.shape, dtype=np.int32))
    lam = ctx.forward(s_true, delta=False, lam=True)["lambda"].double().cpu().numpy()
    return inputs.poisson_counts(lam, R, cfg["r_min"], sd["counts"])


def precision(a):
    import torch

    from paper_2604_26823_amd.api import Context
    base = inputs.config(4)
    R = inputs.response_field(base)
    base["nbar"] = inputs.nbar_for(base, R)
    s0 = inputs.white_noise(base["n_part"], inputs.seeds(4)["start"])
    steps = [int(k) for k in a.steps.split(",")] if a.steps else range(1, base["n_steps"] + 1)
    for k in steps:
        ak = base["a_init"] + k * (base["a_final"] - base["a_init"]) / base["n_steps"]
        cfg = dict(base, n_steps=k, a_final=ak)
        res = {}
        counts = None
        for prec in ("f64", "f32"):
            ctx = Context(cfg, prec, "cuda:0")
            if counts is None:
                counts = _mock_counts(ctx, cfg, R, 4)
            _observe(ctx, R, counts)
            s = torch.tensor(s0, dtype=ctx.dtype, device=ctx.device)
            delta = ctx.forward(s, delta=True)["delta"].double().cpu().numpy()
            L, g, terms, ms = _timed_eval(ctx, s, None)
            L, g, terms, ms = _timed_eval(ctx, s, g)
            res[prec] = dict(delta=delta, L=L, chi2=terms["chi2"], g=g.double().cpu().numpy(),
                             ms=ms)
            ctx.close()
            del ctx, s, g
            torch.cuda.empty_cache()
        r32, r64 = res["f32"], res["f64"]
        _emit(dict(study="precision", workload="256^3 particles, 512^3 mesh, 1000 Mpc/h",
                   step=k, a=ak, density_rel_l2=_rel(r32["delta"], r64["delta"]),
                   chi2_f64=r64["chi2"], chi2_rel=abs(r32["chi2"] - r64["chi2"]) / r64["chi2"],
                   loss_rel=abs(r32["L"] - r64["L"]) / r64["L"],
                   grad_rel_l2=_rel(r32["g"], r64["g"]), eval_ms_f32=r32["ms"],
                   eval_ms_f64=r64["ms"]), a.out)


def scale(a):
    import torch

    from paper_2604_26823_amd.api import Context
    cfg = inputs.config(5, ckpt_every=a.ckpt_every, tape_forces=a.tape_forces)
    R = inputs.response_field(cfg)
    cfg["nbar"] = inputs.nbar_for(cfg, R)
    s_start = inputs.white_noise(cfg["n_part"], inputs.seeds(5)["start"])
    work = ("512^3 particles, 1024^3 mesh, 2000 Mpc/h, 20 steps, ckpt_every %d, tape_forces %d"
            % (a.ckpt_every, a.tape_forces))
    torch.cuda.reset_peak_memory_stats()
    ctx = Context(cfg, "f32", "cuda:0")
    counts = _mock_counts(ctx, cfg, R, 5)
    _observe(ctx, R, counts)
    s = torch.tensor(s_start, dtype=ctx.dtype, device=ctx.device)
    ctx.project_rankmatch(s, _lib.IC_PROJECT, event=0, trial=0)
    s_proj = s.double().cpu().numpy()
    delta32 = ctx.forward(s, delta=True)["delta"].double().cpu().numpy()
    L32, g, terms32, _ = _timed_eval(ctx, s, None)
    L32, g, terms32, ms32 = _timed_eval(ctx, s, g, repeats=a.repeats)
    g32 = g.double().cpu().numpy()
    if a.profile:
        ctx.timing(True)
        ctx.loss_and_grad(s, g)
        rows = ctx.timing_report()
        ctx.timing(False)
        for r in sorted(rows, key=lambda r: -r["ms"])[:20]:
            _emit(dict(study="scale", workload=work, precision="f32", kernel=r["name"],
                       count=r["count"], ms=r["ms"]), a.out)
    free, total = torch.cuda.mem_get_info()
    _emit(dict(study="scale", workload=work, precision="f32", eval_ms=ms32, loss=L32,
               chi2=terms32["chi2"], workspace_gb=ctx.ws_bytes / 1e9,
               peak_allocated_gb=torch.cuda.max_memory_allocated() / 1e9,
               device_used_gb=(total - free) / 1e9, device_total_gb=total / 1e9), a.out)
    L = L32
    t0 = time.perf_counter()
    evals = 0
    for it in range(a.iterations):
        t = time.perf_counter()
        L, info = ctx.lbfgs_step(s, g, L, it)
        evals += info["evaluations"]
        rom = None
        if (it + 1) % 20 == 0:
            rom = ctx.project_rankmatch(s, _lib.IC_PROJECT | _lib.IC_ROM_REAL
                                        | _lib.IC_ROM_FOURIER, event=it + 1)
            ctx.lbfgs_reset()
            L, g, _ = ctx.loss_and_grad(s, g)
            evals += 1
        torch.cuda.synchronize()
        _emit(dict(study="scale", workload=work, iteration=it, loss=L, eps=info["eps"],
                   evaluations=info["evaluations"], rom=rom,
                   seconds=time.perf_counter() - t), a.out)
    if a.iterations:
        _emit(dict(study="scale", workload=work, precision="f32", iterations=a.iterations,
                   evaluations=evals, seconds=time.perf_counter() - t0,
                   peak_allocated_gb=torch.cuda.max_memory_allocated() / 1e9), a.out)
    ctx.close()
    del ctx, s, g
    torch.cuda.empty_cache()
    if a.skip_f64:
        return
    torch.cuda.reset_peak_memory_stats()
    ctx = Context(cfg, "f64", "cuda:0")
    _observe(ctx, R, counts)
    s = torch.tensor(s_proj, dtype=ctx.dtype, device=ctx.device)
    delta64 = ctx.forward(s, delta=True)["delta"].double().cpu().numpy()
    L64, g, terms64, ms64 = _timed_eval(ctx, s, None)
    free, total = torch.cuda.mem_get_info()
    _emit(dict(study="scale", workload=work, precision="f64", eval_ms=ms64, loss=L64,
               chi2=terms64["chi2"], workspace_gb=ctx.ws_bytes / 1e9,
               peak_allocated_gb=torch.cuda.max_memory_allocated() / 1e9,
               device_used_gb=(total - free) / 1e9,
               density_rel_l2_f32=_rel(delta32, delta64),
               loss_rel_f32=abs(L32 - L64) / abs(L64),
               chi2_rel_f32=abs(terms32["chi2"] - terms64["chi2"]) / terms64["chi2"],
               grad_rel_l2_f32=_rel(g32, g.double().cpu().numpy())), a.out)
    ctx.close()


def _white_noise_stats(x):
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    m, sd = float(x.mean()), float(x.std())
    z = (x - m) / sd
    return dict(mean=m, std=sd, max_abs=float(np.abs(x).max()),
                excess_kurtosis=float(np.mean(z ** 4) - 3.0),
                frac_above_4=float(np.mean(np.abs(x) > 4.0)))


def _smooth(x, cells):
    """Gaussian smoothing (sigma in cells) by a host FFT: the large scales the
    data constrain, without the small-scale white noise they leave free."""
    n = x.shape[0]
    j = np.fft.fftfreq(n, 1.0 / n)
    jz = np.arange(n // 2 + 1)
    k2 = (2 * np.pi / n) ** 2 * (j[:, None, None] ** 2 + j[None, :, None] ** 2
                                 + jz[None, None, :] ** 2)
    return np.fft.irfftn(np.fft.rfftn(x) * np.exp(-0.5 * k2 * cells ** 2), s=x.shape,
                         axes=(0, 1, 2))


def _cross_correlation(a, b, box, nbins=10):
    """r_c(k) = P_ab / sqrt(P_aa P_bb) in linear k bins up to the Nyquist
    frequency (host FFT of two fields; a diagnostic, not part of the path)."""
    n = a.shape[0]
    fa, fb = np.fft.rfftn(a), np.fft.rfftn(b)
    kf = 2.0 * np.pi / box
    j = np.fft.fftfreq(n, 1.0 / n)
    jz = np.arange(n // 2 + 1)
    k = kf * np.sqrt(j[:, None, None] ** 2 + j[None, :, None] ** 2 + jz[None, None, :] ** 2)
    w = np.full(fa.shape, 2.0)
    w[..., 0] = 1.0
    w[..., -1] = 1.0
    edges = np.linspace(kf, np.pi * n / box, nbins + 1)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (k >= lo) & (k < hi)
        pab = np.sum(w[m] * (fa[m] * np.conj(fb[m])).real)
        paa = np.sum(w[m] * np.abs(fa[m]) ** 2)
        pbb = np.sum(w[m] * np.abs(fb[m]) ** 2)
        out.append([0.5 * (lo + hi), float(pab / np.sqrt(paa * pbb))])
    return out


def _optimise(ctx, s, g, L, iterations, rom_every, event0, curve_every, progress=None,
              keep=None):
    """Projected (or plain) L-BFGS from (s, g, L) in place; a rank-order
    matching event (real, Fourier, projection, history reset) every
    rom_every iterations when rom_every > 0.  keep: optional dict whose keys
    are iteration counts; a copy of s after that many iterations (after the
    matching event, if one falls there) is stored under each.  Returns the
    loss curve, the evaluation count, a status and the final loss."""
    curve, evals, status = [[0, L]], 0, "ok"
    for it in range(iterations):
        try:
            L, info = ctx.lbfgs_step(s, g, L, it)
        except _lib.IcError as e:
            status = "stopped at iteration %d: %s" % (it, e)
            break
        evals += info["evaluations"]
        if rom_every and (it + 1) % rom_every == 0:
            ctx.project_rankmatch(s, _lib.IC_PROJECT | _lib.IC_ROM_REAL | _lib.IC_ROM_FOURIER,
                                  event=event0 + it + 1)
            ctx.lbfgs_reset()
            L, g, _ = ctx.loss_and_grad(s, g)
            evals += 1
        if (it + 1) % curve_every == 0:
            curve.append([it + 1, L])
            if progress:
                progress(it + 1, L)
        if keep is not None and it + 1 in keep:
            keep[it + 1] = s.clone()
    return curve, evals, status, L


def ablation(a):
    import torch

    from paper_2604_26823_amd.api import Context
    if a.objective == "paper":
        # the paper's objective at its coarse level: c6 geometry on 128^3
        # (3.9 Mpc/h cells), 18 steps, lightcone, Poisson likelihood, no prior
        cid = 6
        base = inputs.config(6, n_part=128, n_mesh=128, lightcone=(0.8, 0.9, 1.0))
        work = ("128^3, 500 Mpc/h, 18 steps, Planck13, disk footprint, lightcone, Poisson "
                "without prior, 1.06e6 galaxies")
    else:
        cid = 2
        base = inputs.config(2)
        work = "128^3, 512 Mpc/h, 10 steps, radial selection, ~1e6 galaxies"
    R = inputs.response_field(base)
    sd = inputs.seeds(cid)
    s_true = inputs.white_noise(base["n_part"], sd["truth"])
    s_start = inputs.white_noise(base["n_part"], sd["start"])
    if a.objective == "paper":
        counts = _catalogue_counts(base, R, s_true, sd["counts"])
    else:
        base["nbar"] = inputs.nbar_for(base, R)
        counts = None
    runs = [("method", dict(project_steps=1, eps_max=1.0), True)]
    runs += [("lbfgs_eps%g" % e, dict(project_steps=0, eps_max=e), False)
             for e in (1.0, 0.1, 0.01, 0.001)]
    # plain L-BFGS (eps_max = 1) from the method's checkpoints 5, 10 and 15
    # (one every 20 iterations, right after a matching event), run to the
    # same total iteration count (table 1: M05L30, M10L30, M15L30)
    restarts = [k for k in (5, 10, 15) if 20 * k < a.iterations] if a.restarts else []
    keep = {20 * k: None for k in restarts}
    first = True
    for name, over, rom in runs:
        cfg = dict(base, **over)
        ctx = Context(cfg, "f32", "cuda:0")
        if first:
            first = False
            if counts is None:
                counts = _mock_counts(ctx, cfg, R, cid)
            _observe(ctx, R, counts)
            zero = torch.zeros(ctx.grid, dtype=ctx.dtype, device=ctx.device)
            L0 = ctx.loss_and_grad(zero)[0]
            _emit(dict(study="ablation", workload=work, run="homogeneous s = 0", loss=L0), a.out)
            st = torch.tensor(s_true, dtype=ctx.dtype, device=ctx.device)
            _emit(dict(study="ablation", workload=work, run="truth s_true",
                       loss=ctx.loss_and_grad(st)[0]), a.out)
        _observe(ctx, R, counts)
        s = torch.tensor(s_start, dtype=ctx.dtype, device=ctx.device)
        ctx.project_rankmatch(s, _lib.IC_PROJECT, event=0, trial=0)
        L, g, _ = ctx.loss_and_grad(s)
        t0 = time.perf_counter()
        curve, evals, status, L = _optimise(ctx, s, g, L, a.iterations, 20 if rom else 0, 0, 10,
                                            keep=keep if name == "method" else None)
        evals += 1
        torch.cuda.synchronize()
        _ablation_record(a, work, name, base, R, s_true, s, L, status, evals, t0, curve)
        ctx.close()
        del ctx, s, g
        torch.cuda.empty_cache()
    for k in restarts:
        ctx = Context(dict(base, project_steps=0, eps_max=1.0), "f32", "cuda:0")
        _observe(ctx, R, counts)
        s = keep[20 * k].to(ctx.device)
        L, g, _ = ctx.loss_and_grad(s)
        t0 = time.perf_counter()
        curve, evals, status, L = _optimise(ctx, s, g, L, a.iterations - 20 * k, 0, 0, 10)
        curve = [[20 * k + i, v] for i, v in curve]
        torch.cuda.synchronize()
        _ablation_record(a, work, "M%02dL (plain L-BFGS from checkpoint %d)" % (k, k), base, R,
                         s_true, s, L, status, evals + 1, t0, curve)
        ctx.close()
        del ctx, s, g
        torch.cuda.empty_cache()


def _ablation_record(a, work, name, base, R, s_true, s, L, status, evals, t0, curve):
    final = s.double().cpu().numpy()
    m = R >= base["r_min"]
    corr_m = float(np.corrcoef(_smooth(final, 4.0)[m], _smooth(s_true, 4.0)[m])[0, 1])
    _emit(dict(study="ablation", workload=work, run=name, status=status, final_loss=L,
               evaluations=evals, seconds=time.perf_counter() - t0, loss_curve=curve,
               white_noise=_white_noise_stats(final), corr_masked=corr_m,
               r_c=_cross_correlation(final, s_true, base["box"])), a.out)


def _catalogue_counts(cfg, R, s_true, seed):
    """Sets cfg["nbar"] so that the truth's rate sums to the catalogue size
    over the mask (the rate is linear in N-bar) and returns Poisson counts at
    that N-bar, from this library's FP32 forward model."""
    import torch

    from paper_2604_26823_amd.api import Context
    cfg["nbar"] = 1.0
    ctx = Context(cfg, "f32", "cuda:0")
    _observe(ctx, R, np.zeros(R.shape, dtype=np.int32))
    lam = ctx.forward(torch.tensor(s_true, dtype=ctx.dtype, device=ctx.device), delta=False,
                      lam=True)["lambda"].double().cpu().numpy()
    ctx.close()
    del ctx
    cfg["nbar"] = cfg["galaxies"] / float(lam[R >= cfg["r_min"]].sum())
    return inputs.poisson_counts(lam * cfg["nbar"], R, cfg["r_min"], seed)


def lightcone(a):
    import torch

    from paper_2604_26823_amd.api import Context
    snaps = (0.8, 0.9, 1.0)
    cfg = inputs.config(6, lightcone=snaps)
    R = inputs.response_field(cfg)
    sd = inputs.seeds(6)
    n = cfg["n_part"]
    s_true = inputs.white_noise(n, sd["truth"])
    counts = _catalogue_counts(cfg, R, s_true, sd["counts"])
    static = dict(cfg, lightcone=())
    work = "c6 with snapshots at a = 0.8, 0.9, 1.0: 256^3, 500 Mpc/h, 18 steps, Poisson"
    s0 = None
    out = {}
    for prec in ("f32", "f64"):
        for name, c in (("lightcone", cfg), ("static", static)):
            ctx = Context(c, prec, "cuda:0")
            _observe(ctx, R, counts)
            s = torch.tensor(inputs.white_noise(n, sd["start"]), dtype=ctx.dtype,
                             device=ctx.device)
            if s0 is None:
                ctx.project_rankmatch(s, _lib.IC_PROJECT, event=0, trial=0)
                s0 = s.double().cpu().numpy()
            else:
                s = torch.tensor(s0, dtype=ctx.dtype, device=ctx.device)
            delta = ctx.forward(s, delta=True)["delta"].double().cpu().numpy()
            L, g, terms, _ = _timed_eval(ctx, s, None)
            L, g, terms, ms = _timed_eval(ctx, s, g, repeats=a.repeats)
            ctx.timing(True)
            ctx.loss_and_grad(s, g)
            rows = {r["name"]: r for r in ctx.timing_report()}
            ctx.timing(False)
            lc_ms = {k: v["ms"] for k, v in rows.items() if k.startswith("lc_")}
            out[(prec, name)] = (delta, L, g.double().cpu().numpy())
            _emit(dict(study="lightcone", workload=work, precision=prec, model=name,
                       eval_ms=ms, loss=L, chi2=terms["chi2"], lightcone_kernels_ms=lc_ms,
                       workspace_gb=ctx.ws_bytes / 1e9), a.out)
            ctx.close()
            del ctx, s, g
            torch.cuda.empty_cache()
    d32, L32, g32 = out[("f32", "lightcone")]
    d64, L64, g64 = out[("f64", "lightcone")]
    ds64 = out[("f64", "static")][0]
    _emit(dict(study="lightcone", workload=work, density_rel_l2_f32=_rel(d32, d64),
               loss_rel_f32=abs(L32 - L64) / abs(L64), grad_rel_l2_f32=_rel(g32, g64),
               lightcone_vs_static_density_rel_l2=_rel(d64, ds64),
               lightcone_vs_static_loss=[L64, out[("f64", "static")][1]]), a.out)


def schedule(a):
    import torch

    from paper_2604_26823_amd.api import Context
    cfg = inputs.config(6, lightcone=(0.8, 0.9, 1.0) if a.lightcone else ())
    R = inputs.response_field(cfg)
    sd = inputs.seeds(6)
    n = cfg["n_part"]
    s_true = inputs.white_noise(n, sd["truth"])
    work = "c6: 256^3, 500 Mpc/h, 18 steps, Planck13, disk footprint, Poisson, 1.06e6 galaxies"
    if a.lightcone:
        work += ", lightcone from snapshots at a = 0.8, 0.9, 1.0"
    counts = _catalogue_counts(cfg, R, s_true, sd["counts"])
    hi = Context(cfg, "f32", "cuda:0")
    _observe(hi, R, counts)
    m = R >= cfg["r_min"]
    zero = torch.zeros(hi.grid, dtype=hi.dtype, device=hi.device)
    _emit(dict(study="schedule", workload=work, run="homogeneous s = 0",
               loss=hi.loss_and_grad(zero)[0], galaxies=int(counts.sum()), nbar=cfg["nbar"]),
          a.out)
    st = torch.tensor(s_true, dtype=hi.dtype, device=hi.device)
    _emit(dict(study="schedule", workload=work, run="truth s_true",
               loss=hi.loss_and_grad(st)[0]), a.out)
    del zero, st

    def progress(tag):
        return lambda it, L: print("%s iteration %d loss %.6e" % (tag, it, L), flush=True)

    def report(name, s, curve, evals, status, L, seconds, extra):
        final = s.double().cpu().numpy()
        corr = float(np.corrcoef(_smooth(final, 4.0)[m], _smooth(s_true, 4.0)[m])[0, 1])
        _emit(dict(study="schedule", workload=work, run=name, status=status, final_loss=L,
                   evaluations=evals, seconds=seconds, loss_curve=curve,
                   white_noise=_white_noise_stats(final), corr_masked=corr,
                   r_c=_cross_correlation(final, s_true, cfg["box"]), **extra), a.out)

    for run in a.runs.split(","):
        t0 = time.perf_counter()
        extra = {}
        if run == "annealed":
            low_cfg = dict(cfg, n_part=n // 2, n_mesh=n // 2, nbar=8.0 * cfg["nbar"])
            Nl, Rl = inputs.coarsen(counts, R)
            lo = Context(low_cfg, "f32", "cuda:0")
            _observe(lo, Rl, Nl)
            sl = torch.tensor(inputs.white_noise(n // 2, sd["start"]), dtype=lo.dtype,
                              device=lo.device)
            lo.project_rankmatch(sl, _lib.IC_PROJECT, event=0, trial=0)
            L, g, _ = lo.loss_and_grad(sl)
            lcurve, levals, lstatus, L = _optimise(lo, sl, g, L, a.low_iterations,
                                                   cfg["low_rom_every"], 0, 10,
                                                   progress("low"))
            torch.cuda.synchronize()
            extra.update(low=dict(cells=n // 2, final_loss=L, evaluations=levals + 1,
                                  status=lstatus, loss_curve=lcurve,
                                  seconds=time.perf_counter() - t0))
            s = hi.upsample_from(lo, sl, 1)
            lo.close()
            del lo, sl, g
            torch.cuda.empty_cache()
        else:
            s = torch.tensor(inputs.white_noise(n, sd["start"]), dtype=hi.dtype, device=hi.device)
        hi.lbfgs_reset()
        hi.project_rankmatch(s, _lib.IC_PROJECT, event=0, trial=0)
        L, g, _ = hi.loss_and_grad(s)
        extra["start_loss"] = L
        curve, evals, status, L = _optimise(hi, s, g, L, a.iterations, cfg["rom_every"], 100000,
                                            50, progress(run))
        torch.cuda.synchronize()
        report(run, s, curve, evals + 1, status, L, time.perf_counter() - t0, extra)
        del s, g
    hi.close()


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    pr = sub.add_parser("precision")
    pr.add_argument("--steps", default="")
    ab = sub.add_parser("ablation")
    ab.add_argument("--iterations", type=int, default=200)
    ab.add_argument("--objective", choices=["c2", "paper"], default="c2")
    ab.add_argument("--restarts", action="store_true")
    sc = sub.add_parser("scale")
    sc.add_argument("--iterations", type=int, default=50)
    sc.add_argument("--repeats", type=int, default=3)
    sc.add_argument("--ckpt-every", type=int, default=5)
    sc.add_argument("--tape-forces", type=int, default=0)
    sc.add_argument("--profile", action="store_true")
    sc.add_argument("--skip-f64", action="store_true")
    lcp = sub.add_parser("lightcone")
    lcp.add_argument("--repeats", type=int, default=3)
    sh = sub.add_parser("schedule")
    sh.add_argument("--iterations", type=int, default=inputs.config(6)["iterations"])
    sh.add_argument("--low-iterations", type=int, default=inputs.config(6)["low_iterations"])
    sh.add_argument("--runs", default="annealed,cold")
    sh.add_argument("--lightcone", action="store_true")
    for p in (pr, sc, ab, sh, lcp):
        p.add_argument("--out", default="")
    a = ap.parse_args()
    {"precision": precision, "scale": scale, "ablation": ablation, "schedule": schedule,
     "lightcone": lightcone}[a.mode](a)


if __name__ == "__main__":
    main()
