"""Benchmark of the reconstruction hot path on one MI355X.

One step is one projected L-BFGS iteration of the method (projection of
s + eps p, loss + gradient evaluations of the line search, two-loop
recursion with FP64 dot products, history update), with the rank-order
matching event (real-space + Fourier-space matching + projection, history
reset, re-evaluation) every ``rom_every`` iterations, on the 256^3 survey-
shaped synthetic workload (c3).  The metric is gradient evaluations per
second: all loss + gradient evaluations made in the K timed steps divided by
their wall time, inputs already resident in HBM.

Also reported: the same loop with the FP64 instantiation of the kernels; a
per-kernel HIP-event table from a profiling pass run before the timed region;
the roofline of the dominant kernel (largest share of that table), whose
launches are timed with HIP events on the library stream during the timed
region itself: algorithmic bytes per launch from the byte ledger of one
gradient evaluation (each field a kernel must read or write counted once, in
units of U = one particle-grid field and U_m = one mesh field) divided by the
average launch time, against the 8 TB/s HBM peak, with the implementation's
own per-launch byte count beside it and its measured HBM traffic when a
hardware-counter summary taken on the current sources is present under
profiles/; the whole evaluation against the same ledger (1167 U at 10 steps)
for FP32 and FP64; the FP64 CPU oracle timed on the host cores on whole
loss + gradient evaluations of the same problem at 32^3 and 128^3; and one
timing of a 256^3 FP32 real FFT round trip through torch.fft (hipFFT/rocFFT)
beside the same round trip through this library's passes, for comparison
only; and the same whole-evaluation timing in the deterministic mode
(fixed-point paints, bitwise repeatable results) at the state the timed loop
ended in, beside the default mode's.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3]
                       [--no-fp64] [--no-cpu-baseline] [--no-fft-compare]
                       [--no-det-compare] [--profile-steps P] [--copy-mib N]
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = {
    1: "c1: 32^3 particles and mesh, 256 Mpc/h, 5 KDK steps, z-axis RSD, half-box mask",
    2: "c2: 128^3 particles and mesh, 512 Mpc/h, 10 KDK steps, radial RSD, 40x40 deg cone, "
       "~1e6 galaxies",
    3: "c3: 256^3 particles on a 256^3 mesh, 1000 Mpc/h, 10 KDK steps, radial RSD, 40x40 deg "
       "cone, r^2 exp(-(r/300)^1.5) selection, ~8e6 galaxies",
    4: "c4: 256^3 particles on a 512^3 mesh, 1000 Mpc/h, 20 KDK steps",
    5: "c5: 512^3 particles on a 1024^3 mesh, 2000 Mpc/h, 20 KDK steps",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(cfg, prec, counts=None, s_start=None):
    import torch

    from paper_2604_26823_amd import _lib, inputs
    from paper_2604_26823_amd.api import Context

    ctx = Context(cfg, prec, "cuda:0")
    R = inputs.response_field(cfg)
    resp = torch.tensor(R, dtype=ctx.dtype, device=ctx.device)
    if counts is None:
        # Mock data: the truth white noise through this library's forward model,
        # Poisson-sampled on the host from the seeded generator.
        sd = inputs.seeds(cfg["id"])
        s_true = torch.tensor(inputs.white_noise(cfg["n_part"], sd["truth"]), dtype=ctx.dtype,
                              device=ctx.device)
        dummy = torch.zeros(ctx.grid, dtype=torch.int32, device=ctx.device)
        ctx.set_observation(dummy, resp)
        lam = ctx.forward(s_true, delta=False, lam=True)["lambda"].double().cpu().numpy()
        counts = inputs.poisson_counts(lam, R, cfg["r_min"], sd["counts"])
        s_start = inputs.white_noise(cfg["n_part"], sd["start"])
    ctx.set_observation(torch.tensor(counts, dtype=torch.int32, device=ctx.device), resp)
    s = torch.tensor(s_start, dtype=ctx.dtype, device=ctx.device)
    ctx.project_rankmatch(s, _lib.IC_PROJECT, event=0, trial=0)
    return ctx, s, counts, s_start


def run_steps(ctx, s, g, L, first, k, rom_every):
    """k L-BFGS iterations starting at iteration index first; returns
    (L, evaluations, rom events)."""
    from paper_2604_26823_amd import _lib
    evals = roms = 0
    for it in range(first, first + k):
        L, info = ctx.lbfgs_step(s, g, L, it)
        evals += info["evaluations"]
        if rom_every and (it + 1) % rom_every == 0:
            ctx.project_rankmatch(s, _lib.IC_PROJECT | _lib.IC_ROM_REAL | _lib.IC_ROM_FOURIER,
                                  event=it + 1)
            ctx.lbfgs_reset()
            L, _, _ = ctx.loss_and_grad(s, g)
            evals += 1
            roms += 1
    return L, evals, roms


# Algorithmic bytes per launch from the evaluation's byte ledger: (a, b)
# means a U + b U_m, U = one particle-grid field (N_p^3 elements) and
# U_m = one mesh field (N_m^3), each field a kernel must read or write
# counted once (accumulation as a read and a write).
LEDGER = {
    "cic_paint_vec": (6, 6),   # positions, cotangent in; 3 meshes accumulated
    "force_adjoint": (15, 4),  # positions, p_bar in/out, d_bar in/out; 3 force meshes, rho_bar
    "pm_step": (12, 3),        # positions, momenta in/out; 3 force meshes
    "cic_paint": (3, 2),       # positions in; density accumulated
    "data_adjoint": (13, 0),   # positions, momenta, seed in; d_bar, p_bar out
    "loss": (5, 0),            # density, counts, response, s in; seed out
    "fft_r2c_z": (0, 2),       # real field in, half spectrum out (mesh chains)
    "fft_y": (0, 2),
    "fft_c2r_z": (0, 2),
    "fft_r2c_zy": (0, 2),      # the z and y passes fused (FP32, 256^3 grids)
    "fft_c2r_yz": (0, 2),
}


def ledger_eval_units(n_steps):
    """Ledger of one loss + gradient evaluation in U (N_m = N_p): forward
    89 (whitening, 2LPT) + 25 (first force) + 37 per step + 14 (last kick,
    RSD, data paint) + 5 (loss); adjoint 13 (data paint and RSD) + 51 per
    force VJP (n_steps + 1 of them) + 90 (2LPT, whitening, prior)."""
    return 89 + 25 + 37 * n_steps + 14 + 5 + 13 + 51 * (n_steps + 1) + 90


def kernel_rows(ctx):
    """Kernel rows of the timing report (tile-window statistics dropped)."""
    return [r for r in ctx.timing_report() if not r["name"].startswith("tiles_")]


def timed_loop(ctx, s, steps, warmup, rom_every, profile_steps=0):
    """Warmup, an optional all-kernel profiling pass, then the timed steps
    with the dominant kernel's launches timed live (FP32 context only)."""
    import torch
    L, g, _ = ctx.loss_and_grad(s)
    L, _, _ = run_steps(ctx, s, g, L, 0, warmup, rom_every)
    first = warmup
    table = dom = None
    if profile_steps:
        ctx.timing(True)
        L, _, _ = run_steps(ctx, s, g, L, first, profile_steps, rom_every)
        table = kernel_rows(ctx)
        ctx.timing(False)
        first += profile_steps
        dom = max(table, key=lambda r: r["ms"])["name"]
        ctx.timing_only(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, evals, roms = run_steps(ctx, s, g, L, first, steps, rom_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    live = None
    if dom is not None:
        live = [r for r in kernel_rows(ctx) if r["name"] == dom][0]
        ctx.timing(False)
    return dict(seconds=dt, evals=evals, roms=roms, loss=L, g=g, table=table, live=live)


def stored_traffic(kernel, dtype_tag):
    """HBM bytes per launch of a kernel from the hardware-counter summary in
    profiles/, or None when there is none or it was taken on other sources."""
    from paper_2604_26823_amd import build
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c3_%s.txt" % dtype_tag)
    if not os.path.exists(path):
        return None, "no counter summary"
    text = open(path).read()
    m = re.search(r"^sources_sha256 (\w+)$", text, re.M)
    if not m or m.group(1) != build.sources_digest():
        return None, "counter summary taken on other sources"
    m = re.search(r"^kernel %s \S+ .* hbm_bytes_per_launch (\S+)$" % re.escape(kernel), text,
                  re.M)
    if not m:
        return None, "kernel not in the counter summary"
    return float(m.group(1)), os.path.relpath(path, ROOT)


def ledger_bytes(name, cfg, elem):
    """Ledger bytes of one launch of a kernel, or None when the ledger has
    no row of its own for it (the x passes count (1 + m) half spectra, as the
    library's own figure does)."""
    if name not in LEDGER:
        return None
    a, b = LEDGER[name]
    return float(elem) * (a * cfg["n_part"] ** 3 + b * cfg["n_mesh"] ** 3)


def roofline(table, live, dtype_tag, cfg):
    """Dominant kernel (largest total time in the profiling pass) and its
    algorithmic bandwidth from the launches timed live in the timed region,
    on the ledger's bytes."""
    tot = sum(r["ms"] for r in table)
    avg_ms = live["ms"] / live["count"]
    kernels = {}
    for r in table:
        avg = r["ms"] / r["count"]
        lb = ledger_bytes(r["name"], cfg, 4)
        kernels[r["name"]] = dict(
            launches=r["count"], total_ms=round(r["ms"], 3), avg_us=round(1e3 * avg, 2),
            gbs_impl=round(r["bytes"] / (avg * 1e-3) / 1e9, 1) if r["bytes"] > 0 else None,
            gbs_ledger=round(lb / (avg * 1e-3) / 1e9, 1) if lb else None,
            share=round(r["ms"] / tot, 4))
    lb = ledger_bytes(live["name"], cfg, 4)
    if lb is None:
        lb = live["bytes"]
    gbs = lb / (avg_ms * 1e-3) / 1e9
    traffic, source = stored_traffic(live["name"], dtype_tag)
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=None if traffic is None else round(traffic),
                kernel=live["name"], launches_timed=live["count"],
                avg_us=round(1e3 * avg_ms, 2), bytes_per_launch=lb,
                bytes_per_launch_impl=live["bytes"],
                ledger="%s U + %s U_m, U = 4 N_p^3 bytes, U_m = 4 N_m^3 bytes"
                % LEDGER.get(live["name"], ("?", "?")),
                traffic_source=source), kernels


def eval_roofline(ctx, s, cfg, elem, n=10):
    """Whole loss + gradient evaluations at s (3 untimed, then n timed by the
    wall clock with the device synchronised around them) against the
    ledger of one evaluation (N_m = N_p only)."""
    import torch
    for _ in range(3):
        ctx.loss_and_grad(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.loss_and_grad(s)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / n
    out = dict(ms_per_eval=round(ms, 3), evals=n)
    if cfg["n_mesh"] == cfg["n_part"]:
        units = ledger_eval_units(cfg["n_steps"])
        b = float(elem) * units * cfg["n_part"] ** 3
        out.update(ledger_units=units, ledger_gb=round(b / 1e9, 2),
                   achieved_gbs=round(b / (ms * 1e-3) / 1e9, 1),
                   frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    return out


def det_compare(cfg, prec, counts, s_start, s_end, elem, ev_default):
    """Whole evaluations in the deterministic mode at s_end, beside the
    default mode's at the same state."""
    import torch
    ctx, _, _, _ = setup(dict(cfg, deterministic=1), prec, counts, s_start)
    out = eval_roofline(ctx, s_end, cfg, elem)
    del ctx
    torch.cuda.empty_cache()
    out["slowdown_vs_default"] = round(out["ms_per_eval"] / ev_default["ms_per_eval"], 4)
    return out


def fft_compare(ctx):
    """One 256^3 FP32 real FFT round trip through torch.fft (hipFFT/rocFFT)
    and through this library's passes (median of 10 each, HIP events).
    Comparison only: the hot path never calls a vendor FFT."""
    import torch
    n = ctx.n
    x = torch.randn((n, n, n), dtype=torch.float32, device=ctx.device)

    def med(fn):
        ts = []
        for i in range(13):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            if i >= 3:
                ts.append(a.elapsed_time(b))
        return sorted(ts)[len(ts) // 2]

    vendor = med(lambda: torch.fft.irfftn(torch.fft.rfftn(x), s=(n, n, n)))
    ours = med(lambda: ctx.irfft(ctx.rfft(x)))
    return dict(n=n, dtype="f32", torch_fft_ms=round(vendor, 3), library_ms=round(ours, 3),
                note="rfftn + irfftn round trip; the library figure includes its copies "
                     "between the padded and the contiguous half-spectrum layouts")


def cpu_baseline(cfg):
    """The FP64 oracle on the host cores: one whole loss + gradient
    evaluation each of the same problem at 32^3 particles (box scaled to keep
    the cell size) and at 128^3, with mock counts from the oracle's own
    forward model.  The oracle's cost grows linearly with the particle count
    (its CIC passes dominate), so the benchmark's rate is the 128^3 rate
    divided by the particle-count ratio; both measured times are reported."""

    from oracle import fourier
    from oracle.model import Model, Problem
    from paper_2604_26823_amd import inputs

    def timed_eval(n):
        c = dict(cfg, n_part=n, n_mesh=n * cfg["n_mesh"] // cfg["n_part"],
                 box=cfg["box"] * n / cfg["n_part"])
        R = inputs.response_field(c)  # same cell size and galaxies per cell as cfg
        mdl = Model(Problem(**{k: c[k] for k in Problem.__dataclass_fields__ if k in c}))
        sd = inputs.seeds(cfg["id"])
        s_true = inputs.white_noise(n, sd["truth"])
        N = inputs.poisson_counts(mdl.observe(mdl.forward(s_true), R), R, c["r_min"],
                                  sd["counts"])
        s0 = inputs.white_noise(n, sd["start"])
        t0 = time.perf_counter()
        mdl.loss_and_grad(s0, N, R)
        return time.perf_counter() - t0

    t_small = timed_eval(32)
    n_mid = min(128, cfg["n_part"])
    t_mid = timed_eval(n_mid)
    ratio = (cfg["n_part"] / n_mid) ** 3
    t_eval = t_mid * ratio
    lin = t_mid / t_small / (n_mid / 32) ** 3
    return dict(value=round(1.0 / t_eval, 6), unit="grad evals/s", cores=fourier._workers(),
                kind="oracle",
                sample="whole oracle loss+gradient evaluations of this problem in this run: "
                       "%.2f s at 32^3, %.1f s at %d^3 (cost per particle %.2fx the 32^3 one); "
                       "rate at %d^3 = 1 / (%d^3 time x %.0f particle-count ratio) = 1 / %.0f s"
                       % (t_small, t_mid, n_mid, lin, cfg["n_part"], n_mid, ratio, t_eval),
                seconds_32=round(t_small, 3), seconds_mid=round(t_mid, 2), n_mid=n_mid,
                seconds_per_eval_scaled=round(t_eval, 1),
                threads_note="scipy.fft workers = cores; CIC passes single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fft-compare", action="store_true")
    ap.add_argument("--no-det-compare", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one device copy of this many MiB (a known-size "
                         "kernel for calibrating hardware byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is single-GPU (multi-GPU sharding is "
              "a design note, not built); got --gpus %d" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_26823_amd import _lib, inputs
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2604_26823_amd import build
        build.build()
    cfg = inputs.config(a.config)
    R = inputs.response_field(cfg)
    cfg["nbar"] = inputs.nbar_for(cfg, R)
    rom_every = cfg["rom_every"]

    log("bench: building FP32 context for %s" % WORKLOAD[a.config])
    ctx, s, counts, s_start = setup(cfg, "f32")
    log("bench: FP32 warmup %d + profiling pass %d + timed %d steps"
        % (a.warmup, a.profile_steps, a.steps))
    r32 = timed_loop(ctx, s, a.steps, a.warmup, rom_every, max(1, a.profile_steps))
    log("bench: FP32 %d evals in %.3f s" % (r32["evals"], r32["seconds"]))
    roof, table = roofline(r32["table"], r32["live"], "fp32", cfg)
    log("bench: FP32 whole-evaluation timing")
    ev32 = eval_roofline(ctx, s, cfg, 4)
    fftc = None
    if not a.no_fft_compare:
        log("bench: FFT round-trip comparison")
        fftc = fft_compare(ctx)
    ws_gb = ctx.ws_bytes / 1e9
    s_end = s.clone()
    del ctx, s
    r32.pop("g")
    torch.cuda.empty_cache()
    det = None
    if not a.no_det_compare:
        log("bench: FP32 deterministic-mode evaluations")
        det = {"fp32": det_compare(cfg, "f32", counts, s_start, s_end, 4, ev32)}
    del s_end

    r64 = ev64 = None
    if not a.no_fp64:
        log("bench: FP64 context")
        ctx64, s64, _, _ = setup(cfg, "f64", counts, s_start)
        r64 = timed_loop(ctx64, s64, a.steps, a.warmup, rom_every)
        r64.pop("g")
        ev64 = eval_roofline(ctx64, s64, cfg, 8)
        log("bench: FP64 %d evals in %.3f s" % (r64["evals"], r64["seconds"]))
        s64_end = s64.clone()
        del ctx64, s64
        torch.cuda.empty_cache()
        if det is not None:
            log("bench: FP64 deterministic-mode evaluations")
            det["fp64"] = det_compare(cfg, "f64", counts, s_start, s64_end, 8, ev64)
        del s64_end

    cpu = None
    if not a.no_cpu_baseline:
        log("bench: CPU oracle evaluations")
        cpu = cpu_baseline(cfg)

    value = r32["evals"] / r32["seconds"]
    out = {
        "metric": "PM forward+adjoint grad evals/s at 256^3, FP32 vs FP64, % HBM peak",
        "value": round(value, 3),
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * r32["seconds"] / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD[a.config], "n_part": cfg["n_part"],
                   "n_mesh": cfg["n_mesh"], "box": cfg["box"], "n_steps": cfg["n_steps"],
                   "rom_every": rom_every, "parallelism": "single GPU"},
        "evaluations": r32["evals"],
        "rom_events": r32["roms"],
        "final_loss": r32["loss"],
        "fp64": None if r64 is None else {
            "value": round(r64["evals"] / r64["seconds"], 3), "unit": "grad evals/s",
            "evaluations": r64["evals"], "ms_per_step": round(1e3 * r64["seconds"] / a.steps, 3)},
        "roofline": roof,
        "eval_roofline": {"fp32": ev32, "fp64": ev64},
        "kernels": table,
        "fft_compare": fftc,
        "deterministic": det,
        "workspace_gb": round(ws_gb, 2),
        "cpu_baseline": cpu,
    }
    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of %d MiB done" % a.copy_mib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
