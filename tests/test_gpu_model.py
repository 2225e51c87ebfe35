"""End-to-end parity of the forward model and its gradient (GPU).

Tolerances (FP32): final density relative L2 <= 1e-5, gradient relative L2
<= 1e-4 against the FP64 oracle on identical seeded inputs; FP64 on the GPU
matches to ~1e-10 (differences are summation order only)."""
import numpy as np
import pytest

from gpu_common import (DEV, cfg_small, context, model, observation, rel_l2, require_gpu,
                        to_dev, to_np, torch)
from paper_2604_26823_amd import inputs

pytestmark = pytest.mark.gpu

CASES = {
    "c1": dict(c=1),
    "c1_16": dict(c=1, n_part=16, n_mesh=16, box=128.0),
    "radial32": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5, galaxies=2e4),
    "radial32_mesh2": dict(c=2, n_part=32, n_mesh=64, box=128.0, n_steps=5, galaxies=2e4),
    # sigma8 = 6: shell crossing everywhere, most particles in a few dense cells,
    # blocks with several work items (the regime of the first L-BFGS steps)
    "clustered32": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5, galaxies=2e4,
                        sigma8=6.0),
    # the same with force meshes recomputed in the adjoint instead of taped
    "clustered32_recompute": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5,
                                  galaxies=2e4, sigma8=6.0, tape_forces=0),
    # particle states kept at steps 0, 2, 4 only, the others replayed in the
    # adjoint (segments of two states; with taped and with recomputed forces)
    "clustered32_ckpt2": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5, galaxies=2e4,
                              sigma8=6.0, ckpt_every=2),
    "radial32_mesh2_ckpt3_recompute": dict(c=2, n_part=32, n_mesh=64, box=128.0, n_steps=5,
                                           galaxies=2e4, ckpt_every=3, tape_forces=0),
    # one step in a 16 Mpc/h box: ~1.4% of the particles leave the 27 blocks
    # around their block in the drift (the per-wavefront rank fallback)
    "far32": dict(c=2, n_part=32, n_mesh=32, box=16.0, n_steps=1, galaxies=2e4),
    "far32_mesh2": dict(c=2, n_part=32, n_mesh=64, box=16.0, n_steps=1, galaxies=2e4),
    # the paper's observation model: power-law x sigmoid bias, Poisson likelihood;
    # with the white-noise prior, and likelihood only (prior weight 0)
    "poisson_c1": dict(c=1, loss="poisson"),
    "poisson_radial32": dict(c=2, n_part=32, n_mesh=32, box=128.0, n_steps=5, galaxies=2e4,
                             loss="poisson", prior_weight=0.0),
    # the paper-scale geometry (observer inside the 500 Mpc/h box, disk footprint,
    # Planck13, Poisson without prior) on a 32^3 lattice
    "disk32": dict(c=6, n_part=32, n_mesh=32, n_steps=4, galaxies=2e4),
    # the lightcone (snapshots at a = 0.8, 0.9, 1.0, three fixed-point
    # iterations) at the paper's 18 steps; with checkpoints and recomputed
    # forces; with the plane-parallel RSD of c1 (snapshots at steps 3 and 4)
    "lightcone32": dict(c=6, n_part=32, n_mesh=32, galaxies=2e4, lightcone=(0.8, 0.9, 1.0)),
    "lightcone32_ckpt4_recompute": dict(c=6, n_part=32, n_mesh=32, galaxies=2e4,
                                        lightcone=(0.8, 0.9, 1.0), ckpt_every=4,
                                        tape_forces=0),
    "lightcone_c1": dict(c=1, lightcone=(0.64, 0.82, 1.0)),
    # four snapshots (the maximum) and a single fixed-point iteration
    "lightcone32_4snap_iter1": dict(c=6, n_part=32, n_mesh=32, galaxies=2e4,
                                    lightcone=(0.7, 0.8, 0.9, 1.0), lc_iterations=1),
    # snapshot readouts on a force mesh twice as fine as the particle grid
    "lightcone32_mesh2": dict(c=6, n_part=32, n_mesh=64, galaxies=2e4,
                              lightcone=(0.8, 0.9, 1.0)),
    # the lightcone without redshift-space distortions (positions only)
    "lightcone32_norsd": dict(c=6, n_part=32, n_mesh=32, galaxies=2e4, rsd="none",
                              lightcone=(0.8, 0.9, 1.0)),
}
TOL_DENS = {"f32": 1e-5, "f64": 1e-10}
TOL_GRAD = {"f32": 1e-4, "f64": 1e-9}


def case(name):
    kw = dict(CASES[name])
    c = kw.pop("c")
    return cfg_small(c, **kw)


def prepared(name, prec):
    cfg = dict(case(name))
    cfg["nbar"] = inputs.nbar_for(cfg, inputs.response_field(cfg))
    mdl = model(cfg)
    R, N, s0 = observation(cfg, mdl)
    ctx = context(cfg, prec)
    ctx.set_observation(torch.tensor(N, dtype=torch.int32, device=DEV), to_dev(R, prec))
    return cfg, mdl, ctx, R, N, s0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_density(prec, name):
    require_gpu()
    cfg, mdl, ctx, R, N, s0 = prepared(name, prec)
    out = ctx.forward(to_dev(s0, prec), delta=True, lam=True, loss=True)
    L_ref, st = mdl.loss(s0, N, R, return_state=True)
    err = rel_l2(to_np(out["delta"]), st["delta_s"])
    print("density rel L2 %.3e, loss rel %.3e" % (err, abs(out["loss"] - L_ref) / abs(L_ref)))
    assert err <= TOL_DENS[prec]
    assert abs(out["loss"] - L_ref) <= TOL_DENS[prec] * abs(L_ref)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_loss_and_gradient(prec, name):
    require_gpu()
    cfg, mdl, ctx, R, N, s0 = prepared(name, prec)
    L, g, terms = ctx.loss_and_grad(to_dev(s0, prec))
    L_ref, g_ref, st = mdl.loss_and_grad(s0, N, R)
    print("loss rel %.3e, gradient rel L2 %.3e" % (abs(L - L_ref) / abs(L_ref),
                                                    rel_l2(to_np(g), g_ref)))
    assert abs(L - L_ref) <= TOL_DENS[prec] * abs(L_ref)
    assert abs(terms["chi2"] - st["chi2"]) <= TOL_DENS[prec] * abs(st["chi2"])
    assert rel_l2(to_np(g), g_ref) <= TOL_GRAD[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_vjp_matches_oracle(prec):
    require_gpu()
    cfg, mdl, ctx, R, N, s0 = prepared("radial32", prec)
    w = np.random.default_rng(5).standard_normal(s0.shape).astype(np.float32).astype(np.float64)
    got = to_np(ctx.vjp(to_dev(s0, prec), to_dev(w, prec)))
    ref = mdl.vjp(s0, w)
    assert rel_l2(got, ref) <= TOL_GRAD[prec]


def test_fp64_gpu_dot_product_identity():
    """<J v, w> from two GPU forwards (central difference in FP64 along v,
    step small enough that CIC weights stay linear) against <v, J^T w>."""
    require_gpu()
    cfg, mdl, ctx, R, N, s0 = prepared("c1_16", "f64")
    rng = np.random.default_rng(6)
    v = rng.standard_normal(s0.shape)
    w = rng.standard_normal(s0.shape)
    jtw = to_np(ctx.vjp(to_dev(s0, "f64"), to_dev(w, "f64")))
    jv = mdl.jvp(s0, v)
    a, b = float(np.sum(jv * w)), float(np.sum(v * jtw))
    assert abs(a - b) <= 1e-10 * abs(a)


# Checkpointed against fully taped adjoint on the same context settings: the
# replayed steps repeat the forward's arithmetic, and only the order of the
# global atomic additions in the recomputed paints can differ.
TOL_CKPT = {"f32": 2e-5, "f64": 1e-11}
TOL_CKPT_LOSS = {"f32": 1e-6, "f64": 1e-12}


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_checkpointed_gradient_matches_taped_c2(prec):
    require_gpu()
    base = cfg_small(2)
    base["nbar"] = inputs.nbar_for(base, inputs.response_field(base))
    R = inputs.response_field(base)
    sd = inputs.seeds(2)
    s0 = inputs.white_noise(base["n_part"], sd["start"])
    counts = None
    grads = {}
    for K, tf in ((0, 1), (5, 1), (3, 0)):
        cfg = dict(base, ckpt_every=K, tape_forces=tf)
        ctx = context(cfg, prec)
        resp = to_dev(R, prec)
        if counts is None:
            ctx.set_observation(torch.zeros(ctx.grid, dtype=torch.int32, device=DEV), resp)
            lam = to_np(ctx.forward(to_dev(inputs.white_noise(base["n_part"], sd["truth"]), prec),
                                    delta=False, lam=True)["lambda"])
            counts = inputs.poisson_counts(lam, R, base["r_min"], sd["counts"])
        ctx.set_observation(torch.tensor(counts, dtype=torch.int32, device=DEV), resp)
        L, g, _ = ctx.loss_and_grad(to_dev(s0, prec))
        grads[(K, tf)] = (L, to_np(g))
    L0, g0 = grads[(0, 1)]
    for key in ((5, 1), (3, 0)):
        L, g = grads[key]
        err = rel_l2(g, g0)
        print("ckpt_every %d tape_forces %d: loss rel %.3e gradient rel L2 %.3e"
              % (key[0], key[1], abs(L - L0) / abs(L0), err))
        assert abs(L - L0) <= TOL_CKPT_LOSS[prec] * abs(L0)
        assert err <= TOL_CKPT[prec]


def test_single_snapshot_lightcone_is_the_static_model():
    """A lightcone of the final snapshot alone places every particle at a_final
    with the final RSD factor: the same density as without the lightcone."""
    require_gpu()
    base = case("lightcone32")
    a = context(dict(base, lightcone=(1.0,)), "f64")
    b = context(dict(base, lightcone=()), "f64")
    R = inputs.response_field(base)
    s0 = inputs.white_noise(32, 11)
    for ctx in (a, b):
        ctx.set_observation(torch.zeros(ctx.grid, dtype=torch.int32, device=DEV),
                            to_dev(R, "f64"))
    da = to_np(a.forward(to_dev(s0, "f64"))["delta"])
    db = to_np(b.forward(to_dev(s0, "f64"))["delta"])
    assert np.max(np.abs(da - db)) <= 1e-12
