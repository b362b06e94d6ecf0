"""The adjoint behind torch.autograd.Function, upstream-gradient mode with an
opacity term, and recompute versus store."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as orc
from parity_util import MAX_KINK_SHARE, assert_close, relu_stable_rays
from synth.arch import ARCH_LARGE
from synth.params import init_params
from synth.workloads import LossSpec, prior_batch, prior_world

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_world = None


def world():
    global _world
    if _world is None:
        _world = prior_world(seed=1, pool_stride=5)
    return _world


def case(n_rays=1024, step=21):
    from paper_2503_01582_amd import api
    b = prior_batch(world(), n_rays, step=step, depth_noise=0.01, loss=LossSpec(lambda_d=0.1))
    arch = ARCH_LARGE
    params = init_params(arch, 5)
    params[:arch.n_table_params] = np.random.default_rng(6).uniform(
        -0.3, 0.3, arch.n_table_params).astype(np.float32)
    s = b.sample
    ref = orc.sample(b.rays_o, b.rays_d, b.xi, n_coarse=s.n_coarse, n_fine=s.n_fine,
                     include_coarse=s.include_coarse, uniform_only=s.uniform_only, eps=s.eps,
                     near=s.near, far=s.far, world_to_obj=b.world_to_obj, prior=b.prior)
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
           ref["dt"].astype(np.float32), ref["flags"])
    model = api.Model(arch, params)
    samp = api.SampleOut(*(torch.as_tensor(g).cuda() for g in geo[:3]),
                         bins=torch.zeros((n_rays, 1), dtype=torch.int32, device="cuda"),
                         flags=torch.as_tensor(geo[3]).cuda())
    return arch, params, b, geo, model, samp


def check_grads(arch, g, g_ref, tol=1e-5):
    nt = arch.n_table_params
    assert_close(g[:nt], g_ref[:nt], tol, "table grads")
    assert_close(g[nt:], g_ref[nt:], tol, "MLP grads")


def test_upstream_gradients_with_opacity():
    print("test_upstream_gradients_with_opacity", flush=True)
    from paper_2503_01582_amd import api
    arch, params, b, geo, model, samp = case(512)
    rng = np.random.default_rng(7)
    d = [rng.normal(size=s).astype(np.float32) for s in ((512, 3), 512, 512)]
    ws = api.Workspace().get(arch, 512, samp.t.shape[1])
    api.prenom_render_fwd(model, samp, None, ws, want_loss=False)
    api.prenom_render_bwd(model, samp, None, ws, d_rgb=torch.as_tensor(d[0]).cuda(),
                          d_depth=torch.as_tensor(d[1]).cuda(), d_opacity=torch.as_tensor(d[2]).cuda())
    torch.cuda.synchronize()
    g_ref = orc.render_bwd(arch, params, *geo, d_rgb=d[0], d_depth=d[1], d_opacity=d[2])
    check_grads(arch, model.grads.cpu().numpy(), g_ref)


@pytest.mark.parametrize("recompute", [False, True])
def test_autograd_function_matches_oracle(recompute):
    """A loss written in torch (colour MSE + 0.1 depth MSE on object rays,
    depth targets with 1 cm noise) back-propagated through PrenomRender equals
    the oracle's gradient of the same loss."""
    print(f"test_autograd_function_matches_oracle[recompute={recompute}]", flush=True)
    from paper_2503_01582_amd.autograd import render
    arch, params, b, geo, model, samp = case(1024)
    model.params.requires_grad_(True)
    rgb, depth, _ = render(model, samp, None, recompute)
    tgt = torch.as_tensor(b.tgt_rgb).cuda()
    tdep = torch.as_tensor(b.tgt_depth).cuda()
    m = torch.as_tensor(b.mask).cuda().float()
    n = b.n_rays
    loss = ((rgb - tgt) ** 2).sum() / (3 * n) + 0.1 * (m * (depth - tdep) ** 2).sum() / n
    loss.backward()
    g = model.params.grad.cpu().numpy()
    g_ref = orc.render_bwd(arch, params, *geo, tgt_rgb=b.tgt_rgb, tgt_depth=b.tgt_depth,
                           mask=b.mask, lambda_d=0.1)
    check_grads(arch, g, g_ref)


def test_recompute_equals_store_and_holds_less_memory():
    print("test_recompute_equals_store_and_holds_less_memory", flush=True)
    from paper_2503_01582_amd.autograd import render
    arch, params, b, geo, model, samp = case(8192)
    model.params.requires_grad_(True)
    held, grads = {}, {}
    for recompute in (False, True):
        model.params.grad = None
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        rgb, depth, _ = render(model, samp, None, recompute)
        torch.cuda.synchronize()
        held[recompute] = torch.cuda.memory_allocated() - base
        ((rgb - torch.as_tensor(b.tgt_rgb).cuda()) ** 2).sum().backward()
        grads[recompute] = model.params.grad.cpu().numpy()
    print(f"  memory held between forward and backward: store {held[False] / 2**20:.1f} MiB, "
          f"recompute {held[True] / 2**20:.1f} MiB", flush=True)
    assert held[True] < 0.1 * held[False]
    check_grads(arch, grads[True], grads[False], tol=1e-6)


# ---------------------------------------------------------------- the differentiation workload at size
N_FULL = 1 << 18       # rays of the differentiation workload (64 samples each)
N_CHECK = 256          # rays the oracle follows

_full = None


def full_case():
    """2^18 rays x 64 samples of the prior scene, depth targets with 1 cm
    Gaussian noise; geometry from the oracle's sampler (the same FP32 inputs
    for both sides)."""
    global _full
    if _full is None:
        from synth.workloads import prior_world as pw
        b = prior_batch(pw(seed=1), N_FULL, step=3, depth_noise=0.01, loss=LossSpec(lambda_d=0.1))
        s = b.sample
        ref = orc.sample(b.rays_o, b.rays_d, b.xi, n_coarse=s.n_coarse, n_fine=s.n_fine,
                         include_coarse=s.include_coarse, uniform_only=s.uniform_only, eps=s.eps,
                         near=s.near, far=s.far, world_to_obj=b.world_to_obj, prior=b.prior)
        geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
               ref["dt"].astype(np.float32), ref["flags"])
        _full = (b, geo)
    return _full


@pytest.mark.parametrize("recompute", [False, True])
def test_autograd_full_size_matches_oracle(recompute):
    """The differentiation workload at its size: a loss written in torch
    through PrenomRender over all 2^18 rays, with its terms weighted so that
    only 256 sampled rays carry gradient (colour MSE + 0.1 depth MSE on
    object rays, both normalised by the whole batch); the parameter gradient
    against the oracle's gradient of the same loss over those rays.  Sampled
    rays whose oracle ReLU pattern changes under 1e-6 relative parameter
    perturbations (FP32 rounding then decides a unit's state) are not
    picked; their share is bounded."""
    print(f"test_autograd_full_size_matches_oracle[recompute={recompute}]", flush=True)
    from paper_2503_01582_amd import api
    from paper_2503_01582_amd.autograd import render
    b, geo = full_case()
    arch = ARCH_LARGE
    params = init_params(arch, 5)
    params[:arch.n_table_params] = np.random.default_rng(6).uniform(
        -0.3, 0.3, arch.n_table_params).astype(np.float32)
    rng = np.random.default_rng(11)
    cand = np.sort(rng.choice(N_FULL, 2 * N_CHECK, replace=False))
    gsub = tuple(x[cand] for x in geo)
    stable = relu_stable_rays(arch, params, gsub, rng)
    share = 1.0 - stable.mean()
    pick = cand[stable][:N_CHECK]
    print(f"  {100 * share:.2f}% of {cand.size} candidate rays near a ReLU kink; {pick.size} checked", flush=True)
    assert share <= MAX_KINK_SHARE and pick.size == N_CHECK
    model = api.Model(arch, params)
    model.params.requires_grad_(True)
    samp = api.SampleOut(*(torch.as_tensor(g).cuda() for g in geo[:3]),
                         bins=torch.zeros((N_FULL, 1), dtype=torch.int32, device="cuda"),
                         flags=torch.as_tensor(geo[3]).cuda())
    sel = np.zeros(N_FULL, np.float32)
    sel[pick] = 1.0
    w = torch.as_tensor(sel).cuda()
    tgt = torch.as_tensor(b.tgt_rgb).cuda()
    tdep = torch.as_tensor(b.tgt_depth).cuda()
    m = torch.as_tensor(b.mask).cuda().float()
    rgb, depth, _ = render(model, samp, None, recompute)
    loss = (w[:, None] * (rgb - tgt) ** 2).sum() / (3 * N_FULL) + 0.1 * (w * m * (depth - tdep) ** 2).sum() / N_FULL
    loss.backward()
    torch.cuda.synchronize()
    g = model.params.grad.cpu().numpy()
    # the oracle's gradient of the same loss over the picked rays (its own forward gives the upstream terms)
    gp = tuple(x[pick] for x in geo)
    ref = orc.render_fwd(arch, params, *gp)
    d_rgb = (2.0 * (ref["rgb"] - b.tgt_rgb[pick]) / (3 * N_FULL)).astype(np.float32)
    d_depth = (0.2 * b.mask[pick] * (ref["depth"] - b.tgt_depth[pick]) / N_FULL).astype(np.float32)
    g_ref = orc.render_bwd(arch, params, *gp, d_rgb=d_rgb, d_depth=d_depth)
    got_rgb = rgb.detach().cpu().numpy()[pick]
    assert_close(got_rgb, ref["rgb"], 1e-5, "rgb of the picked rays")
    check_grads(arch, g, g_ref)
    print(f"  rgb and gradients within 1e-5 (held between forward and backward: "
          f"{'nothing' if recompute else 'features'})", flush=True)


def test_autograd_training_200_steps_store_and_recompute():
    """The differentiation workload trained for 200 steps through
    PrenomRender (colour MSE + 0.1 depth MSE against depths with 1 cm noise,
    then Adam), once storing the features between forward and backward and
    once recomputing them chunk by chunk.  At the same parameters the two
    give the same gradient (to 1e-6: the chunked backward adds each chunk's
    table-gradient tile sums and MLP partials separately, so FP32 rounding
    differs); both losses fall, and the two runs end within 10% of each
    other's loss (Adam with eps = 1e-15 turns gradient rounding on entries
    whose gradient is near zero into steps of up to lr, so the parameters
    themselves drift apart while the fit does not)."""
    print("test_autograd_training_200_steps_store_and_recompute", flush=True)
    from paper_2503_01582_amd.autograd import render
    from paper_2503_01582_amd.trainer import AutogradTrainer, to_device
    b, geo = full_case()
    arch = ARCH_LARGE
    params = init_params(arch, 0)
    db = to_device(b)
    # the first step's gradient, stored against recomputed features
    from paper_2503_01582_amd import api
    samp = api.SampleOut(*(torch.as_tensor(g).cuda() for g in geo[:3]),
                         bins=torch.zeros((N_FULL, 1), dtype=torch.int32, device="cuda"),
                         flags=torch.as_tensor(geo[3]).cuda())
    grads = {}
    for recompute in (False, True):
        model = api.Model(arch, params)
        model.params.requires_grad_(True)
        rgb, depth, _ = render(model, samp, None, recompute)
        m = db.mask.float()
        loss = ((rgb - db.tgt_rgb) ** 2).sum() / (3 * N_FULL) + 0.1 * (m * (depth - db.tgt_depth) ** 2).sum() / N_FULL
        loss.backward()
        grads[recompute] = model.params.grad.cpu().numpy().astype(np.float64)
        del model
    check_grads(arch, grads[True], grads[False], tol=1e-6)
    losses = {}
    for recompute in (False, True):
        tr = AutogradTrainer(arch, params, b.sample, b.loss, recompute=recompute)
        hist = []
        for step in range(200):
            out = tr.step(db)
            if step % 50 == 0 or step == 199:
                hist.append(float(out["loss"].item()))
        torch.cuda.synchronize()
        losses[recompute] = hist
        print(f"  recompute={recompute}: loss every 50 steps {['%.3e' % v for v in hist]}", flush=True)
        del tr
    for rec in (False, True):
        assert losses[rec][-1] < 0.01 * losses[rec][0], losses[rec]
    rel = abs(losses[True][-1] - losses[False][-1]) / losses[False][-1]
    print(f"  final loss store {losses[False][-1]:.4e}, recompute {losses[True][-1]:.4e} ({100 * rel:.1f}% apart)",
          flush=True)
    assert rel <= 0.1, rel
