"""The adjoint behind torch.autograd.Function, upstream-gradient mode with an
opacity term, and recompute versus store."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as orc
from parity_util import assert_close
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
