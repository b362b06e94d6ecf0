"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs.  Integer outputs (sampled bins, flags, hash rows) must match exactly;
floating-point outputs within 1e-5 (max-norm and 2-norm relative, per tensor).
Inputs of the rendering stages come from the oracle's own sampler (rounded to
FP32 as the kernels receive them), never from the GPU."""
from __future__ import annotations

import functools
import sys

import numpy as np
import pytest

import oracle as orc
from parity_util import TOL_FP32, assert_close
from synth.arch import ARCH_LARGE, ARCH_SMALL, Arch
from synth.params import init_params
from synth.workloads import (LossSpec, SampleSpec, prior_batch, prior_world,
                             small_batch, uniform_xi)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def world():
    return prior_world(seed=1, pool_stride=5)


def api():
    from paper_2503_01582_amd import api as A
    return A


def dev(a, dtype=None):
    if a is None:
        return None
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def oracle_sample(b, spec=None):
    s = spec or b.sample
    return orc.sample(b.rays_o, b.rays_d, b.xi[:, :s.n_fine], n_coarse=s.n_coarse, n_fine=s.n_fine,
                      include_coarse=s.include_coarse, uniform_only=s.uniform_only, eps=s.eps,
                      near=s.near, far=s.far, world_to_obj=b.world_to_obj, prior=b.prior)


def gpu_sample(b, spec=None):
    s = spec or b.sample
    A = api()
    out = A.prenom_sample(s, dev(b.rays_o), dev(b.rays_d), dev(b.xi[:, :s.n_fine]), b.world_to_obj,
                          dev(b.prior) if b.prior is not None else None)
    torch.cuda.synchronize()
    return {k: getattr(out, k).cpu().numpy() for k in ("ray_obj", "t", "dt", "bins", "flags")}


def check_sampler(b, spec=None):
    ref = oracle_sample(b, spec)
    got = gpu_sample(b, spec)
    np.testing.assert_array_equal(got["flags"], ref["flags"])
    np.testing.assert_array_equal(got["bins"], ref["bins"])
    live = (ref["flags"] & orc.FLAG_MISS) == 0
    # depths: within 1e-5 of each ray's sampled span, plus the FP32 rounding
    # of the output itself (one ulp of t)
    span = (ref["t"][:, -1] - ref["t"][:, 0])[live][:, None]
    ulp = np.spacing(np.abs(ref["t"][live]).astype(np.float32)).astype(np.float64)
    excess = np.abs(got["t"][live] - ref["t"][live]) - ulp
    assert np.all(excess <= TOL_FP32 * span), (excess / span).max()
    assert np.all(got["t"][~live] == 0) and np.all(got["dt"][~live] == 0)
    assert_close(got["dt"], ref["dt"], name="dt")
    assert_close(got["ray_obj"], ref["ray_obj"], name="ray_obj")
    margin = ref["margin"][np.isfinite(ref["margin"])]
    say(f"  sampler: {live.sum()} live rays, min FP64 decision margin "
        f"{margin.min() if margin.size else float('inf'):.3e}")
    return ref, got


# ---------------------------------------------------------------- sampler

def test_sample_uniform_small():
    say("test_sample_uniform_small: 4096 rays, 32 uniform samples")
    ref, _ = check_sampler(small_batch(0))
    assert np.all(ref["bins"] == -1)


def test_sample_prior_bins_exact():
    say("test_sample_prior_bins_exact: 8192 rays, 16 coarse + 48 CDF draws")
    b = prior_batch(world(), 8192, step=0)
    ref, _ = check_sampler(b)
    assert (ref["bins"] >= 0).mean() > 0.9


def test_sample_escape_miss_and_ragged():
    say("test_sample_escape_miss_and_ragged: zero prior, S = 7 + 17, 1037 rays")
    b = prior_batch(world(), 1037, step=3)
    spec = SampleSpec(n_coarse=7, n_fine=17, include_coarse=True, uniform_only=False)
    check_sampler(b, spec)
    b.prior = np.zeros_like(b.prior)
    ref, _ = check_sampler(b, spec)
    assert np.all(ref["flags"] == orc.FLAG_ESCAPED)
    # rays that miss the box
    sb = small_batch(1)
    sb.prior = b.prior[:8, :8, :8].copy() + 1.0
    sb.sample = SampleSpec(n_coarse=5, n_fine=9, include_coarse=False, uniform_only=False)
    ref, _ = check_sampler(sb)
    assert (ref["flags"] & orc.FLAG_MISS).any()


def test_sample_max_sizes():
    say("test_sample_max_sizes: N_c = N_r = 128 merged (S = 256)")
    b = prior_batch(world(), 256, step=5)
    b.xi = uniform_xi(np.random.default_rng(0), 256, 128)
    check_sampler(b, SampleSpec(n_coarse=128, n_fine=128, include_coarse=True, uniform_only=False))


# ---------------------------------------------------------------- encoding

@pytest.mark.parametrize("arch", [ARCH_SMALL, ARCH_LARGE], ids=["small", "large"])
def test_encode_indices_exact(arch):
    say(f"test_encode_indices_exact: L={arch.n_levels} T=2^{arch.log2_table}")
    rng = np.random.default_rng(21)
    pos = [rng.uniform(0, 1, (20000, 3))]
    for N in arch.resolutions:  # lattice planes and their FP32 neighbours
        k = rng.integers(0, N + 1, 64)
        v = (k / N).astype(np.float32)
        for vv in (v, np.nextafter(v, np.float32(0)), np.nextafter(v, np.float32(1))):
            p = rng.uniform(0, 1, (64, 3)).astype(np.float32)
            p[:, rng.integers(0, 3)] = vv
            pos.append(p)
    pos = np.clip(np.concatenate(pos).astype(np.float32), 0, 1)
    table = init_params(arch, 4)[:arch.n_table_params] * 1e3
    y_ref, idx_ref, _ = orc.encode(arch, table, pos, with_corners=True)
    y, idx = api().prenom_encode(arch, dev(table), dev(pos), with_corners=True)
    np.testing.assert_array_equal(idx.cpu().numpy(), idx_ref)
    assert_close(y.cpu().numpy(), y_ref, name="features")


# ---------------------------------------------------------------- rendering

def render_case(kind, n_rays=None):
    """(arch, params, batch, oracle samples as FP32 geometry, loss spec)."""
    if kind == "small":
        b = small_batch(2)
        arch = ARCH_SMALL
    else:
        b = prior_batch(world(), n_rays or 1024, step=1)
        arch = ARCH_LARGE
    params = init_params(arch, 7)
    rng = np.random.default_rng(8)
    # larger table values than the init so the field is not nearly constant
    params[:arch.n_table_params] = rng.uniform(-0.3, 0.3, arch.n_table_params).astype(np.float32)
    ref = oracle_sample(b)
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
           ref["dt"].astype(np.float32), ref["flags"])
    return arch, params, b, geo


class GpuRender:
    def __init__(self, arch, params, geo, loss=None):
        A = api()
        self.A = A
        self.model = A.Model(arch, params)
        ray_obj, t, dt, flags = geo
        self.samp = A.SampleOut(ray_obj=dev(ray_obj), t=dev(t), dt=dev(dt),
                                bins=torch.zeros((t.shape[0], 1), dtype=torch.int32, device="cuda"),
                                flags=dev(flags))
        self.loss = loss or LossSpec()
        self.ws = A.Workspace().get(arch, t.shape[0], t.shape[1])

    def fwd(self, b, with_targets=True, bg=None):
        n, S = self.samp.t.shape
        so = torch.empty((n, S, 4), dtype=torch.float32, device="cuda")
        kw = {}
        if with_targets:
            kw = dict(tgt_rgb=dev(b.tgt_rgb), tgt_depth=dev(b.tgt_depth), mask=dev(b.mask))
        out = self.A.prenom_render_fwd(self.model, self.samp, self.loss, self.ws, bg=dev(bg),
                                       sample_out=so, **kw)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["samples"] = so.cpu().numpy()
        return res

    def bwd(self, b, d_rgb=None, d_depth=None, bg=None):
        self.model.grads.zero_()
        kw = dict(tgt_rgb=dev(b.tgt_rgb), tgt_depth=dev(b.tgt_depth), mask=dev(b.mask))
        self.A.prenom_render_bwd(self.model, self.samp, self.loss, self.ws, bg=dev(bg),
                                 d_rgb=dev(d_rgb), d_depth=dev(d_depth), **kw)
        torch.cuda.synchronize()
        return self.model.grads.cpu().numpy()


def oracle_fwd(arch, params, geo, b, loss=None, bg=None):
    loss = loss or LossSpec()
    return orc.render_fwd(arch, params, *geo, bg=bg, tgt_rgb=b.tgt_rgb, tgt_depth=b.tgt_depth,
                          mask=b.mask, loss_mode=loss.loss_mode, lambda_d=loss.lambda_d,
                          lambda_sigma=loss.lambda_sigma, want_samples=True)


def oracle_bwd(arch, params, geo, b, loss=None, bg=None, d_rgb=None, d_depth=None):
    loss = loss or LossSpec()
    return orc.render_bwd(arch, params, *geo, bg=bg, tgt_rgb=b.tgt_rgb, tgt_depth=b.tgt_depth,
                          mask=b.mask, d_rgb=d_rgb, d_depth=d_depth, loss_mode=loss.loss_mode,
                          lambda_d=loss.lambda_d, lambda_sigma=loss.lambda_sigma)


def check_fwd(got, ref, live):
    assert_close(got["rgb"], ref["rgb"], name="rgb")
    assert_close(got["depth"], ref["depth"], name="depth")
    assert_close(got["opacity"], ref["opacity"], name="opacity")
    assert_close(got["samples"][live], ref["samples"][live], name="sigma/rgb per sample")
    assert abs(got["loss"][0] - ref["loss"]) <= TOL_FP32 * abs(ref["loss"]), (got["loss"], ref["loss"])


def check_grads(arch, g, g_ref):
    nt = arch.n_table_params
    e_t = assert_close(g[:nt], g_ref[:nt], name="table grads")
    e_m = assert_close(g[nt:], g_ref[nt:], name="MLP grads")
    say(f"  grads: table {e_t[0]:.2e}/{e_t[1]:.2e}, mlp {e_m[0]:.2e}/{e_m[1]:.2e}")


@pytest.mark.parametrize("kind", ["small", "large"])
def test_render_fwd_bwd_parity(kind):
    say(f"test_render_fwd_bwd_parity[{kind}]")
    arch, params, b, geo = render_case(kind)
    live = (geo[3] & orc.FLAG_MISS) == 0
    gr = GpuRender(arch, params, geo)
    got = gr.fwd(b)
    ref = oracle_fwd(arch, params, geo, b)
    check_fwd(got, ref, live)
    say(f"  fwd ok: loss {got['loss'][0]:.6e} vs {ref['loss']:.6e}")
    check_grads(arch, gr.bwd(b), oracle_bwd(arch, params, geo, b))


@pytest.mark.parametrize("hidden", [1, 2])
def test_render_wide_mlp_parity(hidden):
    """128-wide MLP (stored activations, separate chain and weight-gradient
    kernels) against the oracle, on a ragged ray count."""
    say(f"test_render_wide_mlp_parity[hidden={hidden}]")
    b = prior_batch(world(), 777, step=3)
    arch = Arch(n_levels=16, log2_table=15, width=128, hidden=hidden)
    params = init_params(arch, 9)
    params[:arch.n_table_params] = np.random.default_rng(10).uniform(-0.3, 0.3, arch.n_table_params).astype(np.float32)
    ref = oracle_sample(b)
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32), ref["dt"].astype(np.float32), ref["flags"])
    live = (geo[3] & orc.FLAG_MISS) == 0
    gr = GpuRender(arch, params, geo)
    check_fwd(gr.fwd(b), oracle_fwd(arch, params, geo, b), live)
    check_grads(arch, gr.bwd(b), oracle_bwd(arch, params, geo, b))


@pytest.mark.parametrize("mode", [0, 1])
def test_render_loss_terms_and_background(mode):
    say(f"test_render_loss_terms_and_background[mode={mode}]")
    arch, params, b, geo = render_case("small")
    live = (geo[3] & orc.FLAG_MISS) == 0
    loss = LossSpec(loss_mode=mode, lambda_d=0.1, lambda_sigma=1e-3)
    bg = np.random.default_rng(3).uniform(0, 1, (b.n_rays, 3)).astype(np.float32)
    gr = GpuRender(arch, params, geo, loss)
    check_fwd(gr.fwd(b, bg=bg), oracle_fwd(arch, params, geo, b, loss, bg), live)
    check_grads(arch, gr.bwd(b, bg=bg), oracle_bwd(arch, params, geo, b, loss, bg))


def test_render_upstream_gradients():
    say("test_render_upstream_gradients")
    arch, params, b, geo = render_case("large", 512)
    rng = np.random.default_rng(4)
    d_rgb = rng.normal(size=(b.n_rays, 3)).astype(np.float32)
    d_depth = rng.normal(size=b.n_rays).astype(np.float32)
    gr = GpuRender(arch, params, geo)
    gr.fwd(b)
    check_grads(arch, gr.bwd(b, d_rgb=d_rgb, d_depth=d_depth),
                oracle_bwd(arch, params, geo, b, d_rgb=d_rgb, d_depth=d_depth))


def test_bindings_reject_per_ray_arrays_of_the_wrong_size():
    """The C ABI takes plain pointers; the Python binding checks every
    per-ray array against the ray and sample counts before any launch."""
    say("test_bindings_reject_per_ray_arrays_of_the_wrong_size")
    arch, params, b, geo = render_case("small")
    gr = GpuRender(arch, params, geo)
    A, n = gr.A, geo[1].shape[0]
    z = lambda *shape, dtype=torch.float32: torch.zeros(shape, dtype=dtype, device="cuda")
    with pytest.raises(ValueError):
        A.prenom_render_bwd(gr.model, gr.samp, gr.loss, gr.ws, d_rgb=z(n - 1, 3))
    with pytest.raises(ValueError):
        A.prenom_render_fwd(gr.model, gr.samp, gr.loss, gr.ws, tgt_rgb=z(n, 2))
    with pytest.raises(ValueError):
        A.prenom_render_fwd(gr.model, gr.samp, gr.loss, gr.ws, sample_out=z(n, geo[1].shape[1], 3))
    with pytest.raises(TypeError):
        A.prenom_render_fwd(gr.model, gr.samp, gr.loss, gr.ws, tgt_rgb=z(n, 3), mask=z(n))
    gr.fwd(b)  # the right sizes still go through


def test_backward_without_its_forward_adds_no_table_gradient():
    """A backward whose workspace holds no forward of these rays (here: every
    byte 0xff, so the tile histograms claim far more records than there are
    corners) must stay within its arrays: the scatter's check refuses the
    histograms and leaves the table gradient untouched.  A forward and
    backward afterwards give the gradient of a fresh workspace, bit for bit."""
    say("test_backward_without_its_forward_adds_no_table_gradient")
    arch, params, b, geo = render_case("small", 300)
    gr = GpuRender(arch, params, geo)
    gr.ws.fill_(0xFF)
    g = gr.bwd(b)
    assert not np.any(g[:arch.n_table_params]), "table gradient written from histograms no forward made"
    gr.fwd(b)
    g1 = gr.bwd(b)
    fresh = GpuRender(arch, params, geo)
    fresh.fwd(b)
    np.testing.assert_array_equal(g1, fresh.bwd(b))
    assert np.any(g1[:arch.n_table_params])


@pytest.mark.parametrize("nc,nr,n_rays", [(40, 60, 333), (128, 128, 96), (7, 17, 1037)])
def test_render_long_and_ragged_rays(nc, nr, n_rays):
    say(f"test_render_long_and_ragged_rays: S = {nc}+{nr}, {n_rays} rays")
    b = prior_batch(world(), n_rays, step=9)
    b.xi = uniform_xi(np.random.default_rng(5), n_rays, nr)
    b.sample = SampleSpec(n_coarse=nc, n_fine=nr, include_coarse=True, uniform_only=False)
    arch = ARCH_SMALL
    params = init_params(arch, 3)
    params[:arch.n_table_params] = np.random.default_rng(6).uniform(-0.3, 0.3, arch.n_table_params)
    ref = oracle_sample(b)
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
           ref["dt"].astype(np.float32), ref["flags"])
    live = (geo[3] & orc.FLAG_MISS) == 0
    loss = LossSpec(lambda_d=0.05)
    gr = GpuRender(arch, params, geo, loss)
    check_fwd(gr.fwd(b), oracle_fwd(arch, params, geo, b, loss), live)
    check_grads(arch, gr.bwd(b), oracle_bwd(arch, params, geo, b, loss))


def test_empty_batch():
    say("test_empty_batch")
    A = api()
    arch = ARCH_SMALL
    m = A.Model(arch, init_params(arch, 0))
    e = torch.empty((0, 3), device="cuda")
    spec = SampleSpec(n_coarse=0, n_fine=32, include_coarse=False, uniform_only=True)
    samp = A.prenom_sample(spec, e, e, torch.empty((0, 32), device="cuda"), np.eye(3, 4).ravel())
    ws = A.Workspace().get(arch, 0, 32)
    out = A.prenom_render_fwd(m, samp, LossSpec(), ws, tgt_rgb=e)
    A.prenom_render_bwd(m, samp, LossSpec(), ws, tgt_rgb=e)
    torch.cuda.synchronize()
    assert float(out["loss"].item()) == 0.0
    assert float(m.grads.abs().max().item()) == 0.0


# ---------------------------------------------------------------- Adam and the whole step

def test_adam_parity():
    say("test_adam_parity")
    A = api()
    arch = ARCH_SMALL
    rng = np.random.default_rng(9)
    n = arch.n_params
    p = rng.normal(size=n).astype(np.float32)
    g = (rng.normal(size=n) * 1e-3).astype(np.float32)
    g[rng.random(n) < 0.3] = 0.0
    m = (rng.normal(size=n) * 1e-3).astype(np.float32)
    v = (rng.random(n) * 1e-6).astype(np.float32)
    model = A.Model(arch, p)
    model.grads.copy_(torch.as_tensor(g))
    model.adam_m.copy_(torch.as_tensor(m))
    model.adam_v.copy_(torch.as_tensor(v))
    A.prenom_adam_step(model, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=5)
    torch.cuda.synchronize()
    po, mo, vo = orc.adam(p, g, m, v, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=5)
    assert_close(model.params.cpu().numpy(), po, name="params")
    assert_close(model.adam_m.cpu().numpy(), mo, name="m")
    assert_close(model.adam_v.cpu().numpy(), vo, name="v")
    assert float(model.grads.abs().max().item()) == 0.0  # consumed


@pytest.mark.parametrize("kind", ["small", "large"])
def test_full_step_parity(kind):
    """sample -> render_fwd -> render_bwd -> Adam on both sides, each from the
    same inputs; parameters after the step within tolerance of the oracle."""
    say(f"test_full_step_parity[{kind}]")
    from paper_2503_01582_amd.trainer import Trainer, to_device
    if kind == "small":
        b = small_batch(4)
        arch = ARCH_SMALL
    else:
        b = prior_batch(world(), 2048, step=2)
        arch = ARCH_LARGE
    params = init_params(arch, 1)
    tr = Trainer(arch, params, b.sample, b.loss)
    db = to_device(b)
    samp = tr.sample(db)
    out = tr.forward(db, samp)
    tr.backward(db, samp)
    g_gpu = tr.model.grads.cpu().numpy()
    api().prenom_adam_step(tr.model, **tr.adam)
    torch.cuda.synchronize()
    ref = oracle_sample(b)
    np.testing.assert_array_equal(samp.bins.cpu().numpy(), ref["bins"])
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
           ref["dt"].astype(np.float32), ref["flags"])
    fr = oracle_fwd(arch, params, geo, b)
    g = oracle_bwd(arch, params, geo, b)
    assert abs(out["loss"].item() - fr["loss"]) <= 1e-5 * fr["loss"]
    check_grads(arch, g_gpu, g)
    zeros = np.zeros(arch.n_params, np.float32)
    po, _, _ = orc.adam(params, g.astype(np.float32), zeros, zeros, lr=1e-2, beta1=0.9,
                        beta2=0.99, eps=1e-15, step=1)
    # Adam's first step is lr * g / |g|: compare where the gradient is well
    # above the FP32 noise floor, so its sign is not in question
    strong = np.abs(g) >= 1e-3 * np.abs(g).max()
    upd = tr.model.params.cpu().numpy().astype(np.float64) - params
    assert_close(upd[strong], (po - params)[strong], tol=1e-5, name="Adam update")
    say(f"  {strong.sum()} parameters with a strong gradient updated as the oracle")


# ---------------------------------------------------------------- full-size workload

def test_full_size_prior_workload():
    """2^16 rays x 64 samples, 16 levels x 2^19, MLP 64 x 2: the benchmark's
    launch configuration.  Bins of every ray exactly; rendering and gradients
    on 256 sampled rays (the oracle computes them one by one; the GPU gradient
    is restricted to them through upstream gradients that vanish elsewhere)."""
    say("test_full_size_prior_workload: 65536 rays x 64 samples")
    b = prior_batch(world(), 65536, step=11)
    ref, got = check_sampler(b)
    arch = ARCH_LARGE
    params = init_params(arch, 2)
    params[:arch.n_table_params] = np.random.default_rng(12).uniform(
        -0.3, 0.3, arch.n_table_params).astype(np.float32)
    geo = (ref["ray_obj"].astype(np.float32), ref["t"].astype(np.float32),
           ref["dt"].astype(np.float32), ref["flags"])
    gr = GpuRender(arch, params, geo)
    gf = gr.fwd(b)
    pick = np.sort(np.random.default_rng(13).choice(b.n_rays, 256, replace=False))
    sub = (geo[0][pick], geo[1][pick], geo[2][pick], geo[3][pick])
    rf = orc.render_fwd(arch, params, *sub, want_samples=True)
    assert_close(gf["rgb"][pick], rf["rgb"], name="rgb (sampled rays)")
    assert_close(gf["depth"][pick], rf["depth"], name="depth (sampled rays)")
    assert_close(gf["opacity"][pick], rf["opacity"], name="opacity (sampled rays)")
    live = (sub[3] & orc.FLAG_MISS) == 0
    assert_close(gf["samples"][pick][live], rf["samples"][live], name="samples")
    # the full-batch loss equals the mean-squared error of the GPU's own colours
    mse = ((gf["rgb"].astype(np.float64) - b.tgt_rgb) ** 2).sum() / (3 * b.n_rays)
    assert abs(gf["loss"][0] - mse) <= 1e-5 * mse
    rng = np.random.default_rng(14)
    d_rgb = np.zeros((b.n_rays, 3), np.float32)
    d_rgb[pick] = rng.normal(size=(256, 3))
    d_depth = np.zeros(b.n_rays, np.float32)
    d_depth[pick] = rng.normal(size=256)
    g = gr.bwd(b, d_rgb=d_rgb, d_depth=d_depth)
    g_ref = orc.render_bwd(arch, params, *sub, d_rgb=d_rgb[pick], d_depth=d_depth[pick])
    check_grads(arch, g, g_ref)
