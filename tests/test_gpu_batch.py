"""Batched multi-object step on the GPU: every object of the map trained at
once (Fig. 1, Sec. IV-A), one launch per phase over objects with different
architectures, priors, poses and ray counts.

Checked against
  * the FP64 oracle, object by object (bins and flags exact, FP32 outputs and
    gradients within 1e-5, reduced-precision objects within 2e-3);
  * the single-object calls on the same inputs (identical per-sample
    arithmetic: forward outputs bit-exact, gradients to FP32 summation order);
  * itself, replayed from a captured HIP graph, step after step.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle as orc
from parity_util import MAX_KINK_SHARE, TOL_FP32, assert_close, rel_errors, relu_stable_rays
from test_gpu_precision import lowp_ok
from synth.arch import Arch
from synth.multi import multi_batch, multi_objects
from synth.params import init_params
from synth.workloads import PRIOR_SAMPLE, LossSpec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL_LOWP = 2e-3

# (L, log2 T, W, D) per object: every level count, width (the 128-wide MLP runs
# its backward as separate chain and weight-gradient kernels) and depth, hashed
# and dense levels; ray counts ragged, one object without rays, one without a
# prior.
ARCHS = [(8, 14, 64, 1), (12, 15, 32, 2), (16, 15, 128, 2), (8, 16, 32, 1), (16, 14, 32, 1),
         (12, 14, 128, 1), (8, 15, 64, 2)]
COUNTS = [300, 0, 129, 777, 1, 1100, 65]
NO_PRIOR = 3


def say(*a):
    print(*a, flush=True)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def make_objects(seed=11, mlp_dtype="fp32", table_dtype="fp32", counts=COUNTS):
    objs = multi_objects(seed, len(ARCHS), n_cams=4, width=160, height=120, pool_stride=2)
    out = []
    for o, (L, T, W, D), n in zip(objs, ARCHS, counts):
        arch = Arch(n_levels=L, log2_table=T, width=W, hidden=D, mlp_dtype=mlp_dtype, table_dtype=table_dtype)
        out.append(dataclasses.replace(o, arch=arch, n_rays=n))
    return out


def object_params(objs, seed=7):
    ps = []
    for i, o in enumerate(objs):
        p = init_params(o.arch, seed + i)
        rng = np.random.default_rng(seed + 100 + i)
        p[:o.arch.n_table_params] = rng.uniform(-0.3, 0.3, o.arch.n_table_params).astype(np.float32)
        ps.append(p)
    return ps


def batch_objects(objs):
    from paper_2503_01582_amd.batch import BatchObject
    return [BatchObject(o.arch, o.n_rays, None if i == NO_PRIOR else dev(o.prior), o.world_to_obj)
            for i, o in enumerate(objs)]


def oracle_object_sample(o, b, sl, i, spec=PRIOR_SAMPLE):
    return orc.sample(b.rays_o[sl], b.rays_d[sl], b.xi[sl], n_coarse=spec.n_coarse, n_fine=spec.n_fine,
                      include_coarse=spec.include_coarse, uniform_only=spec.uniform_only, eps=spec.eps,
                      near=spec.near, far=spec.far, world_to_obj=o.world_to_obj,
                      prior=None if i == NO_PRIOR else o.prior)


def test_batch_sampler_matches_oracle():
    say("test_batch_sampler_matches_oracle: 7 objects, own priors and poses")
    from paper_2503_01582_amd import batch as B
    objs = make_objects()
    b = multi_batch(objs, step=3)
    bm = B.BatchModel(batch_objects(objs), object_params(objs))
    ws = B.alloc_workspace(bm, PRIOR_SAMPLE.n_samples)
    out = B.prenom_batch_sample(bm, PRIOR_SAMPLE, dev(b.rays_o), dev(b.rays_d), dev(b.xi), ws)
    torch.cuda.synchronize()
    got = {k: getattr(out, k).cpu().numpy() for k in ("ray_obj", "t", "dt", "bins", "flags")}
    for i, o in enumerate(objs):
        sl = b.slice(i)
        if o.n_rays == 0:
            continue
        ref = oracle_object_sample(o, b, sl, i)
        np.testing.assert_array_equal(got["flags"][sl], ref["flags"], err_msg=f"object {i} flags")
        np.testing.assert_array_equal(got["bins"][sl], ref["bins"], err_msg=f"object {i} bins")
        live = (ref["flags"] & orc.FLAG_MISS) == 0
        if live.any():
            span = (ref["t"][:, -1] - ref["t"][:, 0])[live][:, None]
            ulp = np.spacing(np.abs(ref["t"][live]).astype(np.float32)).astype(np.float64)
            excess = np.abs(got["t"][sl][live] - ref["t"][live]) - ulp
            assert np.all(excess <= TOL_FP32 * span), (i, (excess / span).max())
        assert_close(got["dt"][sl], ref["dt"], name=f"object {i} dt")
        assert_close(got["ray_obj"][sl], ref["ray_obj"], name=f"object {i} ray_obj")
        if i == NO_PRIOR:
            assert np.all(ref["flags"] & orc.FLAG_UNIFORM)
        say(f"  object {i}: {o.n_rays} rays, {live.sum()} live, bins exact")


def oracle_geometry(objs, b):
    """Per-object oracle samples, concatenated in batch order (FP32)."""
    parts = [oracle_object_sample(o, b, b.slice(i), i) for i, o in enumerate(objs) if o.n_rays > 0]
    cat = lambda k: np.concatenate([p[k] for p in parts]) if parts else None
    return (cat("ray_obj").astype(np.float32).reshape(-1, 6), cat("t").astype(np.float32).reshape(-1, 64),
            cat("dt").astype(np.float32).reshape(-1, 64), cat("flags").astype(np.uint8))


class BatchRun:
    def __init__(self, objs, params, b, geo, loss, tiles=None, loss_scale=None, record_budget=0):
        from paper_2503_01582_amd import api
        from paper_2503_01582_amd import batch as B
        self.B = B
        self.bm = B.BatchModel(batch_objects(objs), params, tiles=tiles, loss_scale=loss_scale,
                               record_budget=record_budget)
        self.ws = B.alloc_workspace(self.bm, geo[1].shape[1])
        self.samp = api.SampleOut(ray_obj=dev(geo[0]), t=dev(geo[1]), dt=dev(geo[2]),
                                  bins=torch.zeros((geo[1].shape[0], 1), dtype=torch.int32, device="cuda"),
                                  flags=dev(geo[3]))
        self.loss = loss
        self.kw = dict(tgt_rgb=dev(b.tgt_rgb), tgt_depth=dev(b.tgt_depth), mask=dev(b.mask))

    def fwd(self):
        out = self.B.prenom_batch_render_fwd(self.bm, self.samp, self.loss, self.ws, **self.kw)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def bwd(self, recompute=False, d_rgb=None, d_depth=None):
        self.bm.grads.zero_()
        up = {} if d_rgb is None else dict(d_rgb=dev(d_rgb), d_depth=dev(d_depth))
        self.B.prenom_batch_render_bwd(self.bm, self.samp, self.loss, self.ws, recompute=recompute, **self.kw, **up)
        torch.cuda.synchronize()
        return [self.bm.object_grads(i).cpu().numpy() for i in range(len(self.bm.objs))]


# record budgets: one scatter pass over all objects; one pass per object (1
# byte); two passes, objects 0-4 and 5-6 (64 MiB)
@pytest.mark.parametrize("recompute,record_budget", [(False, 0), (True, 0), (False, 1), (True, 64 << 20)])
def test_batch_render_matches_oracle(recompute, record_budget):
    say(f"test_batch_render_matches_oracle[recompute={recompute}, record_budget={record_budget}]")
    objs = make_objects()
    params = object_params(objs)
    b = multi_batch(objs, step=5, depth_noise=0.01)
    geo = oracle_geometry(objs, b)
    loss = LossSpec(lambda_d=0.1, lambda_sigma=0.01)
    run = BatchRun(objs, params, b, geo, loss, record_budget=record_budget)
    got = run.fwd()
    if recompute:  # the workspace must not be needed between the calls
        run.ws[:] = 0
        run.B.prenom_batch_prepare(run.bm, 64, run.ws)
    grads = run.bwd(recompute)
    for i, o in enumerate(objs):
        sl = b.slice(i)
        if o.n_rays == 0:
            assert got["loss"][i] == 0.0 and not np.any(grads[i])
            continue
        g = tuple(x[sl] for x in geo)
        ref = orc.render_fwd(o.arch, params[i], *g, tgt_rgb=b.tgt_rgb[sl], tgt_depth=b.tgt_depth[sl],
                             mask=b.mask[sl], lambda_d=np.float32(0.1), lambda_sigma=np.float32(0.01))
        g_ref = orc.render_bwd(o.arch, params[i], *g, tgt_rgb=b.tgt_rgb[sl], tgt_depth=b.tgt_depth[sl],
                               mask=b.mask[sl], lambda_d=np.float32(0.1), lambda_sigma=np.float32(0.01))
        for k in ("rgb", "depth", "opacity"):
            assert_close(got[k][sl], ref[k], name=f"object {i} {k}")
        assert abs(got["loss"][i] - ref["loss"]) <= TOL_FP32 * abs(ref["loss"]), (i, got["loss"][i], ref["loss"])
        nt = o.arch.n_table_params
        e_t = assert_close(grads[i][:nt], g_ref[:nt], name=f"object {i} table grads")
        e_m = assert_close(grads[i][nt:], g_ref[nt:], name=f"object {i} MLP grads")
        say(f"  object {i} ({o.arch.n_levels}x2^{o.arch.log2_table}, W{o.arch.width} D{o.arch.hidden}, "
            f"{o.n_rays} rays): loss {got['loss'][i]:.6e}, grads {e_t[0]:.1e}/{e_m[0]:.1e}")


def test_batch_equals_single_object_calls():
    """Same samples through prenom_render_* object by object: the forward is
    bit-exact, the table gradient agrees to 1e-6 (its fixed-point sums do not
    depend on order), the MLP gradient to FP32 summation order (1e-5).  Tile
    shapes other than the defaults give the same results."""
    say("test_batch_equals_single_object_calls")
    from paper_2503_01582_amd import api
    objs = make_objects(counts=[2000, 0, 1500, 777, 3, 4100, 650])
    params = object_params(objs)
    b = multi_batch(objs, step=9)
    geo = oracle_geometry(objs, b)
    loss = LossSpec(lambda_d=0.1)
    tiles = [dict(in_dim=o.arch.in_dim, width=o.arch.width, hidden=o.arch.hidden, dtype="fp32", fwd_tiles=12,
                  bwd_tiles=96) for o in objs]
    for tl in (None, tiles):
        run = BatchRun(objs, params, b, geo, loss, tiles=tl)
        got = run.fwd()
        grads = run.bwd()
        for i, o in enumerate(objs):
            if o.n_rays == 0:
                continue
            sl = b.slice(i)
            m = api.Model(o.arch, params[i])
            samp = api.SampleOut(*(dev(x[sl]) for x in geo[:3]),
                                 bins=torch.zeros((o.n_rays, 1), dtype=torch.int32, device="cuda"),
                                 flags=dev(geo[3][sl]))
            ws = api.Workspace().get(o.arch, o.n_rays, 64)
            kw = dict(tgt_rgb=dev(b.tgt_rgb[sl]), tgt_depth=dev(b.tgt_depth[sl]), mask=dev(b.mask[sl]))
            out = api.prenom_render_fwd(m, samp, loss, ws, **kw)
            api.prenom_render_bwd(m, samp, loss, ws, **kw)
            torch.cuda.synchronize()
            for k in ("rgb", "depth", "opacity"):
                np.testing.assert_array_equal(got[k][sl], out[k].cpu().numpy(), err_msg=f"object {i} {k}")
            assert abs(got["loss"][i] - out["loss"].item()) <= 1e-6 * abs(out["loss"].item())
            g1 = m.grads.cpu().numpy()
            nt = o.arch.n_table_params
            assert_close(grads[i][:nt], g1[:nt], tol=1e-6, name=f"object {i} table grads")
            # the MLP gradient's FP32 partial sums run over different sample blocks
            assert_close(grads[i][nt:], g1[nt:], tol=1e-5, name=f"object {i} MLP grads")
        say(f"  tiles {'default' if tl is None else 'fwd 12 / bwd 40'}: batch == single-object calls")


def test_backward_repeats_after_one_forward():
    """The backward only reads what the forward left in the workspace (the
    tile histograms of the table gradient included): two backward calls after
    one forward add the same gradient twice, batched and single-object."""
    say("test_backward_repeats_after_one_forward")
    from paper_2503_01582_amd import api
    objs = make_objects(counts=[900, 0, 400, 777, 3, 1100, 65])
    params = object_params(objs)
    b = multi_batch(objs, step=3)
    geo = oracle_geometry(objs, b)
    loss = LossSpec(lambda_d=0.1)
    run = BatchRun(objs, params, b, geo, loss)
    run.fwd()
    g1 = run.bwd()
    run.B.prenom_batch_render_bwd(run.bm, run.samp, run.loss, run.ws, **run.kw)
    torch.cuda.synchronize()
    for i, o in enumerate(objs):
        if o.n_rays:
            assert_close(run.bm.object_grads(i).cpu().numpy(), 2 * g1[i], tol=1e-6, name=f"object {i} grads")
    i = 5
    sl = b.slice(i)
    m = api.Model(objs[i].arch, params[i])
    samp = api.SampleOut(*(dev(x[sl]) for x in geo[:3]),
                         bins=torch.zeros((objs[i].n_rays, 1), dtype=torch.int32, device="cuda"),
                         flags=dev(geo[3][sl]))
    ws = api.Workspace().get(objs[i].arch, objs[i].n_rays, 64)
    kw = dict(tgt_rgb=dev(b.tgt_rgb[sl]), tgt_depth=dev(b.tgt_depth[sl]), mask=dev(b.mask[sl]))
    api.prenom_render_fwd(m, samp, loss, ws, **kw)
    api.prenom_render_bwd(m, samp, loss, ws, **kw)
    torch.cuda.synchronize()
    one = m.grads.cpu().numpy().copy()
    assert np.any(one[:objs[i].arch.n_table_params])
    api.prenom_render_bwd(m, samp, loss, ws, **kw)
    torch.cuda.synchronize()
    assert_close(m.grads.cpu().numpy(), 2 * one, tol=1e-6, name="single-object grads")
    say("  second backward after one forward: gradient added twice")


def test_batch_adam_device_step():
    """One Adam launch over the batch; bias corrections from the device step
    counter match the oracle's host-step Adam on every object."""
    say("test_batch_adam_device_step")
    from paper_2503_01582_amd import batch as B
    objs = make_objects()
    params = object_params(objs)
    bm = B.BatchModel(batch_objects(objs), params)
    rng = np.random.default_rng(3)
    p_ref = [p.astype(np.float64) for p in params]
    m_ref = [np.zeros_like(p) for p in p_ref]
    v_ref = [np.zeros_like(p) for p in p_ref]
    hp = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15)
    for step in (1, 2, 3):
        gs = [rng.normal(0, 1e-3, p.shape).astype(np.float32) for p in params]
        for i, g in enumerate(gs):
            bm.object_grads(i).copy_(torch.as_tensor(g))
        B.prenom_batch_adam_step(bm, **hp)
        for i, g in enumerate(gs):
            p_ref[i], m_ref[i], v_ref[i] = orc.adam(p_ref[i].astype(np.float32), g, m_ref[i].astype(np.float32),
                                                    v_ref[i].astype(np.float32), step=step, **hp)
    torch.cuda.synchronize()
    assert int(bm.step.item()) == 3
    for i in range(len(objs)):
        assert_close(bm.object_params(i).cpu().numpy(), p_ref[i], name=f"object {i} params")
        assert not torch.any(bm.object_grads(i)).item()


def test_batch_graph_replay_matches_eager():
    """A captured step replayed three times, with eager torch work and
    synchronisations between replays, reproduces three eager steps."""
    say("test_batch_graph_replay_matches_eager")
    from paper_2503_01582_amd.batch import BatchTrainer
    objs = make_objects(counts=[900, 0, 300, 640, 7, 2000, 100])
    params = object_params(objs)
    tr = BatchTrainer(batch_objects(objs), params, PRIOR_SAMPLE, LossSpec(lambda_d=0.1))
    batches = [multi_batch(objs, step=20 + k) for k in range(3)]
    m = tr.model
    state0 = [t.clone() for t in (m.params, m.grads, m.adam_m, m.adam_v, m.step)]
    eager = []
    for bt in batches:
        tr.load(bt)
        out = tr.step()
        torch.cuda.synchronize()
        eager.append((out["loss"].cpu().numpy().copy(), m.params.cpu().numpy().copy()))
    for t, s in zip((m.params, m.grads, m.adam_m, m.adam_v, m.step), state0):
        t.copy_(s)
    torch.cuda.synchronize()
    tr.capture()
    for k, bt in enumerate(batches):
        tr.load(bt)
        scratch = torch.randn(1024, device="cuda")  # unrelated eager work between replays
        (scratch * 2).sum().item()
        tr.replay()
        torch.cuda.synchronize()
        loss, p = tr.out["loss"].cpu().numpy(), m.params.cpu().numpy()
        e_l = rel_errors(loss, eager[k][0])
        e_p = rel_errors(p, eager[k][1])
        say(f"  replay {k}: loss rel {e_l[0]:.1e}, params rel {e_p[0]:.1e}, step {int(m.step.item())}")
        assert e_l[0] <= 1e-6 and e_p[0] <= 1e-6
        assert int(m.step.item()) == k + 1


@pytest.mark.parametrize("mlp_dtype,table_dtype", [("bf16", "fp16"), ("fp16", "fp16")])
def test_batch_reduced_precision(mlp_dtype, table_dtype):
    """Objects in the reduced-precision form: bit-exact against the
    single-object reduced-precision calls, within 2e-3 of the oracle that
    emulates the reduced-precision method in both norms (the plain FP64
    comparison is reported by test_gpu_precision); gradients through random
    upstream gradients on each object's ReLU-stable rays
    (parity_util.relu_stable_rays)."""
    say(f"test_batch_reduced_precision[{mlp_dtype}, table {table_dtype}]")
    from paper_2503_01582_amd import api
    objs = make_objects(mlp_dtype=mlp_dtype, table_dtype=table_dtype, counts=[600, 0, 200, 500, 5, 900, 80])
    params = object_params(objs)
    b = multi_batch(objs, step=13)
    geo = oracle_geometry(objs, b)
    loss = LossSpec(lambda_d=0.1)
    scale = 4096.0
    run = BatchRun(objs, params, b, geo, loss, loss_scale=scale)
    got = run.fwd()
    rng = np.random.default_rng(17)
    n = b.tgt_rgb.shape[0]
    d_rgb, d_depth = np.zeros((n, 3), np.float32), np.zeros(n, np.float32)
    for i, o in enumerate(objs):
        if o.n_rays == 0:
            continue
        sl = b.slice(i)
        keep = relu_stable_rays(o.arch, params[i], tuple(x[sl] for x in geo), rng, emulate=True)
        assert o.n_rays - keep.sum() <= max(1, MAX_KINK_SHARE * o.n_rays), (i, o.n_rays - keep.sum())
        d_rgb[sl][keep] = rng.normal(size=(int(keep.sum()), 3))
        d_depth[sl][keep] = rng.normal(size=int(keep.sum()))
    grads = run.bwd(d_rgb=d_rgb, d_depth=d_depth)
    worst = {}
    for i, o in enumerate(objs):
        if o.n_rays == 0:
            continue
        sl = b.slice(i)
        m = api.Model(o.arch, params[i])
        samp = api.SampleOut(*(dev(x[sl]) for x in geo[:3]),
                             bins=torch.zeros((o.n_rays, 1), dtype=torch.int32, device="cuda"),
                             flags=dev(geo[3][sl]))
        ws = api.Workspace().get(o.arch, o.n_rays, 64)
        out = api.prenom_render_fwd(m, samp, loss, ws, tgt_rgb=dev(b.tgt_rgb[sl]), tgt_depth=dev(b.tgt_depth[sl]),
                                    mask=dev(b.mask[sl]))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got["rgb"][sl], out["rgb"].cpu().numpy(), err_msg=f"object {i} rgb")
        g = tuple(x[sl] for x in geo)
        kw = dict(tgt_rgb=b.tgt_rgb[sl], tgt_depth=b.tgt_depth[sl], mask=b.mask[sl], lambda_d=np.float32(0.1),
                  emulate=True)
        ref = orc.render_fwd(o.arch, params[i], *g, **kw)
        g_ref = orc.render_bwd(o.arch, params[i], *g, loss_scale=scale, d_rgb=d_rgb[sl], d_depth=d_depth[sl], **kw)
        nt = o.arch.n_table_params
        gi = grads[i].astype(np.float64) / scale
        errs = {"rgb": rel_errors(got["rgb"][sl], ref["rgb"]), "depth": rel_errors(got["depth"][sl], ref["depth"]),
                "loss": rel_errors([got["loss"][i]], [ref["loss"]]),
                "g_table": rel_errors(gi[:nt], g_ref[:nt]), "g_mlp": rel_errors(gi[nt:], g_ref[nt:])}
        for k, v in errs.items():
            worst[k] = (max(worst.get(k, (0, 0))[0], v[0]), max(worst.get(k, (0, 0))[1], v[1]))
            assert lowp_ok(k, v), (i, k, v)
    say("  worst per output vs the emulating oracle: " +
        ", ".join(f"{k} {v[0]:.1e}/{v[1]:.1e}" for k, v in worst.items()))
