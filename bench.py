"""Training-step throughput of the per-object NeRF step on one MI355X.

Workloads (--workload):
  headline (default) the target comparison: batch48 with the MLP in BF16
          (graph-replayed) against prior (FP32, one object), both timed in
          the same run; value = batch48 rays/s, the ratio in
          config.speedup_vs_fp32_single_object, and the held-out PSNR of the
          reduced-precision forms against FP32 after 500 steps (three seeds,
          from the committed summary of that test run) beside it.
  prior   one object, prior-based sampling: 65536 rays per step
          drawn from 16 cameras at 640x480 around a random 3-ellipsoid
          object, 16 coarse + 48 inverse-CDF samples per ray (64 rendered),
          hash grid 16 levels x 2^19 x 2 features, MLP 64 x 2 hidden, FP32,
          mean-squared colour loss, Adam.  A step is prenom_sample +
          prenom_render_fwd (fused loss) + prenom_render_bwd +
          prenom_adam_step on resident inputs.  Also timed, outside the
          step: the prior refresh over the 64^3 grid, which runs once every
          50 steps, and the canonical yaw search (360 yaws) of the object's
          depth cloud, which runs once per object.
  autograd the differentiation configuration: the prior scene at 2^18 rays
          x 64 samples, colour + 0.1 x depth MSE (1 cm depth noise) in torch
          on top of PrenomRender, Adam; store vs recompute, with peak memory.
  batch24 24 objects trained together (own scene, prior, pose, log-uniform
          ray count in [1k, 64k], architecture drawn from L {8,12,16},
          T 2^14..2^19, W {32,64,128}, D {1,2}), FP32, one launch per phase,
          the step captured in a HIP graph, MLP tiles from the autotuner;
          also timed: the same objects as 24 single-object steps in turn.
  batch48 48 objects, 2^20 rays in all, MLP in BF16 (--mlp-dtype) on the
          matrix cores with FP32 accumulation, FP16 table copy, dynamic loss
          scaling from 2^12; otherwise as batch24.
  reptile meta-training of a synthetic category's initial parameters: a
          step is one meta-iteration, q = 8 inner gradient-descent steps of
          8 tasks x 4096 rays x 32 uniform samples trained together (12
          levels x 2^17, MLP 64 x 2), then the outer update; value = inner-
          loop rays/s.

Prints one JSON line: rays/s, the roofline position of the dominant kernel
and, for the headline and prior workloads, the FP64 CPU oracle timed on a
bounded sample (single thread and every host CPU).  The timed steps run
without instrumentation; per-kernel times come from a separate pass of the
same steps in which every launch sits between two HIP events on its stream
(eager steps for the batched workloads, whose timed steps are graph
replays).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
LOWP_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
METRIC = "training rays/s (fwd+bwd) vs plain FP32 at equal PSNR; % HBM/MFMA roofline"
# The hash-table gradient is one operation run as six dependent kernels
# (k_scatter_count, _level_max, _scan_blocks, _scan_tiles, _place, _reduce);
# its algorithmic bytes belong to the group, timed as the sum of the six.
SCATTER_GROUP = "k_scatter_* (hash-table gradient)"


def algorithmic_work(arch, n_rays, S, n_fine):
    """Algorithmic bytes (HBM-bound kernels) or FLOPs (MLP) of one step's
    kernels for one object.  Counting rule: every value the kernel must read
    or write once, each hash-grid corner access as one table row (2 x FP32,
    or 2 x FP16 when the forward reads the FP16 copy)."""
    n_s = n_rays * S
    L = arch.n_levels
    in_dim, W, D = arch.in_dim, arch.width, arch.hidden
    macs = W * in_dim + (D - 1) * W * W + 4 * W
    row_fwd = 4 if getattr(arch, "table_dtype", "fp32") == "fp16" else 8
    pos = 4 + 24.0 / S               # t, plus the ray's origin/direction shared by S samples
    return {
        "k_sample": ("hbm", n_rays * (24 + 4 * n_fine + 8 * S + 4 * n_fine + 1 + 24)),
        "k_encode_fwd": ("hbm", n_s * (pos + L * (8 * row_fwd + 8))),
        "k_mlp_fwd": ("mfma", n_s * 2.0 * macs),
        "k_composite_fwd": ("hbm", n_s * 24 + n_rays * (12 + 4 + 4 + 32 + 12 + 4 + 1)),
        "k_composite_bwd": ("hbm", n_s * 40 + n_rays * (32 + 12 + 4 + 1)),
        "k_mlp_bwd": ("mfma", n_s * 6.0 * macs),
        SCATTER_GROUP: ("hbm", n_s * (pos + L * (8 * 8 + 8))),
        "k_adam": ("hbm", arch.n_params * (32 + (2 if getattr(arch, "table_dtype", "fp32") == "fp16" else 0))),
    }


def refresh_work(arch, n):
    """Algorithmic work of one prior refresh over n grid vertices: every
    level's 8 corner rows and its 2 features written (the vertex comes from
    the thread index, nothing else is read), the MLP forward, and the
    density column (a 16-byte head row read, 4 bytes written)."""
    L = arch.n_levels
    in_dim, W, D = arch.in_dim, arch.width, arch.hidden
    macs = W * in_dim + (D - 1) * W * W + 4 * W
    return {"k_encode_grid": ("hbm", n * L * (8 * 8 + 8)),
            "k_mlp_fwd": ("mfma", n * 2.0 * macs),
            "k_density_grid": ("hbm", n * 20.0)}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_prior_65536rays.md")


def measured_traffic(kernel: str, summary: str = TRAFFIC_SUMMARY):
    """HBM bytes per step of `kernel` from a committed counter summary (the
    fenced json block of a profiles/hbm_traffic_*.md file), or None when there
    is none or a source it was measured with has changed since."""
    import hashlib
    try:
        text = open(summary).read()
        block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    entry = block.get("kernels", {}).get(kernel)
    if not entry:
        return None
    for rel, digest in entry.get("sources", {}).items():
        try:
            if hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest() != digest:
                return None
        except OSError:
            return None
    return entry.get("hbm_bytes_per_step")


def summed_work(items):
    """Sum of algorithmic_work over (arch, n_rays, S, n_fine) items."""
    tot = {}
    for it in items:
        for k, (bound, amount) in algorithmic_work(*it).items():
            tot[k] = (bound, tot.get(k, (bound, 0.0))[1] + amount)
    return tot


def kernel_table(kt, steps, ms_per_step, work, mlp_peak, log):
    """Per kernel: time per step, share of the step and, where its
    algorithmic work is known, achieved rate vs the MI355X peak."""
    kern = {}
    kt = dict(kt)
    parts = {k: v for k, v in kt.items() if k.startswith("k_scatter_")}
    if parts:
        kt[SCATTER_GROUP] = (max(v[0] for v in parts.values()), sum(v[1] for v in parts.values()))
    for name, (n, tot) in sorted(kt.items(), key=lambda kv: -kv[1][1]):
        per_step = tot / steps
        entry = dict(avg_ms=tot / n, ms_per_step=per_step, launches_per_step=n / steps, share=per_step / ms_per_step)
        if name in work:
            bound, amount = work[name]
            if bound == "hbm":
                entry.update(bound="hbm", achieved=amount / (per_step * 1e-3) / 1e9, unit="GB/s", peak=HBM_PEAK_GBS)
            else:
                entry.update(bound="mfma", achieved=amount / (per_step * 1e-3) / 1e12, unit="TFLOP/s", peak=mlp_peak)
            entry["frac"] = entry["achieved"] / entry["peak"]
        kern[name] = entry
        log(f"  {name:34s} {per_step * 1e3:9.1f} us/step ({n / steps:.0f} launches)  {100 * entry['share']:5.1f}%  "
            + (f"{entry['achieved']:8.1f} {entry['unit']} ({100 * entry['frac']:.1f}% of peak)"
               if "frac" in entry else ""))
    dom = max((k for k in kern if "frac" in kern[k]), key=lambda k: kern[k]["ms_per_step"])
    d = kern[dom]
    roofline = dict(kernel=dom, bound=d["bound"], achieved=round(d["achieved"], 2), peak=d["peak"],
                    unit=d["unit"], frac=round(d["frac"], 4), traffic=None)
    kern = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()} for k, v in kern.items()}
    return kern, roofline


def cpu_model():
    """Host CPU model name and the number of CPUs this process may use."""
    name = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                name = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def oracle_step_seconds(batch, params, n_sample_rays):
    """FP64 oracle on the first n_sample_rays rays of the batch: (seconds of
    the per-ray work -- sample, forward + loss, backward --, seconds of Adam
    over every parameter)."""
    import oracle as orc
    s = batch.sample
    sel = slice(0, n_sample_rays)
    t0 = time.perf_counter()
    o = orc.sample(batch.rays_o[sel], batch.rays_d[sel], batch.xi[sel], n_coarse=s.n_coarse,
                   n_fine=s.n_fine, include_coarse=s.include_coarse, uniform_only=s.uniform_only,
                   eps=s.eps, near=s.near, far=s.far, world_to_obj=batch.world_to_obj,
                   prior=batch.prior)
    geo = (o["ray_obj"].astype(np.float32), o["t"].astype(np.float32), o["dt"].astype(np.float32),
           o["flags"])
    kw = dict(tgt_rgb=batch.tgt_rgb[sel], tgt_depth=batch.tgt_depth[sel], mask=batch.mask[sel])
    orc.render_fwd(batch.arch, params, *geo, **kw)
    g = orc.render_bwd(batch.arch, params, *geo, **kw)
    t1 = time.perf_counter()
    z = np.zeros_like(params)
    orc.adam(params, g.astype(np.float32), z, z, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=1)
    return t1 - t0, time.perf_counter() - t1


def cpu_baseline(batch, params, n_sample_rays):
    """The FP64 oracle (untuned) on the host cores: the per-ray work of a
    sub-batch of n_sample_rays rays of the single-object prior workload, plus
    Adam over all its parameters, once on one thread and once on every CPU
    this process may use.  Rays/s of a whole batch, extrapolated linearly in
    rays (the per-ray work is linear in rays; Adam is counted once)."""
    import oracle as orc
    model, ncpu = cpu_model()
    res = {}
    for threads in (1, ncpu):
        orc.set_threads(threads)
        log(f"bench: CPU oracle, {n_sample_rays} rays, {threads} thread(s)")
        t_rays, t_adam = oracle_step_seconds(batch, params, n_sample_rays)
        step_s = t_rays * batch.n_rays / n_sample_rays + t_adam
        res[threads] = (batch.n_rays / step_s, t_rays, t_adam)
        log(f"bench:   {t_rays:.2f} s per-ray work, {t_adam:.2f} s Adam -> {batch.n_rays / step_s:.1f} rays/s")
    orc.set_threads(ncpu)
    v1, r1, a1 = res[1]
    vn, rn, an = res[ncpu]
    return dict(value=round(vn, 1), unit="rays/s", cores=orc.max_threads(), kind="oracle",
                single_thread_value=round(v1, 1), cpu_model=model, nproc=ncpu,
                sample=f"{n_sample_rays} of the {batch.n_rays} rays of one batch of the single-object prior "
                       f"workload (sample, forward + loss, backward: {rn:.2f} s on {ncpu} threads, {r1:.2f} s on "
                       f"one), plus Adam over all {batch.arch.n_params} parameters ({an:.2f} s / {a1:.2f} s), "
                       f"FP64; rays/s of the whole {batch.n_rays}-ray step, extrapolated linearly in rays")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_loop(step, steps):
    """Runs `steps` steps between two events on the current stream; returns ms."""
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def copy_calibration():
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("bench: copied 1 GiB device-to-device for counter calibration")


def run_refresh(tr, arch, ms_per_step, R=64, reps=20, m=50):
    """The prior refresh (the NeRF's density over the R^3 grid, recomputed
    every m training steps) timed on its own, and its cost spread over the
    m steps it serves."""
    import torch
    from paper_2503_01582_amd import api
    tr.refresh_prior(R)
    torch.cuda.synchronize()
    log(f"bench: prior refresh, R = {R}, {reps} calls")
    api.prenom_profile_begin()
    ms = timed_loop(lambda: tr.refresh_prior(R), reps) / reps
    kt = api.prenom_profile_end()
    kern, roof = kernel_table(kt, reps, ms, refresh_work(arch, R ** 3), FP32_MFMA_PEAK_TFLOPS, log)
    share = ms / (m * ms_per_step)
    log(f"bench: refresh {ms:.3f} ms per call, {100 * share:.2f}% of the {m} steps it serves")
    return dict(R=R, ms=round(ms, 4), vertices_per_s=round(R ** 3 / (ms * 1e-3), 1), every_m_steps=m,
                amortised_share=round(share, 5), dominant=roof, kernels=kern)


YAW_OPS = 71  # FP64 operations per (point, yaw): turn (x2), extents, normalise, trilinear weights and sum


def run_canon(world, batch, K=360, reps=20):
    """The canonical yaw search (Eq. (3)) on the object's depth cloud (the
    batch's object rays at their true depth, in the object frame) against
    the prior grid, timed on its own; FP64 ALU work counted as YAW_OPS per
    (point, yaw)."""
    import torch
    from paper_2503_01582_amd import api
    m = batch.mask == 1
    P = (batch.rays_o[m] + batch.tgt_depth[m, None] * batch.rays_d[m]).astype(np.float32)
    pts = torch.as_tensor(P).cuda()
    prior = torch.as_tensor(world.prior).cuda()
    api.prenom_canonical_yaw(pts, prior, K)
    torch.cuda.synchronize()
    log(f"bench: canonical yaw search, {P.shape[0]} points x {K} yaws, {reps} calls")
    api.prenom_profile_begin()
    ms = timed_loop(lambda: api.prenom_canonical_yaw(pts, prior, K), reps) / reps
    kt = api.prenom_profile_end()
    kms = kt["k_canonical_yaw"][1] / kt["k_canonical_yaw"][0]
    tflops = YAW_OPS * P.shape[0] * K / (kms * 1e-3) / 1e12
    log(f"bench: yaw search {ms:.3f} ms per call (kernels {kms:.3f} ms), {tflops:.2f} TFLOP/s FP64")
    return dict(points=int(P.shape[0]), yaws=K, ms=round(ms, 4), kernel_ms=round(kms, 4),
                lookups_per_s=round(P.shape[0] * K / (kms * 1e-3), 1),
                roofline=dict(bound="alu", achieved=round(tflops, 3), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4)))


def run_prior(args):
    import torch
    from paper_2503_01582_amd import api
    from paper_2503_01582_amd.trainer import Trainer, to_device
    from synth.params import init_params
    from synth.workloads import prior_batch, prior_world

    log("bench: building the synthetic scene and batch")
    world = prior_world(seed=1)
    batch = prior_batch(world, args.rays, step=0)
    arch = batch.arch
    params = init_params(arch, 0)
    tr = Trainer(arch, params, batch.sample, batch.loss)
    db = to_device(batch)
    S = batch.sample.n_samples
    log(f"bench: {args.warmup} warm-up steps")
    for _ in range(args.warmup):
        tr.step(db)
    torch.cuda.synchronize()
    log(f"bench: {args.steps} timed steps")
    t0 = time.perf_counter()
    ms = timed_loop(lambda: tr.step(db), args.steps)
    wall = time.perf_counter() - t0
    ms_per_step = ms / args.steps
    value = args.rays * args.steps / (ms / 1e3)
    log(f"bench: {ms_per_step:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), "
        f"loss {float(tr._out['loss'].item()):.4e}")
    # per-kernel times: the same steps again, each launch between two HIP events
    prof_steps = max(3, min(args.steps, 20))
    api.prenom_profile_begin()
    ms_prof = timed_loop(lambda: tr.step(db), prof_steps)
    kt = api.prenom_profile_end()
    if args.copy_calibration:
        copy_calibration()
    log(f"bench: {ms_prof / prof_steps:.3f} ms/step with per-launch events ({prof_steps} steps)")
    kern, roofline = kernel_table(kt, prof_steps, ms_prof / prof_steps,
                                  algorithmic_work(arch, args.rays, S, batch.sample.n_fine), FP32_MFMA_PEAK_TFLOPS, log)
    if args.rays == 65536:
        roofline["traffic"] = measured_traffic(roofline["kernel"])
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, params, args.cpu_rays)
    config = dict(workload="prior-sampled object NeRF training step", n_rays=args.rays,
                  samples_per_ray=S, n_coarse=batch.sample.n_coarse, n_fine=batch.sample.n_fine,
                  hash_levels=arch.n_levels, log2_table=arch.log2_table, mlp_width=arch.width,
                  mlp_hidden=arch.hidden, samples_per_s=round(value * S, 1))
    extra = {}
    if not args.no_extras:
        extra = dict(prior_refresh=run_refresh(tr, arch, ms_per_step), canonical_yaw=run_canon(world, batch))
    return value, ms_per_step, "fp32", config, roofline, kern, cpu, extra


def held_between_passes(tr, db):
    """Device memory allocated by one forward through PrenomRender and still
    held when its backward starts (one untimed step)."""
    import torch
    from paper_2503_01582_amd.autograd import render
    samp = tr.sample(db)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    rgb, depth, _ = render(tr.model, samp, db.bg, tr.recompute)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    ((rgb - db.tgt_rgb) ** 2).sum().backward()
    tr.model.params.grad = None
    torch.cuda.synchronize()
    return held


def run_autograd(args):
    """The differentiation configuration: the prior workload's scene at 2^18
    rays x 64 samples, colour MSE plus 0.1 x depth MSE against depths with
    1 cm Gaussian noise, written in torch on top of PrenomRender (the
    hand-written adjoint behind torch.autograd.Function), then Adam.  Timed
    with the features kept between forward and backward (store) and rebuilt
    in the backward (recompute); peak device memory of each."""
    import torch
    from paper_2503_01582_amd import api
    from paper_2503_01582_amd.trainer import AutogradTrainer, to_device
    from synth.params import init_params
    from synth.workloads import LossSpec, prior_batch, prior_world

    n_rays = 1 << 18
    log("bench: building the synthetic scene and batch")
    world = prior_world(seed=1)
    loss = LossSpec(lambda_d=0.1)
    batch = prior_batch(world, n_rays, step=0, depth_noise=0.01, loss=loss)
    arch = batch.arch
    params = init_params(arch, 0)
    db = to_device(batch)
    S = batch.sample.n_samples
    modes, kt = {}, None
    for recompute in (False, True):
        name = "recompute" if recompute else "store"
        torch.cuda.empty_cache()
        tr = AutogradTrainer(arch, params, batch.sample, loss, recompute=recompute)
        log(f"bench: {name}: {args.warmup} warm-up steps")
        for _ in range(args.warmup):
            tr.step(db)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        log(f"bench: {name}: {args.steps} timed steps")
        if recompute:
            api.prenom_profile_begin()
        ms = timed_loop(lambda: tr.step(db), args.steps)
        if recompute:
            kt = api.prenom_profile_end()
        peak = torch.cuda.max_memory_allocated()
        held = held_between_passes(tr, db)
        modes[name] = dict(ms_per_step=round(ms / args.steps, 4),
                           rays_per_s=round(n_rays * args.steps / (ms / 1e3), 1),
                           peak_mib=round(peak / 2**20, 1), held_between_passes_mib=round(held / 2**20, 1))
        log(f"bench: {name}: {ms / args.steps:.3f} ms/step, peak {peak / 2**20:.0f} MiB, "
            f"held between forward and backward {held / 2**20:.0f} MiB")
        del tr
    ms_per_step = modes["recompute"]["ms_per_step"]
    kern, roofline = kernel_table(kt, args.steps, ms_per_step,
                                  algorithmic_work(arch, n_rays, S, batch.sample.n_fine), FP32_MFMA_PEAK_TFLOPS, log)
    config = dict(workload="differentiable rendering step through torch.autograd (recompute)", n_rays=n_rays,
                  samples_per_ray=S, hash_levels=arch.n_levels, log2_table=arch.log2_table, mlp_width=arch.width,
                  mlp_hidden=arch.hidden, lambda_d=0.1, depth_noise_m=0.01,
                  samples_per_s=round(n_rays / (ms_per_step / 1e3) * S, 1))
    return modes["recompute"]["rays_per_s"], ms_per_step, "fp32", config, roofline, kern, None, dict(modes=modes)


def run_batch(args, n_objects, total_rays, mlp_dtype, table_dtype, seed):
    import dataclasses
    import torch
    from paper_2503_01582_amd import api, autotune
    from paper_2503_01582_amd.batch import BatchObject, BatchTrainer
    from paper_2503_01582_amd.trainer import Trainer
    from synth.multi import multi_batch, multi_objects
    from synth.params import init_params
    from synth.workloads import PRIOR_SAMPLE, LossSpec

    log(f"bench: building {n_objects} objects")
    objs = multi_objects(seed, n_objects, total_rays=total_rays, mlp_dtype=mlp_dtype, table_dtype=table_dtype)
    n_rays = sum(o.n_rays for o in objs)
    S = PRIOR_SAMPLE.n_samples
    b = multi_batch(objs, step=0)
    params = [init_params(o.arch, i) for i, o in enumerate(objs)]
    priors = [torch.as_tensor(o.prior).cuda() for o in objs]
    bobjs = [BatchObject(o.arch, o.n_rays, p, o.world_to_obj) for o, p in zip(objs, priors)]
    tiles = autotune.tiles_for([o.arch for o in objs])
    if len(tiles) < len({(o.arch.in_dim, o.arch.width, o.arch.hidden) for o in objs}) and not args.no_tune:
        log("bench: tuning MLP tile shapes (no cached entry for every shape)")
        tiles = autotune.tune([o.arch for o in objs], log=log)
    loss = LossSpec()
    lowp = mlp_dtype != "fp32"
    tr = BatchTrainer(bobjs, params, PRIOR_SAMPLE, loss, tiles=tiles, loss_scale=4096.0 if lowp else None)
    tr.load(b)
    log(f"bench: {n_rays} rays over {n_objects} objects, {len(tr.model.params) / 1e6:.1f} M parameters; "
        f"{args.warmup} eager warm-up steps")
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    # per-kernel times from eager steps (events cannot live inside the graph)
    api.prenom_profile_begin()
    prof_steps = max(3, min(args.steps, 10))
    ms_eager = timed_loop(tr.step, prof_steps)
    kt = api.prenom_profile_end()
    tr.capture()
    for _ in range(3):
        tr.replay()
    log(f"bench: {args.steps} timed graph replays")
    t0 = time.perf_counter()
    ms = timed_loop(tr.replay, args.steps)
    wall = time.perf_counter() - t0
    if args.copy_calibration:
        copy_calibration()
    ms_per_step = ms / args.steps
    value = n_rays * args.steps / (ms / 1e3)
    log(f"bench: {ms_per_step:.3f} ms/step replayed ({wall / args.steps * 1e3:.3f} ms wall), "
        f"{ms_eager / prof_steps:.3f} ms/step eager; mean loss {float(tr.out['loss'].mean().item()):.4e}")
    work = summed_work([(o.arch, o.n_rays, S, PRIOR_SAMPLE.n_fine) for o in objs])
    kern, roofline = kernel_table(kt, prof_steps, ms_eager / prof_steps, work,
                                  LOWP_MFMA_PEAK_TFLOPS if lowp else FP32_MFMA_PEAK_TFLOPS, log)
    extra = dict(eager_ms_per_step=round(ms_eager / prof_steps, 4))
    if not args.no_sequential:
        # the same objects and rays as single-object steps, one after another on one stream
        log("bench: the same objects as single-object steps in turn")
        del tr
        torch.cuda.empty_cache()
        from paper_2503_01582_amd.trainer import DeviceBatch
        trainers, dbs = [], []
        for i, o in enumerate(objs):
            if o.n_rays == 0:
                continue
            sl = b.slice(i)
            t = Trainer(o.arch, params[i], PRIOR_SAMPLE, loss, loss_scale=4096.0 if lowp else None)
            dev = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)
            dbs.append(DeviceBatch(rays_o=dev(b.rays_o[sl]), rays_d=dev(b.rays_d[sl]), xi=dev(b.xi[sl]),
                                   tgt_rgb=dev(b.tgt_rgb[sl]), tgt_depth=dev(b.tgt_depth[sl]),
                                   mask=dev(b.mask[sl], torch.uint8), world_to_obj=o.world_to_obj,
                                   prior=priors[i], bg=None))
            trainers.append(t)

        def seq_step():
            for t, d in zip(trainers, dbs):
                t.step(d)
        for _ in range(max(2, args.warmup // 2)):
            seq_step()
        seq_steps = max(3, args.steps // 2)
        ms_seq = timed_loop(seq_step, seq_steps) / seq_steps
        extra.update(sequential_ms_per_step=round(ms_seq, 4), sequential_rays_per_s=round(n_rays / (ms_seq / 1e3), 1),
                     speedup_vs_sequential=round(ms_seq / ms_per_step, 3))
        log(f"bench: sequential single-object steps {ms_seq:.3f} ms/step -> batched speed-up "
            f"{ms_seq / ms_per_step:.2f}x")
    arch_mix = {}
    for o in objs:
        k = f"L{o.arch.n_levels} T2^{o.arch.log2_table} W{o.arch.width} D{o.arch.hidden}"
        arch_mix[k] = arch_mix.get(k, 0) + 1
    config = dict(workload=f"{n_objects} objects trained together, graph-captured step", n_objects=n_objects,
                  n_rays=n_rays, samples_per_ray=S, mlp_dtype=mlp_dtype, table_dtype=table_dtype,
                  loss_scale_init=4096.0 if lowp else None, tiles=tiles, architectures=arch_mix,
                  samples_per_s=round(value * S, 1))
    return value, ms_per_step, mlp_dtype if lowp else "fp32", config, roofline, kern, None, extra


def run_reptile(args):
    """Meta-training (Reptile, Eq. (1)-(2)) of a synthetic category: a step is
    one meta-iteration, q inner gradient-descent steps of B tasks trained
    together, then the outer update."""
    import torch
    from paper_2503_01582_amd import api
    from paper_2503_01582_amd.meta import ReptileTrainer
    from synth.arch import Arch
    from synth.category import category_pools, stratification
    from synth.params import init_params
    from synth.workloads import LossSpec, SampleSpec, nocs_affine

    arch = Arch(n_levels=12, log2_table=17, width=64, hidden=2)
    spec = SampleSpec(n_coarse=0, n_fine=32, include_coarse=False, uniform_only=True)
    B, q, n, lr, beta = 8, 8, 4096, 80.0, 0.5
    log(f"bench: {2 * B} instances of a synthetic category, {B} tasks per meta-iteration, q = {q}")
    pools = category_pools(2, 2 * B, 8 * n)
    dev = {f: torch.stack([torch.as_tensor(getattr(p, f)) for p in pools]).cuda()
           for f in ("rays_o", "rays_d", "tgt_rgb", "tgt_depth", "mask")}
    xi = torch.as_tensor(stratification(7, 0, 8 * n, spec.n_fine)).cuda()
    tr = ReptileTrainer(arch, init_params(arch, 0), B, n, spec, LossSpec(), inner_lr=lr, beta=beta,
                        world_to_obj=nocs_affine().reshape(3, 4))
    ids_all = [torch.as_tensor([(i * B + b) % (2 * B) for b in range(B)]).cuda() for i in range(2)]
    state = dict(i=0)

    def meta_iteration():
        i = state["i"]
        ids = ids_all[i % 2]
        for k in range(q):
            sl = slice(k * n, (k + 1) * n)
            tr.load_rays(dev["rays_o"][ids, sl].reshape(-1, 3), dev["rays_d"][ids, sl].reshape(-1, 3),
                         xi[sl].repeat(B, 1), dev["tgt_rgb"][ids, sl].reshape(-1, 3),
                         dev["tgt_depth"][ids, sl].reshape(-1), dev["mask"][ids, sl].reshape(-1))
            tr.step()
        tr.outer()
        state["i"] = i + 1

    for _ in range(args.warmup):
        meta_iteration()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 5)
    log(f"bench: {steps} timed meta-iterations")
    api.prenom_profile_begin()
    ms = timed_loop(meta_iteration, steps)
    kt = api.prenom_profile_end()
    ms_per_step = ms / steps
    rays = B * n * q
    value = rays / (ms_per_step * 1e-3)
    log(f"bench: {ms_per_step:.3f} ms per meta-iteration ({rays} inner-loop rays), "
        f"last inner loss {float(tr.out['loss'].mean()):.4e}")
    work = {k: (b, a * q) for k, (b, a) in summed_work([(arch, n, spec.n_samples, spec.n_fine)] * B).items()
            if k != "k_adam"}
    work["k_sgd"] = ("hbm", 16.0 * B * arch.n_params * q)
    work["k_reptile"] = ("hbm", 8.0 * (B + 1) * arch.n_params)
    kern, roofline = kernel_table(kt, steps, ms_per_step, work, FP32_MFMA_PEAK_TFLOPS, log)
    config = dict(workload="Reptile meta-training of a synthetic category (one meta-iteration per step)",
                  n_tasks=B, inner_steps=q, rays_per_task=n, samples_per_ray=spec.n_samples, inner_lr=lr,
                  meta_step_size=beta, hash_levels=arch.n_levels, log2_table=arch.log2_table, mlp_width=arch.width,
                  mlp_hidden=arch.hidden)
    extra = dict(reptile_update=kern.get("k_reptile"))
    return value, ms_per_step, "fp32", config, roofline, kern, None, extra


PSNR_SUMMARY = os.path.join(ROOT, "profiles", "psnr_batch48_2p20rays_500steps.md")
HEADLINE_TRAFFIC = os.path.join(ROOT, "profiles", "hbm_traffic_batch48_2p20rays.md")


def held_psnr_delta():
    """Mean held-out PSNR of the 48-object reduced-precision forms minus the
    FP32 form after 500 steps, three seeds (fenced json block of the
    committed summary of that test's run), or None."""
    try:
        text = open(PSNR_SUMMARY).read()
        return json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None


def run_headline(args):
    """The target comparison: the 48-object batched step with the MLP in
    BF16 (FP16 table copy, FP32 gradients and masters, loss scaling),
    graph-replayed, against the plain FP32 single-object step of the prior
    workload, both timed in this run without per-launch instrumentation."""
    import torch
    args.no_sequential = True
    value, ms, dtype, config, roofline, kern, _, extra = run_batch(args, 48, 1 << 20, args.mlp_dtype, "fp16", seed=5)
    roofline["traffic"] = measured_traffic(roofline["kernel"], HEADLINE_TRAFFIC)
    torch.cuda.empty_cache()
    args.no_extras = True
    v32, ms32, _, cfg32, roof32, _, cpu, _ = run_prior(args)
    ratio = value / v32
    log(f"bench: batched {args.mlp_dtype} {value / 1e6:.2f} M rays/s vs FP32 single object {v32 / 1e6:.2f} M rays/s: "
        f"{ratio:.3f}x")
    config["compared_with"] = dict(workload=cfg32["workload"] + " (FP32, one object)", n_rays=cfg32["n_rays"],
                                   ms_per_step=round(ms32, 4), rays_per_s=round(v32, 1),
                                   dominant=roof32)
    config["speedup_vs_fp32_single_object"] = round(ratio, 4)
    config["psnr_vs_fp32_after_500_steps"] = held_psnr_delta()
    extra = dict(extra, speedup_vs_fp32_single_object=round(ratio, 4))
    return value, ms, dtype, config, roofline, kern, cpu, extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=("headline", "prior", "autograd", "batch24", "batch48", "reptile"),
                    default="headline")
    ap.add_argument("--mlp-dtype", choices=("bf16", "fp16"), default="bf16", help="headline and batch48")
    ap.add_argument("--rays", type=int, default=65536, help="prior workload only")
    ap.add_argument("--cpu-rays", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true", help="batch workloads: skip the sequential comparison")
    ap.add_argument("--no-tune", action="store_true", help="batch workloads: library default tiles if none cached")
    ap.add_argument("--no-extras", action="store_true",
                    help="prior workload: skip the prior-refresh and yaw-search timings after the step (so that a "
                         "counter run sees only the step's launches)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device once (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); nothing here uses a "
              "second GPU", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "headline":
        res = run_headline(args)
    elif args.workload == "prior":
        res = run_prior(args)
    elif args.workload == "autograd":
        res = run_autograd(args)
    elif args.workload == "reptile":
        res = run_reptile(args)
    elif args.workload == "batch24":
        res = run_batch(args, 24, None, "fp32", "fp32", seed=4)
    else:
        res = run_batch(args, 48, 1 << 20, args.mlp_dtype, "fp16", seed=5)
    value, ms_per_step, dtype, config, roofline, kern, cpu, extra = res
    line = dict(metric=METRIC, value=round(value, 1), unit="rays/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype=dtype, data="synthetic", config=config, roofline=roofline,
                kernels=kern, cpu_baseline=cpu)
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
