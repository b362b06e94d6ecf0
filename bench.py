"""Training-step throughput of the per-object NeRF step on one MI355X.

Workload (prior-based sampling): 65536 rays per step drawn from 16 cameras at
640x480 around a random 3-ellipsoid object, 16 coarse + 48 inverse-CDF
samples per ray (64 rendered), hash grid 16 levels x 2^19 x 2 features, MLP
64 x 2 hidden, FP32, mean-squared colour loss, Adam.  A step is
prenom_sample + prenom_render_fwd (fused loss) + prenom_render_bwd +
prenom_adam_step on resident inputs.

Prints one JSON line: rays/s, the roofline position of the dominant kernel
(per-kernel HIP-event timing inside the timed region) and the FP64 CPU oracle
timed on a bounded sample of the same workload.
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


def algorithmic_work(arch, n_rays, S, n_fine):
    """Per-launch algorithmic bytes (HBM-bound kernels) or FLOPs (MLP) of one
    step's kernels.  Counting rule: every value the kernel must read or write
    once, each hash-grid corner access as one 8-byte (2 x FP32) row, FP32
    everywhere."""
    n_s = n_rays * S
    L = arch.n_levels
    in_dim, W, D = arch.in_dim, arch.width, arch.hidden
    macs = W * in_dim + (D - 1) * W * W + 4 * W
    per_level = 8 * 8 + 8            # 8 corner rows + the feature pair (read or write)
    pos = 4 + 24.0 / S               # t, plus the ray's origin/direction shared by S samples
    return {
        "k_sample": ("hbm", n_rays * (24 + 4 * n_fine + 8 * S + 4 * n_fine + 1 + 24)),
        "k_encode_fwd": ("hbm", n_s * (pos + L * per_level)),
        "k_mlp_fwd": ("mfma", n_s * 2.0 * macs),
        "k_composite_fwd": ("hbm", n_s * 24 + n_rays * (12 + 4 + 4 + 32 + 12 + 4 + 1)),
        "k_composite_bwd": ("hbm", n_s * 40 + n_rays * (32 + 12 + 4 + 1)),
        "k_mlp_bwd": ("mfma", n_s * 6.0 * macs),
        "k_encode_bwd": ("hbm", n_s * (pos + L * per_level)),
        "k_adam": ("hbm", arch.n_params * 32),
    }


def cpu_baseline(batch, params, n_sample_rays):
    """FP64 oracle, one full step on a bounded sample of the batch's rays."""
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
    z = np.zeros_like(params)
    orc.adam(params, g.astype(np.float32), z, z, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=1)
    dt = time.perf_counter() - t0
    return dict(value=n_sample_rays / dt, unit="rays/s", cores=orc.max_threads(), kind="oracle",
                sample=f"{n_sample_rays} of the {batch.n_rays} rays of one batch, one full step "
                       f"(sample, fwd + loss, bwd, Adam over all {batch.arch.n_params} parameters), "
                       f"FP64, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--rays", type=int, default=65536)
    ap.add_argument("--cpu-rays", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device once (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); nothing here uses a "
              "second GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_01582_amd import api
    from paper_2503_01582_amd.trainer import Trainer, to_device
    from synth.params import init_params
    from synth.workloads import prior_batch, prior_world

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    log("bench: building the synthetic scene and batch")
    world = prior_world(seed=1)
    batch = prior_batch(world, args.rays, step=0)
    arch = batch.arch
    params = init_params(arch, 0)
    torch.cuda.set_device(0)
    tr = Trainer(arch, params, batch.sample, batch.loss)
    db = to_device(batch)
    S = batch.sample.n_samples

    log(f"bench: {args.warmup} warm-up steps")
    for _ in range(args.warmup):
        tr.step(db)
    torch.cuda.synchronize()

    log(f"bench: {args.steps} timed steps")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    api.prenom_profile_begin()
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = tr.step(db)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = api.prenom_profile_end()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied 1 GiB device-to-device for counter calibration")
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    value = args.rays * args.steps / (ms / 1e3)
    loss = float(out["loss"].item())
    log(f"bench: {ms_per_step:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), loss {loss:.4e}")

    work = algorithmic_work(arch, args.rays, S, batch.sample.n_fine)
    kern = {}
    for name, (n, tot) in sorted(kt.items(), key=lambda kv: -kv[1][1]):
        avg = tot / n
        entry = dict(avg_ms=avg, share=tot / ms)
        if name in work:
            bound, amount = work[name]
            if bound == "hbm":
                entry.update(bound="hbm", achieved=amount / (avg * 1e-3) / 1e9, unit="GB/s",
                             peak=HBM_PEAK_GBS)
            else:
                entry.update(bound="mfma", achieved=amount / (avg * 1e-3) / 1e12, unit="TFLOP/s",
                             peak=FP32_MFMA_PEAK_TFLOPS)
            entry["frac"] = entry["achieved"] / entry["peak"]
        kern[name] = entry
        log(f"  {name:18s} {avg * 1e3:9.1f} us/launch  {100 * tot / ms:5.1f}%  "
            + (f"{entry['achieved']:8.1f} {entry['unit']} ({100 * entry['frac']:.1f}% of peak)"
               if "frac" in entry else ""))
    dom = max((k for k in kern if "frac" in kern[k]), key=lambda k: kern[k]["avg_ms"])
    d = kern[dom]
    roofline = dict(kernel=dom, bound=d["bound"], achieved=round(d["achieved"], 2), peak=d["peak"],
                    unit=d["unit"], frac=round(d["frac"], 4), traffic=None)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle on {args.cpu_rays} rays")
        cpu = cpu_baseline(batch, params, args.cpu_rays)

    line = dict(
        metric="training rays/s (fwd+bwd) vs plain FP32 at equal PSNR; % HBM/MFMA roofline",
        value=round(value, 1), unit="rays/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="fp32", data="synthetic",
        config=dict(workload="prior-sampled object NeRF training step", n_rays=args.rays,
                    samples_per_ray=S, n_coarse=batch.sample.n_coarse, n_fine=batch.sample.n_fine,
                    hash_levels=arch.n_levels, log2_table=arch.log2_table, mlp_width=arch.width,
                    mlp_hidden=arch.hidden, samples_per_s=round(value * S, 1)),
        roofline=roofline,
        kernels={k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                 for k, v in kern.items()},
        cpu_baseline=cpu,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
