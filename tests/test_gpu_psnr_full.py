"""Equal PSNR at the benchmarked shape: 48 objects sharing 2^20 rays x 64
samples, each with its own scene, prior, pose and architecture, trained
together for 500 steps by the batched step, in the FP32 form and in the
reduced-precision forms (MLP operands in BF16 or in FP16 on the matrix
cores with FP32 accumulation and FP32 masters, FP16 table copy, FP32
table-gradient accumulation and scans, dynamic loss scaling from 2^12).
Held-out PSNR per object (2 views at 48 x 48), averaged over the objects and
over three seeds; the reduced-precision means must stay within 0.1 dB of the
FP32 mean.

About ten minutes of GPU time: it runs when PRENOM_LONG_TESTS=1 is set and
is skipped otherwise.  With PRENOM_PSNR_SUMMARY=<file> it writes the numbers
as JSON (the committed summary the benchmark line quotes)."""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np
import pytest

from synth.multi import multi_batch, multi_objects, object_eval_views
from synth.params import init_params
from synth.workloads import LossSpec, PRIOR_SAMPLE
from test_gpu_batch_training import eval_psnr

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("PRENOM_LONG_TESTS") != "1",
                                 reason="about ten minutes of GPU time: set PRENOM_LONG_TESTS=1")]
torch = pytest.importorskip("torch")

N_OBJ, TOTAL_RAYS, STEPS, N_BATCHES = 48, 1 << 20, 500, 8
SEEDS = (5, 6, 7)
BOUND_DB = 0.1
FORMS = (("fp32", "fp32"), ("bf16", "fp16"), ("fp16", "fp16"))


def say(*a):
    print(*a, flush=True)


def train(objs, params, batches, lowp, tiles):
    from paper_2503_01582_amd.batch import BatchObject, BatchTrainer
    bobjs = [BatchObject(o.arch, o.n_rays, torch.as_tensor(o.prior).cuda(), o.world_to_obj) for o in objs]
    tr = BatchTrainer(bobjs, params, PRIOR_SAMPLE, LossSpec(), loss_scale=4096.0 if lowp else None, tiles=tiles)
    losses, t0 = [], time.time()
    for i in range(STEPS):
        tr.load(batches[i % len(batches)])
        out = tr.step()
        if i % 100 == 0 or i == STEPS - 1:
            losses.append(float(out["loss"].mean().item()))
            say(f"    step {i}: mean loss {losses[-1]:.4e} ({time.time() - t0:.0f} s)")
    torch.cuda.synchronize()
    scale = float(tr.model.loss_scale.item()) if lowp else None
    return tr.model, losses, scale


def test_batch48_reduced_precision_psnr_at_full_shape():
    say("test_batch48_reduced_precision_psnr_at_full_shape")
    from paper_2503_01582_amd import autotune
    means = {f[0]: [] for f in FORMS}
    per_seed = []
    for seed in SEEDS:
        base = multi_objects(seed, N_OBJ, total_rays=TOTAL_RAYS)
        say(f"  seed {seed}: {sum(o.n_rays for o in base)} rays over {len(base)} objects; building batches")
        batches = [multi_batch(base, step=k) for k in range(N_BATCHES)]
        views = [object_eval_views(o, n_views=2, res=48) for o in base]
        params = [init_params(o.arch, i) for i, o in enumerate(base)]
        row = dict(seed=seed)
        for mlp_dtype, table_dtype in FORMS:
            objs = [dataclasses.replace(o, arch=dataclasses.replace(o.arch, mlp_dtype=mlp_dtype,
                                                                     table_dtype=table_dtype)) for o in base]
            tiles = autotune.tiles_for([o.arch for o in objs])
            say(f"  seed {seed}, {mlp_dtype} MLP / {table_dtype} table")
            model, losses, scale = train(objs, params, batches, mlp_dtype != "fp32", tiles)
            p = eval_psnr(objs, model.params, model.offsets, views)
            means[mlp_dtype].append(float(p.mean()))
            row[mlp_dtype] = dict(mean_psnr_db=round(float(p.mean()), 4), final_loss=losses[-1], loss_scale=scale,
                                  per_object_db=[round(float(v), 3) for v in p])
            say(f"  seed {seed} {mlp_dtype}: mean held-out PSNR {p.mean():.3f} dB, loss {losses}"
                + (f", loss scale {scale:.0f}" if scale else ""))
            del model
            torch.cuda.empty_cache()
        for k in ("bf16", "fp16"):
            d = np.array(row[k]["per_object_db"]) - np.array(row["fp32"]["per_object_db"])
            row[k]["delta_db"] = round(float(d.mean()), 4)
            say(f"  seed {seed} {k} - fp32: {d.mean():+.3f} dB (per object: min {d.min():+.2f}, max {d.max():+.2f})")
        per_seed.append(row)
    result = dict(n_objects=N_OBJ, total_rays=TOTAL_RAYS, steps=STEPS, seeds=list(SEEDS), bound_db=BOUND_DB,
                  mean_psnr_db={k: round(float(np.mean(v)), 4) for k, v in means.items()},
                  delta_db={k: round(float(np.mean(means[k]) - np.mean(means["fp32"])), 4) for k in ("bf16", "fp16")},
                  per_seed=per_seed)
    say(f"  over seeds {SEEDS}: bf16 - fp32 {result['delta_db']['bf16']:+.3f} dB, "
        f"fp16 - fp32 {result['delta_db']['fp16']:+.3f} dB")
    path = os.environ.get("PRENOM_PSNR_SUMMARY")
    if path:
        with open(path, "w") as f:
            json.dump(result, f, indent=1)
    for k in ("bf16", "fp16"):
        assert abs(result["delta_db"][k]) <= BOUND_DB, (k, result["delta_db"][k])
