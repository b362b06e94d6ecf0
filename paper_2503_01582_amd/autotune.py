"""Tile-shape autotuner for the batched MLP launches.

A batched MLP launch gives each block a run of 16-sample tiles of one object:
long runs amortise loading the object's weight fragments into LDS (and, in
the backward, writing one partial weight gradient per block), short runs give
more blocks for small objects.  For each MLP shape (input features, width,
hidden layers, element type) this module times the batched forward and
backward MLP kernels over candidate run lengths on a synthetic one-object
batch, with the library's per-kernel event timing, and keeps the fastest of
each.  Results are cached in a JSON file keyed by GPU architecture, HIP
runtime version, library version and shape.

    python -m paper_2503_01582_amd.autotune [--out FILE] [--rays N]
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, Iterable, List, Optional

import numpy as np

FWD_CANDIDATES = (16, 32, 64, 128, 256, 512)
BWD_CANDIDATES = (32, 64, 128, 256, 512, 1024)
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_gfx950.json")


def cache_path() -> str:
    return os.environ.get("PRENOM_TILE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "prenom", "tiles.json"))


def device_key() -> str:
    import torch
    from . import api
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    return f"{arch}|hip {torch.version.hip}|{api.version()}"


def shape_key(in_dim: int, width: int, hidden: int, dtype: str) -> str:
    return f"in{in_dim}_w{width}_d{hidden}_{dtype}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _rays(n: int, seed: int):
    """Rays from a radius-1.5 sphere towards random points of the object box."""
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o *= 1.5 / np.linalg.norm(o, axis=1, keepdims=True)
    tgt = rng.uniform(-0.45, 0.45, (n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def time_shape(arch, fwd_tiles: int, bwd_tiles: int, n_rays: int = 16384, reps: int = 4) -> Dict[str, float]:
    """Average ms of the batched MLP forward and backward launches of one
    object of `arch` with n_rays x 64 samples at the given tile shape."""
    import torch
    from synth.params import init_params
    from synth.workloads import LossSpec, SampleSpec, nocs_affine
    from . import api
    from . import batch as B

    spec = SampleSpec(n_coarse=16, n_fine=48, include_coarse=True, uniform_only=True)
    obj = B.BatchObject(arch, n_rays, None, nocs_affine())
    tiles = [dict(in_dim=arch.in_dim, width=arch.width, hidden=arch.hidden, dtype=arch.mlp_dtype,
                  fwd_tiles=fwd_tiles, bwd_tiles=bwd_tiles)]
    bm = B.BatchModel([obj], [init_params(arch, 0)], tiles=tiles,
                      loss_scale=None if arch.mlp_dtype == "fp32" else 4096.0)
    ws = B.alloc_workspace(bm, spec.n_samples)
    o, d = _rays(n_rays, 1)
    dev = lambda a: torch.as_tensor(a).cuda()
    xi = torch.full((n_rays, spec.n_fine), 0.5, device="cuda")
    samp = B.prenom_batch_sample(bm, spec, dev(o), dev(d), xi, ws)
    tgt = torch.full((n_rays, 3), 0.5, device="cuda")
    loss = LossSpec()
    B.prenom_batch_render_fwd(bm, samp, loss, ws, tgt_rgb=tgt)
    B.prenom_batch_render_bwd(bm, samp, loss, ws, tgt_rgb=tgt)
    torch.cuda.synchronize()
    api.prenom_profile_begin()
    for _ in range(reps):
        B.prenom_batch_render_fwd(bm, samp, loss, ws, tgt_rgb=tgt)
        B.prenom_batch_render_bwd(bm, samp, loss, ws, tgt_rgb=tgt)
    kt = api.prenom_profile_end()
    return {k: kt[k][1] / kt[k][0] for k in ("k_mlp_fwd", "k_mlp_bwd") if k in kt}


def tune(arches: Iterable, n_rays: int = 16384, out: Optional[str] = None, log=print) -> List[dict]:
    """Tunes every distinct MLP shape of `arches`; merges into the cache."""
    path = out or cache_path()
    cache = _load(path)
    dk = device_key()
    table = cache.setdefault(dk, {})
    seen = set()
    for a in arches:
        key = shape_key(a.in_dim, a.width, a.hidden, a.mlp_dtype)
        if key in seen:
            continue
        seen.add(key)
        best_f = best_b = None
        for f, b in zip(FWD_CANDIDATES, BWD_CANDIDATES):
            t = time_shape(a, f, b, n_rays)
            log(f"  {key}: fwd {f:4d} tiles {t['k_mlp_fwd'] * 1e3:8.1f} us, bwd {b:5d} tiles "
                f"{t['k_mlp_bwd'] * 1e3:8.1f} us")
            if best_f is None or t["k_mlp_fwd"] < best_f[1]:
                best_f = (f, t["k_mlp_fwd"])
            if best_b is None or t["k_mlp_bwd"] < best_b[1]:
                best_b = (b, t["k_mlp_bwd"])
        table[key] = dict(fwd_tiles=best_f[0], bwd_tiles=best_b[0], fwd_us=best_f[1] * 1e3,
                          bwd_us=best_b[1] * 1e3, n_rays=n_rays)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return tiles_for(arches, path)


def tiles_for(arches: Iterable, path: Optional[str] = None) -> List[dict]:
    """Tile entries (for BatchModel) of the shapes of `arches` found in the
    cache, else in the table shipped with the package; shapes found in
    neither get the library defaults."""
    dk = device_key()
    tables = [_load(path or cache_path()).get(dk, {}), _load(PACKAGED).get(dk, {})]
    out, seen = [], set()
    for a in arches:
        key = shape_key(a.in_dim, a.width, a.hidden, a.mlp_dtype)
        if key in seen:
            continue
        seen.add(key)
        for t in tables:
            if key in t:
                out.append(dict(in_dim=a.in_dim, width=a.width, hidden=a.hidden, dtype=a.mlp_dtype,
                                fwd_tiles=t[key]["fwd_tiles"], bwd_tiles=t[key]["bwd_tiles"]))
                break
    return out


def all_shapes(dtypes=("fp32",)):
    from synth.arch import Arch
    return [Arch(n_levels=L, log2_table=14, width=W, hidden=D, mlp_dtype=dt)
            for dt in dtypes for L in (8, 12, 16) for W in (32, 64, 128) for D in (1, 2)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--rays", type=int, default=16384)
    ap.add_argument("--dtypes", default="fp32,bf16,fp16")
    args = ap.parse_args()
    tune(all_shapes(tuple(args.dtypes.split(","))), args.rays, args.out)


if __name__ == "__main__":
    main()
