"""Seeded inputs for many objects trained together (the map holds many
object NeRFs, each with its own category architecture, prior and pose, all
trained concurrently: Fig. 1 and Sec. IV-A).

Inputs only: scenes, priors, poses, ray counts, architectures and ray
batches.  Nothing here computes any step of the method.

Recipe per object (seeded):
  * scene: union of 2-3 random ellipsoids or boxes (axes U[0.1, 0.35],
    centres U[-0.15, 0.15]^3, random rotation, density 50, colours
    U[0.1, 0.9]^3), the same family as the single-object prior scene;
  * prior: occupancy of a perturbed copy on R^3 vertices, R ~ U{32..64},
    blurred (sigma 2 voxels) + 0.01;
  * rays: n_i = floor(exp(U[ln 1024, ln 65536])), optionally rescaled so the
    batch totals a given count (largest-remainder rounding);
  * architecture: L in {8, 12, 16}, log2 T in {14..19}, MLP width from
    `widths`, depth in {1, 2}; base resolution 16, growth 1.5;
  * pose: the object's frame is rotated about z by U[0, 2 pi) and shifted by
    U[-2, 2]^2 x U[-0.2, 0.2] in the world; rays are generated in the object's
    frame and moved to the world, and world_to_obj maps them back onto NOCS.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional, Sequence

import numpy as np

from .arch import Arch
from .camera import pixel_rays, random_camera_positions
from .prior import occupancy_prior
from .scene import Primitive, Scene, perturbed, random_ellipsoid_scene
from .workloads import FAR, NEAR, PRIOR_SAMPLE, LossSpec, uniform_xi

LEVELS = (8, 12, 16)
LOG2_TABLES = (14, 15, 16, 17, 18, 19)
DEPTHS = (1, 2)


@dataclass
class ObjectSpec:
    arch: Arch
    n_rays: int
    scene: Scene
    prior: np.ndarray          # [R, R, R] float32
    rot: np.ndarray            # object -> world rotation (3x3)
    shift: np.ndarray          # object -> world translation
    cams: np.ndarray           # camera centres (object frame)
    pool: np.ndarray           # [m, 2] (camera, pixel) whose rays meet the unit cube
    width: int
    height: int

    @property
    def world_to_obj(self) -> np.ndarray:
        """Row-major 3x4: x_obj = R^T (x_w - shift) + 0.5 (NOCS)."""
        A = np.empty((3, 4))
        A[:, :3] = self.rot.T
        A[:, 3] = -self.rot.T @ self.shift + 0.5
        return A.astype(np.float32)


def _rot_z(theta: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def largest_remainder(weights: Sequence[float], total: int) -> List[int]:
    w = np.asarray(weights, np.float64)
    q = w / w.sum() * total
    base = np.floor(q).astype(np.int64)
    rest = total - int(base.sum())
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rest]] += 1
    return [int(v) for v in base]


def multi_objects(seed: int, n_objects: int, total_rays: Optional[int] = None,
                  widths: Sequence[int] = (32, 64, 128), mlp_dtype: str = "fp32", table_dtype: str = "fp32",
                  n_cams: int = 16, width: int = 640, height: int = 480,
                  pool_stride: int = 7) -> List[ObjectSpec]:
    rng = np.random.default_rng([seed, 4242])
    cube = Primitive("box", np.zeros(3), np.full(3, 0.5), np.eye(3), np.zeros(3))
    objs = []
    for _ in range(n_objects):
        scene = random_ellipsoid_scene(rng, int(rng.integers(2, 4)), allow_boxes=True)
        R = int(rng.integers(32, 65))
        prior = occupancy_prior(perturbed(scene, rng), R=R).astype(np.float32)
        n = int(np.floor(np.exp(rng.uniform(np.log(1024.0), np.log(65536.0)))))
        arch = Arch(n_levels=int(rng.choice(LEVELS)), log2_table=int(rng.choice(LOG2_TABLES)),
                    width=int(rng.choice(widths)), hidden=int(rng.choice(DEPTHS)),
                    mlp_dtype=mlp_dtype, table_dtype=table_dtype)
        rot = _rot_z(rng.uniform(0.0, 2.0 * np.pi))
        shift = np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-0.2, 0.2)])
        cams = random_camera_positions(rng, n_cams)
        pix = np.arange(0, width * height, pool_stride)
        pool = []
        for c in range(n_cams):
            o, d = pixel_rays(cams[c], width, height, 60.0, "horizontal", pixels=pix)
            t0, t1 = cube.intersect(o, d)
            ok = np.minimum(t1, FAR) > np.maximum(t0, NEAR)
            pool.append(np.stack([np.full(ok.sum(), c), pix[ok]], 1))
        objs.append(ObjectSpec(arch, n, scene, prior, rot, shift, cams, np.concatenate(pool), width, height))
    if total_rays is not None:
        counts = largest_remainder([o.n_rays for o in objs], total_rays)
        objs = [replace(o, n_rays=c) for o, c in zip(objs, counts)]
    return objs


@dataclass
class MultiBatch:
    """Rays of all objects, object after object (world frame)."""
    counts: List[int]
    rays_o: np.ndarray
    rays_d: np.ndarray
    xi: np.ndarray
    tgt_rgb: np.ndarray
    tgt_depth: np.ndarray
    mask: np.ndarray

    @property
    def n_rays(self) -> int:
        return int(self.rays_o.shape[0])

    def slice(self, i: int):
        b = int(np.sum(self.counts[:i]))
        e = b + self.counts[i]
        return slice(b, e)


def multi_batch(objs: Sequence[ObjectSpec], step: int, seed: int = 4, n_fine: int = PRIOR_SAMPLE.n_fine,
                depth_noise: float = 0.0) -> MultiBatch:
    """One training batch: n_i rays per object drawn from its pixel pool, with
    analytic ground truth (rendered in the object frame)."""
    rng = np.random.default_rng([seed, 104729, step])
    os_, ds_, cols, depths, hits = [], [], [], [], []
    for ob in objs:
        n = ob.n_rays
        pick = ob.pool[rng.integers(0, ob.pool.shape[0], n)] if n > 0 else np.zeros((0, 2), np.int64)
        o = np.empty((n, 3))
        d = np.empty((n, 3))
        for c in np.unique(pick[:, 0]):
            sel = pick[:, 0] == c
            oc, dc = pixel_rays(ob.cams[c], ob.width, ob.height, 60.0, "horizontal", pixels=pick[sel, 1])
            o[sel], d[sel] = oc, dc
        col, depth, hit, _ = ob.scene.ground_truth(o, d, NEAR, FAR)
        if depth_noise > 0.0:
            depth = depth + rng.normal(0.0, depth_noise, n) * hit
        os_.append(o @ ob.rot.T + ob.shift)
        ds_.append(d @ ob.rot.T)
        cols.append(col)
        depths.append(depth)
        hits.append(hit)
    n_all = sum(o.n_rays for o in objs)
    return MultiBatch(counts=[o.n_rays for o in objs],
                      rays_o=np.concatenate(os_).astype(np.float32).reshape(n_all, 3),
                      rays_d=np.concatenate(ds_).astype(np.float32).reshape(n_all, 3),
                      xi=uniform_xi(rng, n_all, n_fine),
                      tgt_rgb=np.concatenate(cols).astype(np.float32).reshape(n_all, 3),
                      tgt_depth=np.concatenate(depths).astype(np.float32),
                      mask=np.concatenate(hits).astype(np.uint8))


def object_eval_views(ob: ObjectSpec, n_views: int = 2, seed: int = 100, res: int = 48):
    """Held-out views of one object, rays in the world frame."""
    rng = np.random.default_rng([seed, 31])
    out = []
    for pos in random_camera_positions(rng, n_views):
        o, d = pixel_rays(pos, res, res, 60.0, "vertical")
        col, depth, hit, _ = ob.scene.ground_truth(o, d, NEAR, FAR)
        out.append(((o @ ob.rot.T + ob.shift).astype(np.float32), (d @ ob.rot.T).astype(np.float32),
                    col.astype(np.float32), depth.astype(np.float32), hit.astype(np.uint8)))
    return out


DEFAULT_LOSS = LossSpec()
