"""Seeded workloads at the paper's object-level shapes (Sec. IV-A: 4096 rays per
iteration, N_c = N_r = 32, R = 64, epsilon = 1e-4) and at the larger prior-based
configurations used for measurement.

Workloads
---------
small   : sphere + box scene, one random 64x64 camera per step (4096 rays),
          near/far 0.5/2.5, 32 stratified uniform samples, 8 levels x 2^14,
          MLP 64 x 1, mean-squared colour loss.
prior   : union of 3 random ellipsoids; prior = blurred occupancy of a
          perturbed copy on 64^3 vertices + 0.01; 16 cameras at 640x480
          (horizontal FOV 60 deg); rays drawn uniformly among pixels whose ray
          meets the NOCS cube; 16 coarse + 48 inverse-CDF samples, coarse
          samples rendered too (64 per ray); 16 levels x 2^19, MLP 64 x 2.
          n_rays = 2^16 (prior sampling) or 2^18 (+ depth loss 0.1 with
          1 cm Gaussian depth noise).

The datasets the paper evaluates on are not available; these analytic scenes
stand in for them.  Every random number comes from numpy's seeded generators.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .arch import ARCH_LARGE, ARCH_SMALL, Arch
from .camera import pixel_rays, random_camera_positions
from .prior import occupancy_prior
from .scene import Primitive, Scene, perturbed, random_ellipsoid_scene, sphere_box_scene

NEAR, FAR = 0.5, 2.5


def nocs_affine(offset: float = 0.5) -> np.ndarray:
    """World -> NOCS affine (row-major 3x4) for an object centred at the
    origin with unit extent: x_nocs = x_world + offset."""
    A = np.zeros((3, 4), np.float32)
    A[:, :3] = np.eye(3)
    A[:, 3] = offset
    return A.reshape(12)


def uniform_xi(rng, n: int, k: int) -> np.ndarray:
    """Stratification jitter xi in (0, 1): ((u32 >> 8) + 1/2) 2^-24, exact in FP32."""
    u = rng.integers(0, 2**32, size=(n, k), dtype=np.uint64) >> np.uint64(8)
    return ((u.astype(np.float64) + 0.5) * 2.0**-24).astype(np.float32)


@dataclass
class SampleSpec:
    n_coarse: int
    n_fine: int
    include_coarse: bool
    uniform_only: bool
    eps: float = 1e-4
    near: float = NEAR
    far: float = FAR

    @property
    def n_samples(self) -> int:
        return self.n_fine + (self.n_coarse if self.include_coarse else 0)


@dataclass
class LossSpec:
    loss_mode: int = 0
    lambda_d: float = 0.0
    lambda_sigma: float = 0.0


@dataclass
class Batch:
    arch: Arch
    sample: SampleSpec
    loss: LossSpec
    rays_o: np.ndarray          # [n, 3] float32, world
    rays_d: np.ndarray          # [n, 3] float32, world, unit
    xi: np.ndarray              # [n, N_r] float32 in (0, 1)
    tgt_rgb: np.ndarray         # [n, 3] float32
    tgt_depth: np.ndarray       # [n] float32
    mask: np.ndarray            # [n] uint8 (1 = object ray)
    world_to_obj: np.ndarray    # [12] float32
    prior: Optional[np.ndarray] = None  # [R, R, R] float32
    bg: Optional[np.ndarray] = None     # [n, 3] float32 or None (black)
    meta: dict = field(default_factory=dict)

    @property
    def n_rays(self) -> int:
        return self.rays_o.shape[0]


# ------------------------------------------------------------------ small

SMALL_SAMPLE = SampleSpec(n_coarse=0, n_fine=32, include_coarse=False, uniform_only=True)


def small_batch(step: int, seed: int = 0, arch: Arch = ARCH_SMALL, res: int = 64) -> Batch:
    scene = sphere_box_scene()
    rng = np.random.default_rng([seed, step])
    pos = random_camera_positions(rng, 1)[0]
    o, d = pixel_rays(pos, res, res, 60.0, "vertical")
    col, depth, hit, _ = scene.ground_truth(o, d, NEAR, FAR)
    n = o.shape[0]
    return Batch(arch=arch, sample=SMALL_SAMPLE, loss=LossSpec(),
                 rays_o=o.astype(np.float32), rays_d=d.astype(np.float32),
                 xi=uniform_xi(rng, n, SMALL_SAMPLE.n_fine),
                 tgt_rgb=col.astype(np.float32), tgt_depth=depth.astype(np.float32),
                 mask=hit.astype(np.uint8), world_to_obj=nocs_affine(),
                 meta=dict(workload="small", camera=pos))


# ------------------------------------------------------------------ prior

PRIOR_SAMPLE = SampleSpec(n_coarse=16, n_fine=48, include_coarse=True, uniform_only=False)


@dataclass
class PriorWorld:
    scene: Scene
    prior: np.ndarray
    cams: np.ndarray
    width: int
    height: int
    pool: np.ndarray          # [m, 2] (camera, pixel) of rays that meet the cube


def prior_world(seed: int = 1, R: int = 64, n_cams: int = 16, width: int = 640,
                height: int = 480, pool_stride: int = 1) -> PriorWorld:
    rng = np.random.default_rng(seed)
    scene = random_ellipsoid_scene(rng, 3)
    prior = occupancy_prior(perturbed(scene, rng), R=R)
    cams = random_camera_positions(rng, n_cams)
    cube = Primitive("box", np.zeros(3), np.full(3, 0.5), np.eye(3), np.zeros(3))
    pool = []
    pix = np.arange(0, width * height, pool_stride)
    for c in range(n_cams):
        o, d = pixel_rays(cams[c], width, height, 60.0, "horizontal", pixels=pix)
        t0, t1 = cube.intersect(o, d)
        ok = (np.minimum(t1, FAR) > np.maximum(t0, NEAR))
        pool.append(np.stack([np.full(ok.sum(), c), pix[ok]], 1))
    return PriorWorld(scene, prior, cams, width, height, np.concatenate(pool))


def prior_batch(world: PriorWorld, n_rays: int, step: int, seed: int = 1,
                arch: Arch = ARCH_LARGE, depth_noise: float = 0.0,
                loss: Optional[LossSpec] = None) -> Batch:
    rng = np.random.default_rng([seed, 7919, step])
    pick = world.pool[rng.integers(0, world.pool.shape[0], n_rays)]
    o = np.empty((n_rays, 3))
    d = np.empty((n_rays, 3))
    for c in np.unique(pick[:, 0]):
        sel = pick[:, 0] == c
        oc, dc = pixel_rays(world.cams[c], world.width, world.height, 60.0, "horizontal",
                            pixels=pick[sel, 1])
        o[sel], d[sel] = oc, dc
    col, depth, hit, _ = world.scene.ground_truth(o, d, NEAR, FAR)
    if depth_noise > 0.0:
        depth = depth + rng.normal(0.0, depth_noise, n_rays) * hit
    return Batch(arch=arch, sample=PRIOR_SAMPLE, loss=loss or LossSpec(),
                 rays_o=o.astype(np.float32), rays_d=d.astype(np.float32),
                 xi=uniform_xi(rng, n_rays, PRIOR_SAMPLE.n_fine),
                 tgt_rgb=col.astype(np.float32), tgt_depth=depth.astype(np.float32),
                 mask=hit.astype(np.uint8), world_to_obj=nocs_affine(), prior=world.prior,
                 meta=dict(workload="prior"))


def eval_views(scene: Scene, n_views: int = 8, seed: int = 100, res: int = 64):
    """Held-out cameras: (rays_o, rays_d, rgb, depth, mask) per view."""
    rng = np.random.default_rng(seed)
    out = []
    for pos in random_camera_positions(rng, n_views):
        o, d = pixel_rays(pos, res, res, 60.0, "vertical")
        col, depth, hit, _ = scene.ground_truth(o, d, NEAR, FAR)
        out.append((o.astype(np.float32), d.astype(np.float32), col.astype(np.float32),
                    depth.astype(np.float32), hit.astype(np.uint8)))
    return out
