"""Seeded synthetic object categories for meta-learning the initial
parameters (Sec. III-A: tasks are reconstructions of instances of one
category, built from a random number of posed RGB-D frames).

Inputs only: scenes, rays and their analytic targets.  Nothing here computes
any step of the method.

Recipe (the category meshes the paper uses are not available):
  * category template: union of 3 random ellipsoids (the prior scene's
    family: semi-axes U[0.1, 0.35], centres U[-0.15, 0.15]^3, random
    rotation, density 50, colours U[0.1, 0.9]^3);
  * instance: every part of the template scaled per axis by U[0.8, 1.2],
    its centre moved by N(0, 0.03^2) per axis, its colour moved by
    U[-0.1, 0.1] per channel (clipped to [0.05, 0.95]);
  * task pool of an instance: n_rays rays from the pixels of n_cams cameras
    at 96x96 (vertical FOV 60 deg, 1.5 from the centre) whose ray meets the
    NOCS cube, half drawn uniformly among those that hit the object and half
    among the rest, with analytic colour, first-hit depth and mask;
    the object frame is the NOCS frame of the prior workload (world + 0.5).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .camera import pixel_rays, random_camera_positions
from .scene import Primitive, Scene, random_ellipsoid_scene
from .workloads import FAR, NEAR, uniform_xi


def category_template(seed: int) -> Scene:
    return random_ellipsoid_scene(np.random.default_rng([seed, 3571]), 3)


def category_instance(template: Scene, seed: int, scale=(0.8, 1.2), shift_std: float = 0.03,
                      colour_jitter: float = 0.1) -> Scene:
    rng = np.random.default_rng([seed, 6007])
    prims = []
    for p in template.prims:
        col = np.clip(p.color + rng.uniform(-colour_jitter, colour_jitter, 3), 0.05, 0.95)
        prims.append(Primitive(p.kind, p.center + rng.normal(0.0, shift_std, 3), p.size * rng.uniform(*scale, 3),
                               p.rot, col))
    return Scene(prims, template.sigma0)


@dataclass
class TaskPool:
    """Rays of one instance (world frame; object frame = world + 0.5)."""
    scene: Scene
    rays_o: np.ndarray     # [n, 3] float32
    rays_d: np.ndarray     # [n, 3] float32
    tgt_rgb: np.ndarray    # [n, 3] float32
    tgt_depth: np.ndarray  # [n] float32
    mask: np.ndarray       # [n] uint8


def task_pool(scene: Scene, n_rays: int, seed: int, n_cams: int = 8, res: int = 96) -> TaskPool:
    rng = np.random.default_rng([seed, 7727])
    cube = Primitive("box", np.zeros(3), np.full(3, 0.5), np.eye(3), np.zeros(3))
    os_, ds_ = [], []
    for pos in random_camera_positions(rng, n_cams):
        o, d = pixel_rays(pos, res, res, 60.0, "vertical")
        t0, t1 = cube.intersect(o, d)
        ok = np.minimum(t1, FAR) > np.maximum(t0, NEAR)
        os_.append(o[ok])
        ds_.append(d[ok])
    o = np.concatenate(os_)
    d = np.concatenate(ds_)
    _, _, on_obj, _ = scene.ground_truth(o, d, NEAR, FAR)
    obj, rest = np.flatnonzero(on_obj), np.flatnonzero(~on_obj)
    n_obj = n_rays // 2
    pick = np.concatenate([obj[rng.integers(0, obj.size, n_obj)], rest[rng.integers(0, rest.size, n_rays - n_obj)]])
    pick = pick[rng.permutation(n_rays)]
    o, d = o[pick], d[pick]
    col, depth, hit, _ = scene.ground_truth(o, d, NEAR, FAR)
    return TaskPool(scene, o.astype(np.float32), d.astype(np.float32), col.astype(np.float32),
                    depth.astype(np.float32), hit.astype(np.uint8))


def category_pools(seed: int, n_instances: int, n_rays: int, first_instance: int = 0) -> List[TaskPool]:
    """Pools of instances first_instance .. first_instance + n_instances - 1 of
    category `seed`."""
    template = category_template(seed)
    return [task_pool(category_instance(template, 1000 * seed + k), n_rays, 1000 * seed + k)
            for k in range(first_instance, first_instance + n_instances)]


def stratification(seed: int, step: int, n_rays: int, n_fine: int) -> np.ndarray:
    return uniform_xi(np.random.default_rng([seed, 8191, step]), n_rays, n_fine)
