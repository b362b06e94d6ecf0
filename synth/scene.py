"""Analytic scenes and their closed-form ground truth.

A scene is an ordered list of primitives (sphere, box, ellipsoid), each with a
constant colour, filled with a constant density sigma0 (the union has density
sigma0; where primitives overlap, the first-listed primitive's colour wins).
Given rays, the ground truth is integrated exactly, segment by segment:

    C_gt = sum_seg T_in c_seg (1 - exp(-sigma0 L_seg)) + T_out C_bg
    D_gt = distance to the first surface hit (a depth sensor's reading)
    mask = the ray hits the union inside [near, far]

These are targets and masks for training and evaluation; they are not the
method (the method renders a discrete quadrature of a learned field).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np


@dataclass
class Primitive:
    kind: str                # "sphere" | "box" | "ellipsoid"
    center: np.ndarray       # (3,)
    size: np.ndarray         # sphere: (r,r,r); box: half extents; ellipsoid: semi-axes
    rot: np.ndarray          # (3,3) local -> world rotation
    color: np.ndarray        # (3,)

    def _local(self, o, d):
        # world -> local (rotation only), then scale so the primitive is a unit shape
        R = self.rot
        ol = (o - self.center) @ R
        dl = d @ R
        return ol, dl

    def intersect(self, o, d):
        """Entry / exit distance along each ray (inf, -inf when missed)."""
        ol, dl = self._local(o, d)
        n = o.shape[0]
        if self.kind in ("sphere", "ellipsoid"):
            os_ = ol / self.size
            ds_ = dl / self.size
            a = np.sum(ds_ * ds_, axis=1)
            b = np.sum(ds_ * os_, axis=1)
            c = np.sum(os_ * os_, axis=1) - 1.0
            disc = b * b - a * c
            hit = disc > 0.0
            sq = np.sqrt(np.where(hit, disc, 0.0))
            t0 = np.where(hit, (-b - sq) / a, np.inf)
            t1 = np.where(hit, (-b + sq) / a, -np.inf)
            return t0, t1
        if self.kind == "box":
            t_enter = np.full(n, -np.inf)
            t_exit = np.full(n, np.inf)
            for ax in range(3):
                da = dl[:, ax]
                oa = ol[:, ax]
                h = self.size[ax]
                with np.errstate(divide="ignore", invalid="ignore"):
                    ta = (-h - oa) / da
                    tb = (h - oa) / da
                par = da == 0.0
                inside = np.abs(oa) <= h
                lo = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(ta, tb))
                hi = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(ta, tb))
                t_enter = np.maximum(t_enter, lo)
                t_exit = np.minimum(t_exit, hi)
            hit = t_enter < t_exit
            return np.where(hit, t_enter, np.inf), np.where(hit, t_exit, -np.inf)
        raise ValueError(self.kind)

    def contains(self, p):
        pl = (p - self.center) @ self.rot
        if self.kind in ("sphere", "ellipsoid"):
            return np.sum((pl / self.size) ** 2, axis=1) <= 1.0
        return np.all(np.abs(pl) <= self.size, axis=1)


@dataclass
class Scene:
    prims: List[Primitive]
    sigma0: float = 50.0

    def contains(self, p):
        inside = np.zeros(p.shape[0], bool)
        for pr in self.prims:
            inside |= pr.contains(p)
        return inside

    def ground_truth(self, o, d, near, far, bg=None):
        """Closed-form colour, first-hit depth and mask for unit-direction rays."""
        o = np.asarray(o, np.float64)
        d = np.asarray(d, np.float64)
        n = o.shape[0]
        P = len(self.prims)
        ints = [pr.intersect(o, d) for pr in self.prims]
        t_in = np.stack([a for a, _ in ints], 1)     # [n, P]
        t_out = np.stack([b for _, b in ints], 1)
        t_in = np.clip(t_in, near, far)
        t_out = np.clip(t_out, near, far)
        brk = np.sort(np.concatenate([t_in, t_out], 1), axis=1)  # [n, 2P]
        brk = np.where(np.isfinite(brk), brk, far)
        T = np.ones(n)
        col = np.zeros((n, 3))
        depth = np.zeros(n)
        hit = np.zeros(n, bool)
        for s in range(2 * P - 1):
            a = brk[:, s]
            b = brk[:, s + 1]
            L = np.maximum(b - a, 0.0)
            mid = 0.5 * (a + b)
            c_seg = np.zeros((n, 3))
            covered = np.zeros(n, bool)
            for p in range(P - 1, -1, -1):  # first-listed wins
                cov = (t_in[:, p] <= mid) & (mid <= t_out[:, p]) & (t_in[:, p] < t_out[:, p])
                c_seg[cov] = self.prims[p].color
                covered |= cov
            covered &= L > 0.0
            att = np.exp(-self.sigma0 * L)
            contrib = np.where(covered, T * (1.0 - att), 0.0)
            col += contrib[:, None] * c_seg
            first = covered & ~hit
            depth = np.where(first, a, depth)
            hit |= covered
            T = np.where(covered, T * att, T)
        if bg is not None:
            col += T[:, None] * np.asarray(bg, np.float64)
        return col, depth, hit, T


def _rand_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def sphere_box_scene() -> Scene:
    """Sphere (r = 0.3) and axis-aligned box (half extent 0.2) inside
    [-0.5, 0.5]^3, density 50, fixed colours."""
    I = np.eye(3)
    return Scene([
        Primitive("sphere", np.array([-0.15, 0.0, 0.0]), np.full(3, 0.3), I, np.array([0.9, 0.3, 0.2])),
        Primitive("box", np.array([0.25, 0.0, 0.0]), np.full(3, 0.2), I, np.array([0.2, 0.5, 0.9])),
    ], sigma0=50.0)


def random_ellipsoid_scene(rng, n_prims: int = 3, allow_boxes: bool = False) -> Scene:
    """Union of random ellipsoids (semi-axes U[0.1, 0.35], centres
    U[-0.15, 0.15]^3, uniform random rotation, colours U[0.1, 0.9]^3)."""
    prims = []
    for _ in range(n_prims):
        kind = "ellipsoid"
        if allow_boxes and rng.random() < 0.5:
            kind = "box"
        axes = rng.uniform(0.1, 0.35, 3)
        if kind == "box":
            axes = axes * 0.7
        prims.append(Primitive(kind, rng.uniform(-0.15, 0.15, 3), axes, _rand_rotation(rng),
                               rng.uniform(0.1, 0.9, 3)))
    return Scene(prims, sigma0=50.0)


def perturbed(scene: Scene, rng, scale=(0.85, 1.15), shift_std=0.02) -> Scene:
    """An imprecise copy of a scene (sizes scaled, centres jittered), the
    stand-in for a category prior that does not fit the instance exactly."""
    prims = []
    for p in scene.prims:
        prims.append(Primitive(p.kind, p.center + rng.normal(0.0, shift_std, 3),
                               p.size * rng.uniform(*scale, 3), p.rot, p.color))
    return Scene(prims, scene.sigma0)


def riemann_ground_truth(scene: Scene, o, d, near, far, n_steps=100000, bg=None):
    """Slow midpoint-rule reference for ground_truth() (used to pin it)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    out = np.zeros((o.shape[0], 3))
    dt = (far - near) / n_steps
    for r in range(o.shape[0]):
        ts = near + (np.arange(n_steps) + 0.5) * dt
        p = o[r] + ts[:, None] * d[r]
        col = np.zeros((n_steps, 3))
        dens = np.zeros(n_steps)
        for pr in reversed(scene.prims):
            inside = pr.contains(p)
            col[inside] = pr.color
            dens[inside] = scene.sigma0
        tau = dens * dt
        T = np.exp(-np.concatenate([[0.0], np.cumsum(tau)[:-1]]))
        w = T * (1.0 - np.exp(-tau))
        out[r] = (w[:, None] * col).sum(0)
        if bg is not None:
            out[r] += np.exp(-tau.sum()) * np.asarray(bg)
    return out
