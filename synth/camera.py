"""Pinhole cameras on a sphere around the object, and their pixel rays."""
from __future__ import annotations

import numpy as np


def random_camera_positions(rng, n: int, radius: float = 1.5) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * radius


def look_at(pos, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world rotation with columns (right, up, forward)."""
    pos = np.asarray(pos, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, np.float64)
    if np.linalg.norm(np.cross(fwd, up)) < 1e-6:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    return np.stack([right, true_up, fwd], 1)


def pixel_rays(pos, width: int, height: int, fov_deg: float, fov_axis: str = "vertical",
               pixels=None):
    """Unit-direction world rays through pixel centres (i + 1/2, j + 1/2).
    pixels: optional flat pixel indices (row-major); all pixels when None."""
    R = look_at(pos)
    extent = height if fov_axis == "vertical" else width
    focal = 0.5 * extent / np.tan(0.5 * np.deg2rad(fov_deg))
    if pixels is None:
        pixels = np.arange(width * height)
    pixels = np.asarray(pixels, np.int64)
    i = (pixels % width).astype(np.float64)
    j = (pixels // width).astype(np.float64)
    x = (i + 0.5 - 0.5 * width) / focal
    y = -(j + 0.5 - 0.5 * height) / focal
    dirs = x[:, None] * R[:, 0] + y[:, None] * R[:, 1] + R[:, 2]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    origins = np.broadcast_to(np.asarray(pos, np.float64), dirs.shape).copy()
    return origins, dirs
