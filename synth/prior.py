"""Category-prior density grids F (Sec. III-A: the density of the prior NeRF on
an R^3 grid in NOCS).  No trained priors exist here, so the stand-in is the
blurred binary occupancy of a (possibly perturbed) analytic shape."""
from __future__ import annotations

import numpy as np


def nocs_vertices(R: int) -> np.ndarray:
    """NOCS coordinates of grid vertex (ix, iy, iz) = (ix, iy, iz)/(R-1),
    x fastest: array [R^3, 3]."""
    g = np.arange(R, dtype=np.float64) / (R - 1)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1)


def gaussian_blur3(vol: np.ndarray, sigma: float, radius: int) -> np.ndarray:
    """Separable, normalised Gaussian blur with clamp-to-edge borders."""
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    ker = np.exp(-0.5 * (k / sigma) ** 2)
    ker /= ker.sum()
    out = vol.astype(np.float64)
    for ax in range(3):
        pad = [(0, 0)] * 3
        pad[ax] = (radius, radius)
        p = np.pad(out, pad, mode="edge")
        acc = np.zeros_like(out)
        for i, kv in enumerate(ker):
            sl = [slice(None)] * 3
            sl[ax] = slice(i, i + out.shape[ax])
            acc += kv * p[tuple(sl)]
        out = acc
    return out


def occupancy_prior(scene, R: int = 64, blur_sigma: float = 2.0, radius: int = 6,
                    floor: float = 0.01, nocs_offset: float = 0.5) -> np.ndarray:
    """[R][R][R] float32 grid, x fastest: blurred occupancy of `scene` sampled
    at the NOCS vertices (world = NOCS - nocs_offset), plus a floor."""
    pts = nocs_vertices(R) - nocs_offset
    occ = scene.contains(pts).astype(np.float64).reshape(R, R, R)  # [z][y][x]
    grid = gaussian_blur3(occ, blur_sigma, radius) + floor
    return np.ascontiguousarray(grid.astype(np.float32))
