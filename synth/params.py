"""Initial NeRF parameters (random initialisation, Sec. III-B: objects of an
unknown category start from a default architecture with random parameters).

Hash tables: U(-1e-4, 1e-4); MLP layers: Xavier-uniform.  Layout: tables
[L][T][F], then W_1 [W][L*F], W_2..W_D [W][W], W_out [4][W], row-major."""
from __future__ import annotations

import numpy as np


def init_params(arch, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    table = rng.uniform(-1e-4, 1e-4, arch.n_table_params)
    layers = []
    for out_dim, in_dim in arch.layer_shapes():
        lim = np.sqrt(6.0 / (in_dim + out_dim))
        layers.append(rng.uniform(-lim, lim, out_dim * in_dim))
    return np.concatenate([table] + layers).astype(np.float32)


def mlp_layers(arch, mlp: np.ndarray):
    """Split a flat MLP parameter vector into its row-major matrices."""
    out, off = [], 0
    for o, i in arch.layer_shapes():
        out.append(mlp[off:off + o * i].reshape(o, i))
        off += o * i
    return out
