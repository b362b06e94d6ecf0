"""Meta-learning of a category's initial parameters with Reptile (Sec. III-A,
Eq. (1)-(2)) on the batched step: B tasks (instances of the category) are
the B objects of one batch, all with the category architecture, trained from
the meta-parameters theta for q inner iterations; prenom_reptile_update then
moves theta by beta times the mean of their differences and restarts every
task slot from the new theta.  Argument marshalling only; every step runs in
libprenom's HIP kernels.

The inner step is Eq. (1)'s gradient descent (prenom_batch_sgd_step); the
mapping optimiser (Adam, with its moments and step counter reset at each
meta-iteration by the same outer call) can be chosen instead.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import api
from .batch import (BatchObject, BatchTrainer, prenom_batch_adam_step, prenom_batch_render_bwd,
                    prenom_batch_render_fwd, prenom_batch_sample, prenom_batch_sgd_step)


class ReptileTrainer(BatchTrainer):
    def __init__(self, arch, theta, n_tasks: int, n_rays: int, sample_spec, loss_spec, *, inner_lr: float,
                 beta: float, inner: str = "sgd", world_to_obj=None, prior: Optional[torch.Tensor] = None,
                 device="cuda", tiles=None, **adam):
        if inner not in ("sgd", "adam"):
            raise ValueError("inner must be 'sgd' or 'adam'")
        if world_to_obj is None:
            raise ValueError("world_to_obj (3x4) is required")
        objs = [BatchObject(arch, n_rays, prior, world_to_obj) for _ in range(n_tasks)]
        if tiles is None:  # MLP tile shapes measured for this architecture, where cached
            from . import autotune
            tiles = autotune.tiles_for([arch])
        theta = np.asarray(theta.detach().cpu() if torch.is_tensor(theta) else theta, np.float32)
        super().__init__(objs, [theta] * n_tasks, sample_spec, loss_spec, lr=inner_lr, device=device, tiles=tiles,
                         **adam)
        self.inner, self.inner_lr, self.beta = inner, inner_lr, beta
        self.n_tasks, self.n_params = n_tasks, arch.n_params
        offs = self.model.offsets
        self.stride = offs[1] - offs[0] if n_tasks > 1 else (arch.n_params + 63) // 64 * 64
        if any(offs[i] != i * self.stride for i in range(n_tasks)):
            raise ValueError("task slots are not evenly spaced")
        self.theta = torch.as_tensor(theta).to(device).clone()
        self.meta_step = 0

    def load_rays(self, rays_o, rays_d, xi, tgt_rgb, tgt_depth, mask):
        """Copy device tensors (tasks one after another) into the static buffers."""
        for name, v in (("rays_o", rays_o), ("rays_d", rays_d), ("xi", xi), ("tgt_rgb", tgt_rgb),
                        ("tgt_depth", tgt_depth), ("mask", mask)):
            getattr(self, name).copy_(v)

    def step(self):
        """One inner iteration of every task: sample, render, backward, and the
        inner update."""
        m = self.model
        prenom_batch_sample(m, self.sample_spec, self.rays_o, self.rays_d, self.xi, self.ws, out=self.samp)
        prenom_batch_render_fwd(m, self.samp, self.loss_spec, self.ws, tgt_rgb=self.tgt_rgb,
                                tgt_depth=self.tgt_depth, mask=self.mask, out=self.out)
        prenom_batch_render_bwd(m, self.samp, self.loss_spec, self.ws, tgt_rgb=self.tgt_rgb,
                                tgt_depth=self.tgt_depth, mask=self.mask, recompute=self.recompute)
        if self.inner == "sgd":
            prenom_batch_sgd_step(m, lr=self.inner_lr, growth_interval=self.adam["growth_interval"])
        else:
            prenom_batch_adam_step(m, **self.adam)
        return self.out

    def outer(self):
        """Eq. (2) over the tasks; every task slot restarts from the new theta."""
        m = self.model
        adam = self.inner == "adam"
        api.prenom_reptile_update(self.theta, m.params, self.n_params, self.n_tasks, self.stride, self.beta,
                                  adam_m=m.adam_m if adam else None, adam_v=m.adam_v if adam else None,
                                  tasks_lp=m.params_lp, n_lp=self.n_params if m.params_lp is not None else 0,
                                  step=m.step)
        self.meta_step += 1
