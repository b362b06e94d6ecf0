"""One object's training loop on the device: sample -> render_fwd (fused loss)
-> render_bwd -> Adam, all through the C ABI (Sec. III-B, one iteration of an
object-level NeRF)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import api


@dataclass
class DeviceBatch:
    rays_o: torch.Tensor
    rays_d: torch.Tensor
    xi: torch.Tensor
    tgt_rgb: torch.Tensor
    tgt_depth: torch.Tensor
    mask: torch.Tensor
    world_to_obj: np.ndarray
    prior: Optional[torch.Tensor]
    bg: Optional[torch.Tensor]

    @property
    def n_rays(self) -> int:
        return self.rays_o.shape[0]


def to_device(batch, device="cuda") -> DeviceBatch:
    """Copy a host batch (numpy arrays: rays_o, rays_d, xi, tgt_rgb, tgt_depth,
    mask, world_to_obj, prior, bg) to the device."""
    def t(a, dt=torch.float32):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):  # e.g. a prior refreshed on the device
            return a.to(device=device, dtype=dt)
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    return DeviceBatch(rays_o=t(batch.rays_o), rays_d=t(batch.rays_d), xi=t(batch.xi),
                       tgt_rgb=t(batch.tgt_rgb), tgt_depth=t(batch.tgt_depth),
                       mask=t(batch.mask, torch.uint8),
                       world_to_obj=np.asarray(batch.world_to_obj, np.float32),
                       prior=t(batch.prior), bg=t(batch.bg))


class Trainer:
    def __init__(self, arch, params, sample_spec, loss_spec, lr=1e-2, beta1=0.9, beta2=0.99,
                 eps=1e-15, device="cuda", loss_scale=None, growth_interval=2000):
        self.model = api.Model(arch, params, device, loss_scale=loss_scale)
        self.sample_spec = sample_spec
        self.loss_spec = loss_spec
        self.adam = dict(lr=lr, beta1=beta1, beta2=beta2, eps=eps, growth_interval=growth_interval)
        self.ws = api.Workspace(device)
        self._samp: Optional[api.SampleOut] = None
        self._out = None

    def _buffers(self, n_rays: int):
        spec = self.sample_spec
        if self._samp is None or self._samp.t.shape[0] != n_rays:
            dev = self.model.params.device
            self._samp = api.alloc_sample_out(n_rays, spec.n_fine, spec.n_samples, dev)
            self._out = dict(rgb=torch.empty((n_rays, 3), device=dev),
                             depth=torch.empty((n_rays,), device=dev),
                             opacity=torch.empty((n_rays,), device=dev),
                             loss=torch.zeros((1,), device=dev))
        return self._samp, self._out

    def sample(self, b: DeviceBatch) -> api.SampleOut:
        samp, _ = self._buffers(b.n_rays)
        return api.prenom_sample(self.sample_spec, b.rays_o, b.rays_d, b.xi, b.world_to_obj, b.prior,
                                 out=samp)

    def forward(self, b: DeviceBatch, samp: api.SampleOut, want_loss=True):
        _, out = self._buffers(b.n_rays)
        ws = self.ws.get(self.model.arch, b.n_rays, samp.n_samples)
        return api.prenom_render_fwd(self.model, samp, self.loss_spec, ws, bg=b.bg, tgt_rgb=b.tgt_rgb,
                                     tgt_depth=b.tgt_depth, mask=b.mask, want_loss=want_loss, out=out)

    def backward(self, b: DeviceBatch, samp: api.SampleOut):
        ws = self.ws.get(self.model.arch, b.n_rays, samp.n_samples)
        api.prenom_render_bwd(self.model, samp, self.loss_spec, ws, bg=b.bg, tgt_rgb=b.tgt_rgb,
                              tgt_depth=b.tgt_depth, mask=b.mask)

    def refresh_prior(self, R: int = 64) -> torch.Tensor:
        """The model's own density grid [R, R, R] at the vertices (i, j, k) /
        (R - 1), for use as the sampling prior of later steps."""
        return api.prenom_prior_refresh(self.model, R)

    def step(self, b: DeviceBatch):
        """One full training iteration; returns the forward outputs (device)."""
        samp = self.sample(b)
        out = self.forward(b, samp)
        self.backward(b, samp)
        api.prenom_adam_step(self.model, **self.adam)
        return out


class AutogradTrainer(Trainer):
    """The same iteration with the loss written in torch on top of
    PrenomRender: colour MSE over all rays plus lambda_d * depth MSE over
    object rays (the mean-squared form of Eq. (8)-(9)), then Adam."""

    def __init__(self, *a, recompute=False, **k):
        super().__init__(*a, **k)
        self.recompute = recompute
        self.model.params.requires_grad_(True)

    def step(self, b: DeviceBatch):
        from .autograd import render
        samp = self.sample(b)
        rgb, depth, _ = render(self.model, samp, b.bg, self.recompute)
        n = b.n_rays
        loss = ((rgb - b.tgt_rgb) ** 2).sum() / (3 * n)
        if self.loss_spec.lambda_d > 0:
            m = b.mask.float()
            loss = loss + self.loss_spec.lambda_d * (m * (depth - b.tgt_depth) ** 2).sum() / n
        self.model.params.grad = None
        loss.backward()
        with torch.no_grad():
            self.model.grads.add_(self.model.params.grad)
        api.prenom_adam_step(self.model, **self.adam)
        return dict(rgb=rgb.detach(), depth=depth.detach(), loss=loss.detach().reshape(1))
