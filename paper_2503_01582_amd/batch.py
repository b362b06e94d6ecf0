"""Python binding of the batched calls of the C ABI (prenom_batch_* in
include/prenom.h): many object NeRFs, each with its own architecture, prior
and pose, trained by one launch per phase.  Argument marshalling only; every
step runs in libprenom's HIP kernels.  A BatchTrainer step can be captured in
a HIP graph (torch.cuda.CUDAGraph) and replayed.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .api import SampleOut, _check_rays, _dev, _ptr, _stream, alloc_sample_out, make_arch, render_cfg, sample_cfg


@dataclass
class BatchObject:
    arch: object                       # synth.arch.Arch-like
    n_rays: int
    prior: Optional[torch.Tensor]      # device [R, R, R] float32, or None (uniform sampling)
    world_to_obj: np.ndarray           # 3x4


def _c_objects(objs: Sequence[BatchObject]):
    arr = (L.PrenomObject * len(objs))()
    for i, o in enumerate(objs):
        arr[i].arch = make_arch(o.arch)
        arr[i].n_rays = int(o.n_rays)
        if o.prior is not None:
            _dev(o.prior, torch.float32, "prior")
            if o.prior.dim() != 3 or len(set(o.prior.shape)) != 1:
                raise ValueError(f"object {i}: prior must be an [R, R, R] grid, got {tuple(o.prior.shape)}")
            arr[i].prior = o.prior.data_ptr()
            arr[i].prior_res = int(o.prior.shape[0])
        else:
            arr[i].prior = None
            arr[i].prior_res = 0
        A = np.asarray(o.world_to_obj, np.float32).reshape(12)
        for k in range(12):
            arr[i].world_to_obj[k] = float(A[k])
    return arr


def _c_tiles(tiles):
    tiles = list(tiles or [])
    arr = (L.PrenomMlpTiles * max(len(tiles), 1))()
    for i, t in enumerate(tiles):
        arr[i].in_dim, arr[i].width, arr[i].hidden = t["in_dim"], t["width"], t["hidden"]
        arr[i].dtype = {"fp32": L.F32, "bf16": L.BF16, "fp16": L.F16}[t["dtype"]] if isinstance(t["dtype"], str) \
            else int(t["dtype"])
        arr[i].fwd_tiles, arr[i].bwd_tiles = int(t.get("fwd_tiles", 0)), int(t.get("bwd_tiles", 0))
    return arr, len(tiles)


def prenom_batch_param_count(objs: Sequence[BatchObject]) -> int:
    arr = _c_objects(objs)
    return int(L.lib().prenom_batch_param_count(arr, len(objs)))


def prenom_batch_param_offset(objs: Sequence[BatchObject], i: int) -> int:
    arr = _c_objects(objs)
    return int(L.lib().prenom_batch_param_offset(arr, len(objs), i))


class BatchModel:
    """Parameters, gradients and Adam moments of every object of a batch, in
    the batch layout (object i at its 64-float aligned offset)."""

    def __init__(self, objs: Sequence[BatchObject], params: Sequence, device="cuda", loss_scale=None,
                 tiles=None, device_step: bool = True, record_budget: int = 0):
        self.objs = list(objs)
        self.record_budget = int(record_budget)
        self._c_objs = _c_objects(self.objs)
        n_obj = len(self.objs)
        n = int(L.lib().prenom_batch_param_count(self._c_objs, n_obj))
        if n < 0:
            raise ValueError("invalid batch: " + L.lib().prenom_last_error().decode())
        self.offsets = [int(L.lib().prenom_batch_param_offset(self._c_objs, n_obj, i)) for i in range(n_obj)]
        self.params = torch.zeros(n, dtype=torch.float32, device=device)
        for i, (o, p) in enumerate(zip(self.objs, params)):
            p = torch.as_tensor(np.asarray(p, np.float32)) if not torch.is_tensor(p) else p
            if p.numel() != o.arch.n_params:
                raise ValueError(f"object {i}: expected {o.arch.n_params} parameters, got {p.numel()}")
            self.params[self.offsets[i]:self.offsets[i] + p.numel()] = p.to(device=device, dtype=torch.float32)
        self.grads = torch.zeros_like(self.params)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self.any_f16_table = any(getattr(o.arch, "table_dtype", "fp32") == "fp16" for o in self.objs)
        self.params_lp = torch.empty(n, dtype=torch.float16, device=device) if self.any_f16_table else None
        self.loss_scale = self.scaler_state = None
        if loss_scale is not None:
            self.loss_scale = torch.full((1,), float(loss_scale), dtype=torch.float32, device=device)
            self.scaler_state = torch.zeros(2, dtype=torch.int32, device=device)
        self.step = torch.zeros(1, dtype=torch.int64, device=device) if device_step else None
        self.host_step = 0
        self._c_tiles, self._n_tiles = _c_tiles(tiles)
        if self.params_lp is not None:
            prenom_batch_refresh_lowp(self)

    def object_params(self, i: int) -> torch.Tensor:
        return self.params[self.offsets[i]:self.offsets[i] + self.objs[i].arch.n_params]

    def object_grads(self, i: int) -> torch.Tensor:
        return self.grads[self.offsets[i]:self.offsets[i] + self.objs[i].arch.n_params]

    @property
    def n_rays(self) -> int:
        return sum(o.n_rays for o in self.objs)

    def c_struct(self) -> L.PrenomBatch:
        b = L.PrenomBatch()
        b.n_objects = len(self.objs)
        b.objects = C.cast(self._c_objs, C.POINTER(L.PrenomObject))
        b.n_tiles = self._n_tiles
        b.tiles = C.cast(self._c_tiles, C.POINTER(L.PrenomMlpTiles))
        b.params = self.params.data_ptr()
        b.grads = self.grads.data_ptr()
        b.adam_m = self.adam_m.data_ptr()
        b.adam_v = self.adam_v.data_ptr()
        b.params_lp = None if self.params_lp is None else self.params_lp.data_ptr()
        b.loss_scale = None if self.loss_scale is None else self.loss_scale.data_ptr()
        b.scaler_state = None if self.scaler_state is None else self.scaler_state.data_ptr()
        b.step = None if self.step is None else self.step.data_ptr()
        b.record_budget = self.record_budget
        return b


def prenom_batch_workspace_size(bm: BatchModel, n_samples: int) -> int:
    b = bm.c_struct()
    return int(L.lib().prenom_batch_workspace_size(C.byref(b), n_samples))


def prenom_batch_prepare(bm: BatchModel, n_samples: int, ws: torch.Tensor):
    b = bm.c_struct()
    L.check(L.lib().prenom_batch_prepare(C.byref(b), n_samples, _ptr(ws), ws.numel(), _stream()),
            "prenom_batch_prepare")


def alloc_workspace(bm: BatchModel, n_samples: int, device="cuda") -> torch.Tensor:
    need = prenom_batch_workspace_size(bm, n_samples)
    if need == 0:
        raise L.PrenomError("prenom_batch_workspace_size: " + L.lib().prenom_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    prenom_batch_prepare(bm, n_samples, ws)
    return ws


def prenom_batch_sample(bm: BatchModel, spec, rays_o, rays_d, xi, ws: torch.Tensor,
                        out: Optional[SampleOut] = None) -> SampleOut:
    _dev(rays_o, torch.float32, "rays_o")
    _dev(rays_d, torch.float32, "rays_d")
    _dev(xi, torch.float32, "xi")
    n = bm.n_rays
    if rays_o.shape != (n, 3) or rays_d.shape != (n, 3) or xi.shape != (n, spec.n_fine):
        raise ValueError("rays_o, rays_d must be [n, 3] and xi [n, n_fine] over all objects")
    if out is None:
        out = alloc_sample_out(n, spec.n_fine, spec.n_samples, rays_o.device)
    cfg = sample_cfg(spec, np.zeros((3, 4), np.float32), None)
    b = bm.c_struct()
    st = L.lib().prenom_batch_sample(C.byref(b), C.byref(cfg), _ptr(rays_o), _ptr(rays_d), _ptr(xi),
                                     _ptr(out.ray_obj), _ptr(out.t), _ptr(out.dt), _ptr(out.bins),
                                     _ptr(out.flags), _ptr(ws), ws.numel(), _stream())
    L.check(st, "prenom_batch_sample")
    return out


def alloc_render_out(bm: BatchModel, device="cuda") -> dict:
    n = bm.n_rays
    return dict(rgb=torch.empty((n, 3), dtype=torch.float32, device=device),
                depth=torch.empty((n,), dtype=torch.float32, device=device),
                opacity=torch.empty((n,), dtype=torch.float32, device=device),
                loss=torch.zeros((len(bm.objs),), dtype=torch.float32, device=device))


def prenom_batch_render_fwd(bm: BatchModel, samp: SampleOut, loss_spec, ws: torch.Tensor, *, bg=None,
                            tgt_rgb=None, tgt_depth=None, mask=None, want_loss=True, out=None, recompute=False):
    if out is None:
        out = alloc_render_out(bm, samp.t.device)
    _check_rays(samp, bm.n_rays, bg=bg, tgt_rgb=tgt_rgb, tgt_depth=tgt_depth, mask=mask)
    cfg = render_cfg(samp.n_samples, loss_spec, recompute)
    b = bm.c_struct()
    st = L.lib().prenom_batch_render_fwd(
        C.byref(b), C.byref(cfg), _ptr(samp.ray_obj), _ptr(samp.t), _ptr(samp.dt), _ptr(samp.flags), _ptr(bg),
        _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask), _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["opacity"]),
        _ptr(out["loss"]) if (want_loss and tgt_rgb is not None) else None, _ptr(ws), ws.numel(), _stream())
    L.check(st, "prenom_batch_render_fwd")
    return out


def prenom_batch_render_bwd(bm: BatchModel, samp: SampleOut, loss_spec, ws: torch.Tensor, *, bg=None,
                            tgt_rgb=None, tgt_depth=None, mask=None, d_rgb=None, d_depth=None, d_opacity=None,
                            recompute=False):
    _check_rays(samp, bm.n_rays, bg=bg, tgt_rgb=tgt_rgb, tgt_depth=tgt_depth, mask=mask, d_rgb=d_rgb,
                d_depth=d_depth, d_opacity=d_opacity)
    cfg = render_cfg(samp.n_samples, loss_spec, recompute)
    b = bm.c_struct()
    st = L.lib().prenom_batch_render_bwd(
        C.byref(b), C.byref(cfg), _ptr(samp.ray_obj), _ptr(samp.t), _ptr(samp.dt), _ptr(samp.flags), _ptr(bg),
        _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask), _ptr(d_rgb), _ptr(d_depth), _ptr(d_opacity), _ptr(ws),
        ws.numel(), _stream())
    L.check(st, "prenom_batch_render_bwd")


def prenom_batch_adam_step(bm: BatchModel, *, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=None,
                           growth_interval=2000):
    c = L.PrenomAdamCfg()
    if bm.step is None:
        if step is None:
            bm.host_step += 1
            step = bm.host_step
    else:
        step = 0  # the device counter supplies it
    c.lr, c.beta1, c.beta2, c.eps, c.step = lr, beta1, beta2, eps, step
    c.growth_interval = growth_interval
    b = bm.c_struct()
    L.check(L.lib().prenom_batch_adam_step(C.byref(b), C.byref(c), _stream()), "prenom_batch_adam_step")


def prenom_batch_sgd_step(bm: BatchModel, *, lr: float, growth_interval=2000):
    c = L.PrenomSgdCfg()
    c.lr, c.growth_interval = lr, growth_interval
    b = bm.c_struct()
    L.check(L.lib().prenom_batch_sgd_step(C.byref(b), C.byref(c), _stream()), "prenom_batch_sgd_step")


def prenom_batch_refresh_lowp(bm: BatchModel):
    b = bm.c_struct()
    L.check(L.lib().prenom_batch_refresh_lowp(C.byref(b), _stream()), "prenom_batch_refresh_lowp")


class BatchTrainer:
    """sample -> render_fwd (per-object losses) -> render_bwd -> Adam for every
    object at once, over static device buffers so the step can be captured."""

    def __init__(self, objs: Sequence[BatchObject], params: Sequence, sample_spec, loss_spec, lr=1e-2,
                 beta1=0.9, beta2=0.99, eps=1e-15, device="cuda", loss_scale=None, growth_interval=2000,
                 tiles=None, recompute=False, record_budget=0):
        self.model = BatchModel(objs, params, device, loss_scale=loss_scale, tiles=tiles, device_step=True,
                                record_budget=record_budget)
        self.sample_spec = sample_spec
        self.loss_spec = loss_spec
        self.recompute = recompute
        self.adam = dict(lr=lr, beta1=beta1, beta2=beta2, eps=eps, growth_interval=growth_interval)
        n = self.model.n_rays
        f = dict(device=device)
        self.rays_o = torch.zeros((n, 3), dtype=torch.float32, **f)
        self.rays_d = torch.zeros((n, 3), dtype=torch.float32, **f)
        self.xi = torch.full((n, sample_spec.n_fine), 0.5, dtype=torch.float32, **f)
        self.tgt_rgb = torch.zeros((n, 3), dtype=torch.float32, **f)
        self.tgt_depth = torch.zeros((n,), dtype=torch.float32, **f)
        self.mask = torch.zeros((n,), dtype=torch.uint8, **f)
        self.ws = alloc_workspace(self.model, sample_spec.n_samples, device)
        self.samp = alloc_sample_out(n, sample_spec.n_fine, sample_spec.n_samples, device)
        self.out = alloc_render_out(self.model, device)
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def load(self, batch):
        """Copy a host batch (synth.multi.MultiBatch) into the static buffers."""
        for name in ("rays_o", "rays_d", "xi", "tgt_rgb", "tgt_depth", "mask"):
            getattr(self, name).copy_(torch.as_tensor(np.ascontiguousarray(getattr(batch, name))))

    def step(self):
        m = self.model
        prenom_batch_sample(m, self.sample_spec, self.rays_o, self.rays_d, self.xi, self.ws, out=self.samp)
        prenom_batch_render_fwd(m, self.samp, self.loss_spec, self.ws, tgt_rgb=self.tgt_rgb,
                                tgt_depth=self.tgt_depth, mask=self.mask, out=self.out)
        prenom_batch_render_bwd(m, self.samp, self.loss_spec, self.ws, tgt_rgb=self.tgt_rgb,
                                tgt_depth=self.tgt_depth, mask=self.mask, recompute=self.recompute)
        prenom_batch_adam_step(m, **self.adam)
        return self.out

    def capture(self):
        """Record one step in a graph (nothing runs during the capture)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.out
