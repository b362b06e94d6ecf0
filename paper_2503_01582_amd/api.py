"""Python binding of the C ABI (include/prenom.h), one function per entry point
with the same name.  PyTorch supplies device memory and the current stream;
every step of the computation runs in libprenom's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_rays(samp: "SampleOut", n: int, **arrays):
    """The library takes plain pointers and cannot check sizes: every per-ray
    array (the samples' own and the optional ones given by keyword) must be a
    contiguous device tensor of the expected dtype holding exactly n rays."""
    S = samp.t.shape[1] if samp.t.dim() == 2 else -1
    per = dict(ray_obj=(torch.float32, 6), t=(torch.float32, S), dt=(torch.float32, S),
               flags=(torch.uint8, 1), bg=(torch.float32, 3), tgt_rgb=(torch.float32, 3),
               tgt_depth=(torch.float32, 1), mask=(torch.uint8, 1), d_rgb=(torch.float32, 3),
               d_depth=(torch.float32, 1), d_opacity=(torch.float32, 1), sample_out=(torch.float32, 4 * S))
    given = dict(ray_obj=samp.ray_obj, t=samp.t, dt=samp.dt, flags=samp.flags, **arrays)
    for name, t in given.items():
        dtype, k = per[name]
        _dev(t, dtype, name)
        if t is not None and (k < 0 or t.numel() != n * k):
            raise ValueError(f"{name} holds {t.numel()} values, expected {n} rays x {k}")


def _dev(t: Optional[torch.Tensor], dtype, name: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def make_arch(arch) -> L.PrenomArch:
    """arch: object with n_levels, log2_table, n_features, resolutions, width, hidden."""
    a = L.PrenomArch()
    a.n_levels = arch.n_levels
    a.log2_table = arch.log2_table
    a.n_features = arch.n_features
    for i, r in enumerate(arch.resolutions):
        a.resolution[i] = int(r)
    a.mlp_width = arch.width
    a.mlp_hidden = arch.hidden
    a.mlp_dtype = {"fp32": L.F32, "bf16": L.BF16, "fp16": L.F16}[getattr(arch, "mlp_dtype", "fp32")]
    a.table_dtype = {"fp32": L.F32, "fp16": L.F16}[getattr(arch, "table_dtype", "fp32")]
    return a


def prenom_param_count(arch) -> int:
    return int(L.lib().prenom_param_count(C.byref(make_arch(arch))))


def prenom_table_param_count(arch) -> int:
    return int(L.lib().prenom_table_param_count(C.byref(make_arch(arch))))


def prenom_workspace_size(arch, n_rays: int, n_samples: int, recompute: bool = False) -> int:
    return int(L.lib().prenom_workspace_size(C.byref(make_arch(arch)), n_rays, n_samples, int(bool(recompute))))


class Model:
    """One object NeRF on the device: parameters, gradients and Adam moments,
    plus the FP16 table copy and the loss-scaling state of the
    reduced-precision form (arch.table_dtype == "fp16", loss_scale given)."""

    def __init__(self, arch, params, device="cuda", loss_scale=None):
        self.arch = arch
        n = prenom_param_count(arch)
        if n < 0:
            raise ValueError("invalid architecture")
        p = torch.as_tensor(np.asarray(params, np.float32) if not torch.is_tensor(params) else params)
        if p.numel() != n:
            raise ValueError(f"expected {n} parameters, got {p.numel()}")
        self.params = p.to(device=device, dtype=torch.float32).contiguous().clone()
        self.grads = torch.zeros_like(self.params)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self.step = 0
        self._c_arch = make_arch(arch)
        self.table_lp = None
        if self._c_arch.table_dtype == L.F16:
            self.table_lp = torch.empty(arch.n_table_params, dtype=torch.float16, device=device)
        self.loss_scale = None
        self.scaler_state = None
        if loss_scale is not None:
            self.loss_scale = torch.full((1,), float(loss_scale), dtype=torch.float32, device=device)
            self.scaler_state = torch.zeros(2, dtype=torch.int32, device=device)
        if self.table_lp is not None:
            prenom_refresh_lowp(self)

    def c_struct(self, grads: Optional[torch.Tensor] = None) -> L.PrenomModel:
        m = L.PrenomModel()
        m.arch = self._c_arch
        m.params = self.params.data_ptr()
        m.grads = (grads if grads is not None else self.grads).data_ptr()
        m.adam_m = self.adam_m.data_ptr()
        m.adam_v = self.adam_v.data_ptr()
        m.table_lp = None if self.table_lp is None else self.table_lp.data_ptr()
        m.loss_scale = None if self.loss_scale is None else self.loss_scale.data_ptr()
        m.scaler_state = None if self.scaler_state is None else self.scaler_state.data_ptr()
        return m

    @property
    def n_table(self) -> int:
        return self.arch.n_table_params


@dataclass
class SampleOut:
    ray_obj: torch.Tensor
    t: torch.Tensor
    dt: torch.Tensor
    bins: torch.Tensor
    flags: torch.Tensor

    @property
    def n_samples(self) -> int:
        return self.t.shape[1]


def alloc_sample_out(n_rays: int, n_fine: int, n_samples: int, device="cuda") -> SampleOut:
    f = dict(device=device)
    return SampleOut(ray_obj=torch.empty((n_rays, 6), dtype=torch.float32, **f),
                     t=torch.empty((n_rays, n_samples), dtype=torch.float32, **f),
                     dt=torch.empty((n_rays, n_samples), dtype=torch.float32, **f),
                     bins=torch.empty((n_rays, n_fine), dtype=torch.int32, **f),
                     flags=torch.empty((n_rays,), dtype=torch.uint8, **f))


def sample_cfg(spec, world_to_obj, prior: Optional[torch.Tensor]) -> L.PrenomSampleCfg:
    c = L.PrenomSampleCfg()
    c.n_coarse = spec.n_coarse
    c.n_fine = spec.n_fine
    c.include_coarse = int(spec.include_coarse)
    c.uniform_only = int(spec.uniform_only)
    c.eps = spec.eps
    c.near_t = spec.near
    c.far_t = spec.far
    A = np.asarray(world_to_obj, np.float32).reshape(12)
    for i in range(12):
        c.world_to_obj[i] = float(A[i])
    if prior is not None:
        _dev(prior, torch.float32, "prior")
        if prior.dim() != 3 or len(set(prior.shape)) != 1:
            raise ValueError(f"prior must be an [R, R, R] grid, got {tuple(prior.shape)}")
        c.prior = prior.data_ptr()
        c.prior_res = prior.shape[0]
    else:
        c.prior = None
        c.prior_res = 0
    return c


def prenom_sample(spec, rays_o: torch.Tensor, rays_d: torch.Tensor, xi: torch.Tensor, world_to_obj,
                  prior: Optional[torch.Tensor] = None, out: Optional[SampleOut] = None) -> SampleOut:
    _dev(rays_o, torch.float32, "rays_o")
    _dev(rays_d, torch.float32, "rays_d")
    _dev(xi, torch.float32, "xi")
    n = rays_o.shape[0]
    if rays_d.shape != (n, 3) or rays_o.shape != (n, 3) or xi.shape != (n, spec.n_fine):
        raise ValueError("rays_o, rays_d must be [n, 3] and xi [n, n_fine]")
    if out is None:
        out = alloc_sample_out(n, spec.n_fine, spec.n_samples, rays_o.device)
    else:
        if out.t.dim() != 2 or out.t.shape != (n, spec.n_samples):
            raise ValueError(f"out.t must be [{n}, {spec.n_samples}]")
        _check_rays(out, n)
        _dev(out.bins, torch.int32, "bins")
        if out.bins.numel() != n * spec.n_fine:
            raise ValueError(f"out.bins must hold {n} x {spec.n_fine} values")
    cfg = sample_cfg(spec, world_to_obj, prior)
    st = L.lib().prenom_sample(C.byref(cfg), _ptr(rays_o), _ptr(rays_d), _ptr(xi), n,
                               _ptr(out.ray_obj), _ptr(out.t), _ptr(out.dt), _ptr(out.bins),
                               _ptr(out.flags), _stream())
    L.check(st, "prenom_sample")
    return out


def render_cfg(n_samples: int, loss, recompute: bool = False) -> L.PrenomRenderCfg:
    c = L.PrenomRenderCfg()
    c.n_samples = n_samples
    c.recompute = int(recompute)
    c.loss_mode = loss.loss_mode if loss is not None else 0
    c.lambda_d = loss.lambda_d if loss is not None else 0.0
    c.lambda_sigma = loss.lambda_sigma if loss is not None else 0.0
    return c


class Workspace:
    """Device scratch for render_fwd/render_bwd, grown on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf: Optional[torch.Tensor] = None

    def get(self, arch, n_rays: int, n_samples: int, recompute: bool = False) -> torch.Tensor:
        need = prenom_workspace_size(arch, n_rays, n_samples, recompute)
        if self.buf is None or self.buf.numel() < need:
            self.buf = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self.buf


def prenom_render_fwd(model: Model, samp: SampleOut, loss_spec, ws: torch.Tensor, *, bg=None,
                      tgt_rgb=None, tgt_depth=None, mask=None, want_loss=True, sample_out=None,
                      out=None, recompute=False):
    n, S = samp.t.shape
    dev = samp.t.device
    if out is None:
        out = dict(rgb=torch.empty((n, 3), dtype=torch.float32, device=dev),
                   depth=torch.empty((n,), dtype=torch.float32, device=dev),
                   opacity=torch.empty((n,), dtype=torch.float32, device=dev),
                   loss=torch.zeros((1,), dtype=torch.float32, device=dev))
    _check_rays(samp, n, bg=bg, tgt_rgb=tgt_rgb, tgt_depth=tgt_depth, mask=mask, sample_out=sample_out)
    cfg = render_cfg(S, loss_spec, recompute)
    mc = model.c_struct()
    st = L.lib().prenom_render_fwd(
        C.byref(mc), C.byref(cfg), _ptr(samp.ray_obj), _ptr(samp.t), _ptr(samp.dt), _ptr(samp.flags), n,
        _ptr(bg), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask), _ptr(out["rgb"]), _ptr(out["depth"]),
        _ptr(out["opacity"]), _ptr(out["loss"]) if (want_loss and tgt_rgb is not None) else None,
        _ptr(sample_out), _ptr(ws), ws.numel(), _stream())
    L.check(st, "prenom_render_fwd")
    return out


def prenom_render_bwd(model: Model, samp: SampleOut, loss_spec, ws: torch.Tensor, *, bg=None,
                      tgt_rgb=None, tgt_depth=None, mask=None, d_rgb=None, d_depth=None,
                      d_opacity=None, grads: Optional[torch.Tensor] = None, recompute=False):
    n, S = samp.t.shape
    _check_rays(samp, n, bg=bg, tgt_rgb=tgt_rgb, tgt_depth=tgt_depth, mask=mask, d_rgb=d_rgb, d_depth=d_depth,
                d_opacity=d_opacity)
    cfg = render_cfg(S, loss_spec, recompute)
    mc = model.c_struct(grads)
    st = L.lib().prenom_render_bwd(
        C.byref(mc), C.byref(cfg), _ptr(samp.ray_obj), _ptr(samp.t), _ptr(samp.dt), _ptr(samp.flags), n,
        _ptr(bg), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask), _ptr(d_rgb), _ptr(d_depth),
        _ptr(d_opacity), _ptr(ws), ws.numel(), _stream())
    L.check(st, "prenom_render_bwd")


def prenom_refresh_lowp(model: Model):
    mc = model.c_struct()
    L.check(L.lib().prenom_refresh_lowp(C.byref(mc), _stream()), "prenom_refresh_lowp")


def prenom_adam_step(model: Model, *, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=None,
                     growth_interval=2000):
    if step is None:
        model.step += 1
        step = model.step
    c = L.PrenomAdamCfg()
    c.lr, c.beta1, c.beta2, c.eps, c.step = lr, beta1, beta2, eps, step
    c.growth_interval = growth_interval
    mc = model.c_struct()
    L.check(L.lib().prenom_adam_step(C.byref(mc), C.byref(c), _stream()), "prenom_adam_step")


def prenom_sgd_step(model: Model, *, lr: float, growth_interval=2000):
    """Eq. (1): params -= lr * grads, gradients zeroed."""
    c = L.PrenomSgdCfg()
    c.lr, c.growth_interval = lr, growth_interval
    mc = model.c_struct()
    L.check(L.lib().prenom_sgd_step(C.byref(mc), C.byref(c), _stream()), "prenom_sgd_step")


def prenom_reptile_update(theta: torch.Tensor, tasks: torch.Tensor, n_params: int, n_tasks: int, task_stride: int,
                          beta: float, adam_m: Optional[torch.Tensor] = None, adam_v: Optional[torch.Tensor] = None,
                          tasks_lp: Optional[torch.Tensor] = None, n_lp: int = 0,
                          step: Optional[torch.Tensor] = None):
    """Eq. (2) over n_tasks task vectors (task b at tasks[b * task_stride:]);
    every task slot restarts from the new theta."""
    _dev(theta, torch.float32, "theta")
    _dev(tasks, torch.float32, "tasks")
    if theta.numel() < n_params or tasks.numel() < (n_tasks - 1) * task_stride + n_params:
        raise ValueError("theta or tasks smaller than the layout they are given")
    for t, dt, name in ((adam_m, torch.float32, "adam_m"), (adam_v, torch.float32, "adam_v"),
                        (tasks_lp, torch.float16, "tasks_lp")):
        _dev(t, dt, name)
        if t is not None and t.numel() < (n_tasks - 1) * task_stride + (n_lp if name == "tasks_lp" else n_params):
            raise ValueError(f"{name} smaller than the task layout")
    if step is not None and (step.dtype != torch.int64 or not step.is_cuda):
        raise TypeError("step must be a device int64 tensor")
    st = L.lib().prenom_reptile_update(_ptr(theta), _ptr(tasks), n_params, n_tasks, task_stride, beta, _ptr(adam_m),
                                       _ptr(adam_v), _ptr(tasks_lp), n_lp, _ptr(step), _stream())
    L.check(st, "prenom_reptile_update")


def prenom_canonical_yaw(points: torch.Tensor, prior: torch.Tensor, n_yaw: int = 360) -> dict:
    """Eq. (3): scores [n_yaw] of the yaws 2 pi k / n_yaw, the extents and
    centres [n_yaw, 3] of the turned cloud (FP64, device) and the best index
    (device int32 [1])."""
    _dev(points, torch.float32, "points")
    _dev(prior, torch.float32, "prior")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [n, 3]")
    if prior.dim() != 3 or not (prior.shape[0] == prior.shape[1] == prior.shape[2]):
        raise ValueError("prior must be [R, R, R]")
    n = points.shape[0]
    need = L.lib().prenom_canonical_yaw_workspace_size(n, n_yaw)
    if need == 0:
        raise ValueError(f"invalid sizes: {n} points, {n_yaw} yaws")
    dev = points.device
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    out = dict(scores=torch.empty(n_yaw, dtype=torch.float64, device=dev),
               extents=torch.empty((n_yaw, 3), dtype=torch.float64, device=dev),
               centers=torch.empty((n_yaw, 3), dtype=torch.float64, device=dev),
               best=torch.empty(1, dtype=torch.int32, device=dev))
    st = L.lib().prenom_canonical_yaw(_ptr(points), n, _ptr(prior), prior.shape[0], n_yaw, _ptr(out["scores"]),
                                      _ptr(out["extents"]), _ptr(out["centers"]), _ptr(out["best"]),
                                      C.c_void_p(ws.data_ptr() + off), need, _stream())
    L.check(st, "prenom_canonical_yaw")
    return out


def prenom_prior_refresh(model: Model, R: int = 64, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The model's density grid [R, R, R] (indexed [k][j][i], x fastest):
    sigma at the vertices (i, j, k) / (R - 1), ready to pass to prenom_sample
    as the prior."""
    dev = model.params.device
    c_arch = make_arch(model.arch)
    need = L.lib().prenom_prior_refresh_workspace_size(C.byref(c_arch), R)
    if need == 0:
        raise ValueError(f"invalid architecture or R = {R}")
    ws = torch.empty(need // 4 + 64, dtype=torch.float32, device=dev)
    off = (-ws.data_ptr()) % 256
    if out is None:
        out = torch.empty((R, R, R), dtype=torch.float32, device=dev)
    mc = model.c_struct()
    st = L.lib().prenom_prior_refresh(C.byref(mc), R, _ptr(out), C.c_void_p(ws.data_ptr() + off),
                                      need, _stream())
    L.check(st, "prenom_prior_refresh")
    return out


def prenom_prior_refresh_noalloc(model: Model, R: int = 64, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """prenom_prior_refresh without a workspace: the library's fixed scratch
    array holds the per-chunk intermediates, so nothing is allocated on the
    device by the call (`out` is the caller's; pass one to allocate nothing)."""
    if out is None:
        out = torch.empty((R, R, R), dtype=torch.float32, device=model.params.device)
    _dev(out, torch.float32, "out")
    if out.numel() != R * R * R:
        raise ValueError(f"out holds {out.numel()} floats, not R^3 = {R ** 3}")
    mc = model.c_struct()
    st = L.lib().prenom_prior_refresh_noalloc(C.byref(mc), R, _ptr(out), _stream())
    L.check(st, "prenom_prior_refresh_noalloc")
    return out


def prenom_encode(arch, table: torch.Tensor, pos: torch.Tensor, with_corners=False):
    _dev(table, torch.float32, "table")
    _dev(pos, torch.float32, "pos")
    n = pos.shape[0]
    feats = torch.empty((arch.n_levels, n, arch.n_features), dtype=torch.float32, device=pos.device)
    idx = torch.empty((arch.n_levels, n, 8), dtype=torch.int32, device=pos.device) if with_corners else None
    a = make_arch(arch)
    st = L.lib().prenom_encode(C.byref(a), _ptr(table), _ptr(pos), n, _ptr(feats), _ptr(idx), _stream())
    L.check(st, "prenom_encode")
    return (feats, idx) if with_corners else feats


def prenom_profile_begin():
    L.check(L.lib().prenom_profile_begin(), "prenom_profile_begin")


def prenom_profile_end(capacity: int = 64) -> dict:
    """{kernel name: (launches, total milliseconds)} since profile_begin."""
    arr = (L.PrenomKernelTime * capacity)()
    n = C.c_int32(0)
    L.check(L.lib().prenom_profile_end(arr, capacity, C.byref(n)), "prenom_profile_end")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


def version() -> str:
    return L.lib().prenom_version().decode()
