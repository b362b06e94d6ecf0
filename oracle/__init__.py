"""numpy bridge to the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The oracle shares no code with the
GPU library.  Array inputs that the GPU receives in FP32 are passed here as the
same FP32 arrays (promotion to FP64 happens inside, exactly); outputs are FP64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

MAX_LEVELS = 32
FLAG_MISS, FLAG_ESCAPED, FLAG_UNIFORM = 1, 2, 4

_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class OrcArch(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("log2_table", C.c_int32),
        ("n_features", C.c_int32),
        ("res", C.c_int32 * MAX_LEVELS),
        ("width", C.c_int32),
        ("hidden", C.c_int32),
        ("mlp_dtype", C.c_int32),
        ("table_dtype", C.c_int32),
    ]


class OrcSampleCfg(C.Structure):
    _fields_ = [
        ("n_coarse", C.c_int32),
        ("n_fine", C.c_int32),
        ("include_coarse", C.c_int32),
        ("uniform_only", C.c_int32),
        ("eps", C.c_double),
        ("near_t", C.c_double),
        ("far_t", C.c_double),
        ("A", C.c_double * 12),
        ("prior", _f32p),
        ("prior_res", C.c_int32),
    ]


class OrcRenderCfg(C.Structure):
    _fields_ = [
        ("arch", OrcArch),
        ("n_samples", C.c_int32),
        ("loss_mode", C.c_int32),
        ("lambda_d", C.c_double),
        ("lambda_sigma", C.c_double),
        ("grad_scale", C.c_double),
        ("jitter", C.c_double),
        ("jitter_features", C.c_double),
        ("jitter_seed", C.c_uint64),
    ]


_lib = None


def lib():
    """Load liboracle.so, compiling it first only if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        L.orc_param_count.restype = C.c_int64
        L.orc_param_count.argtypes = [C.POINTER(OrcArch)]
        L.orc_prior_lookup.argtypes = [_f32p, C.c_int32, _f64p, C.c_int64, _f64p]
        L.orc_sample.argtypes = [C.POINTER(OrcSampleCfg), _f32p, _f32p, _f32p, C.c_int64,
                                 _f64p, _f64p, _f64p, _i32p, _u8p, _f64p]
        L.orc_encode.argtypes = [C.POINTER(OrcArch), _f32p, _f32p, C.c_int64, _f64p, _i32p, _f64p]
        L.orc_mlp_fwd.argtypes = [C.POINTER(OrcArch), _f32p, _f64p, C.c_int64, _f64p]
        L.orc_prior_refresh.argtypes = [C.POINTER(OrcArch), _f32p, C.c_int32, _f64p]
        L.orc_canonical_yaw.argtypes = [_f32p, C.c_int64, _f32p, C.c_int32, C.c_int32, _f64p, _f64p, _f64p, _i32p]
        L.orc_round16_array.argtypes = [_f64p, C.c_int64, C.c_int32, _f64p]
        L.orc_composite_fwd.argtypes = [C.c_int64, C.c_int32, _f64p, _f64p, _f64p, _f64p, _f64p,
                                        _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_composite_bwd.argtypes = [C.c_int64, C.c_int32, _f64p, _f64p, _f64p, _f64p, _f64p,
                                        _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_render_fwd.argtypes = [C.POINTER(OrcRenderCfg), _f32p, _f32p, _f32p, _f32p, _u8p,
                                     C.c_int64, _f32p, _f32p, _f32p, _u8p, _f64p, _f64p, _f64p,
                                     _f64p, _f64p, _f64p, C.POINTER(C.c_uint64)]
        L.orc_render_bwd.argtypes = [C.POINTER(OrcRenderCfg), _f32p, _f32p, _f32p, _f32p, _u8p,
                                     C.c_int64, _f32p, _f32p, _f32p, _u8p, _f32p, _f32p, _f32p,
                                     _f64p]
        L.orc_adam.argtypes = [C.c_int64, _f32p, _f32p, _f32p, _f32p, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int64, _f64p, _f64p, _f64p]
        L.orc_positions.argtypes = [_f32p, _f32p, C.c_int64, C.c_int32, _f32p]
        L.orc_max_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctype)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def make_arch(arch, emulate: bool = False) -> OrcArch:
    """arch: any object with n_levels, log2_table, n_features, resolutions,
    width, hidden (e.g. synth.arch.Arch).  emulate: take the arch's
    mlp_dtype / table_dtype into account (reduced-precision emulation);
    otherwise the oracle is plain FP64 whatever the arch says."""
    a = OrcArch()
    a.n_levels = arch.n_levels
    a.log2_table = arch.log2_table
    a.n_features = arch.n_features
    for i, r in enumerate(arch.resolutions):
        a.res[i] = int(r)
    a.width = arch.width
    a.hidden = arch.hidden
    a.mlp_dtype = {"fp32": 0, "bf16": 1, "fp16": 2}[getattr(arch, "mlp_dtype", "fp32")] if emulate else 0
    a.table_dtype = {"fp32": 0, "fp16": 2}[getattr(arch, "table_dtype", "fp32")] if emulate else 0
    return a


def param_count(arch) -> int:
    return int(lib().orc_param_count(C.byref(make_arch(arch))))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's per-ray loops from now on (timing only)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- sampler

def prior_lookup(prior, pts):
    prior = _f32(prior)
    pts = _f64(pts).reshape(-1, 3)
    R = prior.shape[0]
    out = np.empty(pts.shape[0], np.float64)
    lib().orc_prior_lookup(_p(prior, _f32p), R, _p(pts, _f64p), pts.shape[0], _p(out, _f64p))
    return out


def sample(rays_o, rays_d, xi, *, n_coarse, n_fine, include_coarse, uniform_only, eps,
           near, far, world_to_obj, prior=None):
    """Probabilistic ray sampling.  Returns a dict of FP64 ray_obj [n,6],
    t [n,S], dt [n,S], int32 bins [n,N_r], uint8 flags [n] and the per-ray
    minimum FP64 decision margin (inf where no CDF draw was made)."""
    rays_o = _f32(rays_o).reshape(-1, 3)
    rays_d = _f32(rays_d).reshape(-1, 3)
    n = rays_o.shape[0]
    xi = _f32(xi).reshape(n, n_fine)
    cfg = OrcSampleCfg()
    cfg.n_coarse, cfg.n_fine = n_coarse, n_fine
    cfg.include_coarse, cfg.uniform_only = int(include_coarse), int(uniform_only)
    cfg.eps = float(np.float32(eps))
    cfg.near_t, cfg.far_t = float(np.float32(near)), float(np.float32(far))
    A = np.asarray(world_to_obj, np.float32).reshape(12)
    for i in range(12):
        cfg.A[i] = float(A[i])
    prior = _f32(prior)
    cfg.prior = _p(prior, _f32p)
    cfg.prior_res = 0 if prior is None else prior.shape[0]
    S = n_fine + (n_coarse if include_coarse else 0)
    out = dict(
        ray_obj=np.empty((n, 6), np.float64),
        t=np.empty((n, S), np.float64),
        dt=np.empty((n, S), np.float64),
        bins=np.empty((n, n_fine), np.int32),
        flags=np.empty(n, np.uint8),
        margin=np.empty(n, np.float64),
    )
    lib().orc_sample(C.byref(cfg), _p(rays_o, _f32p), _p(rays_d, _f32p), _p(xi, _f32p), n,
                     _p(out["ray_obj"], _f64p), _p(out["t"], _f64p), _p(out["dt"], _f64p),
                     _p(out["bins"], _i32p), _p(out["flags"], _u8p), _p(out["margin"], _f64p))
    return out


# ---------------------------------------------------------------- encoding / MLP

def positions(ray_obj, t):
    """FP32 sample positions clamp(fmaf(t, d, o), 0, 1), [n, S, 3]."""
    ray_obj = _f32(ray_obj).reshape(-1, 6)
    n = ray_obj.shape[0]
    t = _f32(t).reshape(n, -1)
    out = np.empty((n, t.shape[1], 3), np.float32)
    lib().orc_positions(_p(ray_obj, _f32p), _p(t, _f32p), n, t.shape[1], _p(out, _f32p))
    return out


def encode(arch, table, pos, with_corners=False, emulate=False):
    """Hash-grid features y [L, n, F] (FP64); optionally the corner indices
    and weights [L, n, 8]."""
    table = _f32(table)
    pos = _f32(pos).reshape(-1, 3)
    n = pos.shape[0]
    a = make_arch(arch, emulate)
    y = np.empty((arch.n_levels, n, arch.n_features), np.float64)
    idx = np.empty((arch.n_levels, n, 8), np.int32) if with_corners else None
    w = np.empty((arch.n_levels, n, 8), np.float64) if with_corners else None
    lib().orc_encode(C.byref(a), _p(table, _f32p), _p(pos, _f32p), n, _p(y, _f64p),
                     _p(idx, _i32p), _p(w, _f64p))
    return (y, idx, w) if with_corners else y


def mlp_fwd(arch, mlp, y, emulate=False):
    """Raw head outputs [n, 4] for row-major inputs y [n, L*F]."""
    mlp = _f32(mlp)
    y = _f64(y)
    n = y.shape[0]
    out = np.empty((n, 4), np.float64)
    lib().orc_mlp_fwd(C.byref(make_arch(arch, emulate)), _p(mlp, _f32p), _p(y, _f64p), n, _p(out, _f64p))
    return out


def prior_refresh(arch, params, R, emulate=False):
    """Density grid of the NeRF: sigma = exp(o_0) at the vertices
    (i, j, k) / (R - 1), as [R, R, R] FP64 indexed [k][j][i] (x fastest), the
    layout the sampler's prior lookup reads."""
    params = _f32(params)
    out = np.empty((R, R, R), np.float64)
    lib().orc_prior_refresh(C.byref(make_arch(arch, emulate)), _p(params, _f32p), R, _p(out, _f64p))
    return out


def canonical_yaw(points, prior, n_yaw):
    """Eq. (3): scores [K] of the yaws 2 pi k / K, the extents and centres
    [K, 3] of the rotated cloud, and the first index of largest score."""
    points = _f32(points).reshape(-1, 3)
    prior = _f32(prior)
    K = int(n_yaw)
    scores, ext, cen = np.empty(K), np.empty((K, 3)), np.empty((K, 3))
    best = np.zeros(1, np.int32)
    lib().orc_canonical_yaw(_p(points, _f32p), points.shape[0], _p(prior, _f32p), prior.shape[0], K,
                            _p(scores, _f64p), _p(ext, _f64p), _p(cen, _f64p), _p(best, _i32p))
    return dict(scores=scores, extents=ext, centers=cen, best=int(best[0]))


def round16(x, dtype: str):
    """The emulation's rounding: via FP32 to the nearest bfloat16 / binary16
    value, ties to even ("fp32" leaves x unchanged)."""
    x = _f64(np.asarray(x, np.float64)).ravel()
    out = np.empty_like(x)
    lib().orc_round16_array(_p(x, _f64p), x.size, {"fp32": 0, "bf16": 1, "fp16": 2}[dtype], _p(out, _f64p))
    return out


# ---------------------------------------------------------------- compositing

def composite_fwd(sigma, rgb, t, dt, bg):
    sigma, rgb, t, dt, bg = (_f64(v) for v in (sigma, rgb, t, dt, bg))
    n, S = sigma.shape
    C3 = np.empty((n, 3)); D = np.empty(n); A = np.empty(n)
    w = np.empty((n, S)); T = np.empty((n, S + 1))
    lib().orc_composite_fwd(n, S, _p(sigma, _f64p), _p(rgb, _f64p), _p(t, _f64p), _p(dt, _f64p),
                            _p(bg, _f64p), _p(C3, _f64p), _p(D, _f64p), _p(A, _f64p),
                            _p(w, _f64p), _p(T, _f64p))
    return dict(rgb=C3, depth=D, opacity=A, w=w, T=T)


def composite_bwd(sigma, rgb, t, dt, bg, gC, gD, gA=None):
    sigma, rgb, t, dt, bg, gC, gD, gA = (_f64(v) for v in (sigma, rgb, t, dt, bg, gC, gD, gA))
    n, S = sigma.shape
    dsig = np.empty((n, S)); drgb = np.empty((n, S, 3))
    lib().orc_composite_bwd(n, S, _p(sigma, _f64p), _p(rgb, _f64p), _p(t, _f64p), _p(dt, _f64p),
                            _p(bg, _f64p), _p(gC, _f64p), _p(gD, _f64p), _p(gA, _f64p),
                            _p(dsig, _f64p), _p(drgb, _f64p))
    return dsig, drgb


# ---------------------------------------------------------------- render

def _render_cfg(arch, n_samples, loss_mode, lambda_d, lambda_sigma, emulate=False, grad_scale=1.0,
                jitter=0.0, jitter_features=None, jitter_seed=0):
    c = OrcRenderCfg()
    c.jitter = float(jitter)
    c.jitter_features = float(jitter if jitter_features is None else jitter_features)
    c.jitter_seed = int(jitter_seed)
    c.arch = make_arch(arch, emulate)
    c.n_samples = n_samples
    c.loss_mode = loss_mode
    c.lambda_d = float(np.float32(lambda_d))
    c.lambda_sigma = float(np.float32(lambda_sigma))
    c.grad_scale = float(grad_scale)
    return c


def render_fwd(arch, params, ray_obj, t, dt, flags, *, bg=None, tgt_rgb=None, tgt_depth=None,
               mask=None, loss_mode=0, lambda_d=0.0, lambda_sigma=0.0, want_samples=False,
               want_relu_signature=False, emulate=False, jitter=0.0, jitter_features=None, jitter_seed=0):
    """Per-ray colour, depth, opacity (and loss terms with targets).  jitter
    (diagnostic, 0 = off): every encoded feature and MLP pre-activation is
    moved by a pseudo-random amount of up to `jitter` times the sum of the
    absolute terms that formed it, before it is rounded or its ReLU decided,
    so that want_relu_signature can reveal the rays whose ReLU pattern
    arithmetic at that scale could change; jitter_features (default: jitter)
    sets the scale for the encoded features alone."""
    params = _f32(params)
    ray_obj = _f32(ray_obj).reshape(-1, 6)
    n = ray_obj.shape[0]
    t = _f32(t).reshape(n, -1)
    S = t.shape[1]
    dt = _f32(dt).reshape(n, S)
    flags = _u8(flags)
    bg, tgt_rgb, tgt_depth, mask = _f32(bg), _f32(tgt_rgb), _f32(tgt_depth), _u8(mask)
    cfg = _render_cfg(arch, S, loss_mode, lambda_d, lambda_sigma, emulate, jitter=jitter,
                      jitter_features=jitter_features, jitter_seed=jitter_seed)
    out = dict(rgb=np.empty((n, 3)), depth=np.empty(n), opacity=np.empty(n))
    ray_loss = np.empty(n) if tgt_rgb is not None else None
    loss = np.zeros(1) if tgt_rgb is not None else None
    samples = np.empty((n, S, 4)) if want_samples else None
    sig = np.empty(n, np.uint64) if want_relu_signature else None
    lib().orc_render_fwd(C.byref(cfg), _p(params, _f32p), _p(ray_obj, _f32p), _p(t, _f32p),
                         _p(dt, _f32p), _p(flags, _u8p), n, _p(bg, _f32p), _p(tgt_rgb, _f32p),
                         _p(tgt_depth, _f32p), _p(mask, _u8p), _p(out["rgb"], _f64p),
                         _p(out["depth"], _f64p), _p(out["opacity"], _f64p), _p(ray_loss, _f64p),
                         _p(loss, _f64p), _p(samples, _f64p), _p(sig, C.POINTER(C.c_uint64)))
    if tgt_rgb is not None:
        out["ray_loss"] = ray_loss
        out["loss"] = float(loss[0])
    if want_samples:
        out["samples"] = samples
    if want_relu_signature:
        out["relu_signature"] = sig
    return out


def render_bwd(arch, params, ray_obj, t, dt, flags, *, bg=None, tgt_rgb=None, tgt_depth=None,
               mask=None, d_rgb=None, d_depth=None, d_opacity=None, loss_mode=0, lambda_d=0.0,
               lambda_sigma=0.0, emulate=False, loss_scale=1.0):
    """Parameter gradient [n_params] (FP64) of the fused loss, or of
    sum(d_rgb * rgb + d_depth * depth + d_opacity * opacity) when d_rgb is given.
    emulate: the reduced-precision method's own gradient (operands rounded
    as the arch's mlp_dtype / table_dtype say, gradient operands carrying
    the power-of-two loss_scale when rounded); the result is unscaled."""
    params = _f32(params)
    ray_obj = _f32(ray_obj).reshape(-1, 6)
    n = ray_obj.shape[0]
    t = _f32(t).reshape(n, -1)
    S = t.shape[1]
    dt = _f32(dt).reshape(n, S)
    flags = _u8(flags)
    bg, tgt_rgb, tgt_depth, mask = _f32(bg), _f32(tgt_rgb), _f32(tgt_depth), _u8(mask)
    d_rgb, d_depth, d_opacity = _f32(d_rgb), _f32(d_depth), _f32(d_opacity)
    cfg = _render_cfg(arch, S, loss_mode, lambda_d, lambda_sigma, emulate, loss_scale)
    grads = np.zeros(params.shape[0], np.float64)
    lib().orc_render_bwd(C.byref(cfg), _p(params, _f32p), _p(ray_obj, _f32p), _p(t, _f32p),
                         _p(dt, _f32p), _p(flags, _u8p), n, _p(bg, _f32p), _p(tgt_rgb, _f32p),
                         _p(tgt_depth, _f32p), _p(mask, _u8p), _p(d_rgb, _f32p),
                         _p(d_depth, _f32p), _p(d_opacity, _f32p), _p(grads, _f64p))
    return grads


# ---------------------------------------------------------------- Adam

def adam(params, grads, m, v, *, lr, beta1, beta2, eps, step):
    params, grads, m, v = (_f32(a) for a in (params, grads, m, v))
    n = params.shape[0]
    p_out, m_out, v_out = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_adam(n, _p(params, _f32p), _p(grads, _f32p), _p(m, _f32p), _p(v, _f32p),
                   float(np.float32(lr)), float(np.float32(beta1)), float(np.float32(beta2)),
                   float(np.float32(eps)), int(step), _p(p_out, _f64p), _p(m_out, _f64p),
                   _p(v_out, _f64p))
    return p_out, m_out, v_out


# ---------------------------------------------------------------- meta-learning

def sgd(params, grads, *, lr):
    """Eq. (1): one gradient-descent step theta - eta grad, in FP64 (eta as
    the FP32 value the device receives)."""
    return _f64(params) - float(np.float32(lr)) * _f64(grads)


def reptile_outer(theta, task_params, *, beta):
    """Eq. (2): theta + beta (theta^(q) - theta).  For several tasks trained
    from the same theta, the mean of their differences takes the place of
    the one difference (one task: Eq. (2) itself).  FP64."""
    theta = _f64(theta)
    diffs = [_f64(p) - theta for p in task_params]
    return theta + float(np.float32(beta)) * (np.sum(diffs, axis=0) / len(diffs))


def reptile_meta_step(theta, tasks, *, q, lr, beta, grad, store=np.float32):
    """One meta-iteration: every task trained from theta by q steps of
    Eq. (1), grad(task, k, params) giving the task loss's gradient at inner
    step k, then Eq. (2) over the tasks' results.  Between steps the
    parameters are kept in `store` (FP32: the precision they are stored in
    on the device; FP64 for closed-form checks)."""
    finals = []
    for task in tasks:
        p = np.asarray(theta, store)
        for k in range(q):
            p = sgd(p, grad(task, k, p), lr=lr).astype(store)
        finals.append(p)
    return reptile_outer(theta, finals, beta=beta)
