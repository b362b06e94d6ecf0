"""ctypes view of libprenom.so (the C ABI declared in include/prenom.h).

Argument marshalling only.  Loading fails loudly when the HIP library has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

MAX_LEVELS = 32
F32, BF16, F16 = 0, 1, 2
N_OUT = 4
FLAG_MISS, FLAG_ESCAPED, FLAG_UNIFORM = 1, 2, 4

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libprenom.so")

STATUS = {0: "PRENOM_OK", 1: "PRENOM_ERR_INVALID_ARG", 2: "PRENOM_ERR_SHAPE",
          3: "PRENOM_ERR_UNSUPPORTED", 4: "PRENOM_ERR_WORKSPACE", 5: "PRENOM_ERR_HIP"}


class PrenomArch(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("log2_table", C.c_int32), ("n_features", C.c_int32),
                ("resolution", C.c_int32 * MAX_LEVELS), ("mlp_width", C.c_int32),
                ("mlp_hidden", C.c_int32), ("mlp_dtype", C.c_int32), ("table_dtype", C.c_int32)]


class PrenomModel(C.Structure):
    _fields_ = [("arch", PrenomArch), ("params", C.c_void_p), ("grads", C.c_void_p),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p), ("table_lp", C.c_void_p),
                ("loss_scale", C.c_void_p), ("scaler_state", C.c_void_p)]


class PrenomSampleCfg(C.Structure):
    _fields_ = [("n_coarse", C.c_int32), ("n_fine", C.c_int32), ("include_coarse", C.c_int32),
                ("uniform_only", C.c_int32), ("eps", C.c_float), ("near_t", C.c_float),
                ("far_t", C.c_float), ("world_to_obj", C.c_float * 12), ("prior", C.c_void_p),
                ("prior_res", C.c_int32)]


class PrenomRenderCfg(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("loss_mode", C.c_int32), ("lambda_d", C.c_float),
                ("lambda_sigma", C.c_float), ("recompute", C.c_int32)]


class PrenomAdamCfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int64), ("growth_interval", C.c_int32)]


class PrenomSgdCfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("growth_interval", C.c_int32)]


class PrenomObject(C.Structure):
    _fields_ = [("arch", PrenomArch), ("n_rays", C.c_int64), ("prior", C.c_void_p),
                ("prior_res", C.c_int32), ("world_to_obj", C.c_float * 12)]


class PrenomMlpTiles(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("width", C.c_int32), ("hidden", C.c_int32), ("dtype", C.c_int32),
                ("fwd_tiles", C.c_int32), ("bwd_tiles", C.c_int32)]


class PrenomBatch(C.Structure):
    _fields_ = [("n_objects", C.c_int32), ("objects", C.POINTER(PrenomObject)), ("n_tiles", C.c_int32),
                ("tiles", C.POINTER(PrenomMlpTiles)), ("params", C.c_void_p), ("grads", C.c_void_p),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p), ("params_lp", C.c_void_p),
                ("loss_scale", C.c_void_p), ("scaler_state", C.c_void_p), ("step", C.c_void_p),
                ("record_budget", C.c_int64)]


class PrenomKernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


class PrenomError(RuntimeError):
    pass


_vp = C.c_void_p
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PrenomError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        L.prenom_param_count.restype = C.c_int64
        L.prenom_param_count.argtypes = [C.POINTER(PrenomArch)]
        L.prenom_table_param_count.restype = C.c_int64
        L.prenom_table_param_count.argtypes = [C.POINTER(PrenomArch)]
        L.prenom_workspace_size.restype = C.c_size_t
        L.prenom_workspace_size.argtypes = [C.POINTER(PrenomArch), C.c_int64, C.c_int32, C.c_int32]
        L.prenom_sample.restype = C.c_int
        L.prenom_sample.argtypes = [C.POINTER(PrenomSampleCfg), _vp, _vp, _vp, C.c_int64,
                                    _vp, _vp, _vp, _vp, _vp, _vp]
        L.prenom_render_fwd.restype = C.c_int
        L.prenom_render_fwd.argtypes = [C.POINTER(PrenomModel), C.POINTER(PrenomRenderCfg),
                                        _vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.prenom_render_bwd.restype = C.c_int
        L.prenom_render_bwd.argtypes = [C.POINTER(PrenomModel), C.POINTER(PrenomRenderCfg),
                                        _vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.prenom_adam_step.restype = C.c_int
        L.prenom_adam_step.argtypes = [C.POINTER(PrenomModel), C.POINTER(PrenomAdamCfg), _vp]
        L.prenom_refresh_lowp.restype = C.c_int
        L.prenom_refresh_lowp.argtypes = [C.POINTER(PrenomModel), _vp]
        L.prenom_encode.restype = C.c_int
        L.prenom_encode.argtypes = [C.POINTER(PrenomArch), _vp, _vp, C.c_int64, _vp, _vp, _vp]
        L.prenom_prior_refresh_workspace_size.restype = C.c_size_t
        L.prenom_prior_refresh_workspace_size.argtypes = [C.POINTER(PrenomArch), C.c_int32]
        L.prenom_prior_refresh.restype = C.c_int
        L.prenom_prior_refresh.argtypes = [C.POINTER(PrenomModel), C.c_int32, _vp, _vp, C.c_size_t, _vp]
        L.prenom_noalloc_scratch_bytes.restype = C.c_size_t
        L.prenom_noalloc_scratch_bytes.argtypes = []
        L.prenom_prior_refresh_noalloc.restype = C.c_int
        L.prenom_prior_refresh_noalloc.argtypes = [C.POINTER(PrenomModel), C.c_int32, _vp, _vp]
        PB = C.POINTER(PrenomBatch)
        L.prenom_batch_param_count.restype = C.c_int64
        L.prenom_batch_param_count.argtypes = [C.POINTER(PrenomObject), C.c_int32]
        L.prenom_batch_param_offset.restype = C.c_int64
        L.prenom_batch_param_offset.argtypes = [C.POINTER(PrenomObject), C.c_int32, C.c_int32]
        L.prenom_batch_workspace_size.restype = C.c_size_t
        L.prenom_batch_workspace_size.argtypes = [PB, C.c_int32]
        L.prenom_batch_prepare.restype = C.c_int
        L.prenom_batch_prepare.argtypes = [PB, C.c_int32, _vp, C.c_size_t, _vp]
        L.prenom_batch_sample.restype = C.c_int
        L.prenom_batch_sample.argtypes = [PB, C.POINTER(PrenomSampleCfg), _vp, _vp, _vp, _vp, _vp, _vp,
                                          _vp, _vp, _vp, C.c_size_t, _vp]
        L.prenom_batch_render_fwd.restype = C.c_int
        L.prenom_batch_render_fwd.argtypes = [PB, C.POINTER(PrenomRenderCfg), _vp, _vp, _vp, _vp, _vp, _vp,
                                              _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.prenom_batch_render_bwd.restype = C.c_int
        L.prenom_batch_render_bwd.argtypes = [PB, C.POINTER(PrenomRenderCfg), _vp, _vp, _vp, _vp, _vp, _vp,
                                              _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.prenom_batch_adam_step.restype = C.c_int
        L.prenom_batch_adam_step.argtypes = [PB, C.POINTER(PrenomAdamCfg), _vp]
        L.prenom_batch_refresh_lowp.restype = C.c_int
        L.prenom_batch_refresh_lowp.argtypes = [PB, _vp]
        L.prenom_canonical_yaw_workspace_size.restype = C.c_size_t
        L.prenom_canonical_yaw_workspace_size.argtypes = [C.c_int64, C.c_int32]
        L.prenom_canonical_yaw.restype = C.c_int
        L.prenom_canonical_yaw.argtypes = [_vp, C.c_int64, _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp,
                                           C.c_size_t, _vp]
        L.prenom_sgd_step.restype = C.c_int
        L.prenom_sgd_step.argtypes = [C.POINTER(PrenomModel), C.POINTER(PrenomSgdCfg), _vp]
        L.prenom_batch_sgd_step.restype = C.c_int
        L.prenom_batch_sgd_step.argtypes = [PB, C.POINTER(PrenomSgdCfg), _vp]
        L.prenom_reptile_update.restype = C.c_int
        L.prenom_reptile_update.argtypes = [_vp, _vp, C.c_int64, C.c_int32, C.c_int64, C.c_float, _vp, _vp, _vp,
                                            C.c_int64, _vp, _vp]
        L.prenom_profile_begin.restype = C.c_int
        L.prenom_profile_begin.argtypes = []
        L.prenom_profile_end.restype = C.c_int
        L.prenom_profile_end.argtypes = [C.POINTER(PrenomKernelTime), C.c_int32, C.POINTER(C.c_int32)]
        L.prenom_status_string.restype = C.c_char_p
        L.prenom_status_string.argtypes = [C.c_int]
        L.prenom_last_error.restype = C.c_char_p
        L.prenom_last_error.argtypes = []
        L.prenom_version.restype = C.c_char_p
        L.prenom_version.argtypes = []
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != 0:
        msg = lib().prenom_last_error().decode(errors="replace")
        raise PrenomError(f"{what}: {STATUS.get(status, status)}: {msg}")
