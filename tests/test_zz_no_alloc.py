"""The allocation-free prior refresh against the workspace form, through the
C ABI: two calls in a row on one GPU (the second on a smaller grid, reusing
the library's scratch array), each checked against prenom_prior_refresh on
the same model, plus the host-side rejection of an out-of-range grid."""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import pytest

from synth.arch import ARCH_LARGE
from synth.params import init_params

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _model(arch, seed):
    from paper_2503_01582_amd import api
    p = init_params(arch, seed)
    n = arch.n_table_params
    p[:n] = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, n).astype(np.float32)
    p[n:] *= 1.5
    return api.Model(arch, p)


@pytest.mark.parametrize("mlp_dtype,table_dtype", [("fp32", "fp32"), ("bf16", "fp16")])
def test_noalloc_prior_refresh_matches_workspace_form(mlp_dtype, table_dtype):
    print(f"test_noalloc_prior_refresh_matches_workspace_form[{mlp_dtype}, {table_dtype}]", flush=True)
    from paper_2503_01582_amd import _lib, api
    from parity_util import assert_close
    arch = dataclasses.replace(ARCH_LARGE, mlp_dtype=mlp_dtype, table_dtype=table_dtype)
    model = _model(arch, 21)
    scratch = _lib.lib().prenom_noalloc_scratch_bytes()
    per_vertex = arch.n_levels * 2 * 4 + 16
    # 129^3 vertices span several scratch chunks; 33^3 fits in one
    assert 129 ** 3 > scratch // per_vertex > 33 ** 3
    for R in (129, 33):
        out = torch.full((R, R, R), float("nan"), dtype=torch.float32, device="cuda")
        api.prenom_prior_refresh_noalloc(model, R, out)
        ref = api.prenom_prior_refresh(model, R)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        want = ref.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got))
        err = assert_close(got, want, 1e-5, f"noalloc R={R}")
        print(f"  R={R}: max/2-rel {err[0]:.2e}/{err[1]:.2e}, bit-identical {np.array_equal(got, want)}",
              flush=True)


def test_noalloc_rejects_out_of_range_grid():
    print("test_noalloc_rejects_out_of_range_grid", flush=True)
    from paper_2503_01582_amd import _lib
    model = _model(ARCH_LARGE, 22)
    mc = model.c_struct()
    out = torch.zeros(8, dtype=torch.float32, device="cuda")
    for R in (1, 513):
        st = _lib.lib().prenom_prior_refresh_noalloc(C.byref(mc), R, C.c_void_p(out.data_ptr()), None)
        assert _lib.STATUS[st] == "PRENOM_ERR_SHAPE"
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
