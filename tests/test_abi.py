"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, reports sizes consistent with the parameter layout, and
rejects bad arguments on the host before anything is launched."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

from synth.arch import ARCH_LARGE, ARCH_SMALL, Arch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "prenom.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(prenom_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2503_01582_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 12, names
    lib = L.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_param_and_workspace_sizes(L):
    from paper_2503_01582_amd import api
    for arch in (ARCH_SMALL, ARCH_LARGE):
        assert api.prenom_param_count(arch) == arch.n_params
        assert api.prenom_table_param_count(arch) == arch.n_table_params
        a = api.prenom_workspace_size(arch, 1000, 64)
        b = api.prenom_workspace_size(arch, 2000, 64)
        assert 0 < a < b and a % 256 == 0
        # the recompute form holds one pass of about 2^21 samples, whatever the batch
        r1 = api.prenom_workspace_size(arch, 1 << 16, 64, recompute=True)
        r2 = api.prenom_workspace_size(arch, 1 << 20, 64, recompute=True)
        assert 0 < r1 <= r2 < 1.01 * r1 and r2 < api.prenom_workspace_size(arch, 1 << 16, 64) / 1.5
    bad = Arch(n_levels=4, log2_table=8, width=16, hidden=1)  # log2_table below 10
    assert api.prenom_param_count(bad) == -1


def test_unsupported_architecture_is_rejected_before_launch(L):
    from paper_2503_01582_amd import api
    arch = Arch(n_levels=16, log2_table=19, width=96, hidden=2)  # MLP width not compiled
    m = L.PrenomModel()
    m.arch = api.make_arch(arch)
    cfg = L.PrenomRenderCfg(64, 0, 0.0, 0.0)
    st = L.lib().prenom_render_fwd(C.byref(m), C.byref(cfg), *([None] * 4), 0, *([None] * 10), 0, None)
    assert L.STATUS[st] == "PRENOM_ERR_UNSUPPORTED"
    assert b"not compiled" in L.lib().prenom_last_error()


def test_invalid_sampler_arguments(L):
    c = L.PrenomSampleCfg()
    c.n_coarse, c.n_fine, c.include_coarse, c.uniform_only = 16, 0, 1, 0
    c.eps, c.near_t, c.far_t = 1e-4, 0.5, 2.5
    st = L.lib().prenom_sample(C.byref(c), *([None] * 3), 10, *([None] * 5), None)
    assert L.STATUS[st] == "PRENOM_ERR_SHAPE"
    c.n_fine = 48
    c.far_t = 0.1  # near > far
    st = L.lib().prenom_sample(C.byref(c), *([None] * 3), 10, *([None] * 5), None)
    assert L.STATUS[st] == "PRENOM_ERR_INVALID_ARG"
    c.far_t = 2.5
    st = L.lib().prenom_sample(C.byref(c), *([None] * 3), 10, *([None] * 5), None)  # NULL arrays
    assert L.STATUS[st] == "PRENOM_ERR_INVALID_ARG"
    assert L.lib().prenom_status_string(0) == b"ok"


def test_encode_rejects_misaligned_table(L):
    """Table rows are read in aligned pairs (16 bytes); an 8-byte aligned
    table is refused on the host, before any launch."""
    from paper_2503_01582_amd import api
    a = api.make_arch(ARCH_SMALL)
    fake = 1 << 20  # never dereferenced: the checks fail first
    st = L.lib().prenom_encode(C.byref(a), C.c_void_p(fake + 8), C.c_void_p(fake), 4, C.c_void_p(fake), None, None)
    assert L.STATUS[st] == "PRENOM_ERR_INVALID_ARG"
    assert b"16-byte" in L.lib().prenom_last_error()


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2503_01582_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", txt.replace("oracle-free", "")), f


def test_no_stray_c_exports():
    """Every exported symbol with C linkage is part of the ABI (prenom_*);
    helpers stay internal (C++ names, or file-local)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    from paper_2503_01582_amd import _lib
    out = subprocess.run([nm, "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    names = [ln.split()[-1] for ln in out.stdout.splitlines() if ln.strip()]
    stray = [n for n in names if not n.startswith(("prenom_", "_Z", "__hip_cuid"))]
    assert stray == []
