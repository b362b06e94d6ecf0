"""Tolerance rules shared by the GPU parity tests.

Floating-point outputs: per tensor, max|x - ref| <= tol * max|ref| and
||x - ref||_2 <= tol * ||ref||_2 (tol = 1e-5 for the FP32 path).  Integer
outputs (bins, flags, hash rows): exact equality."""
from __future__ import annotations

import numpy as np

TOL_FP32 = 1e-5


def rel_errors(x, ref):
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = x - ref
    mx = np.abs(ref).max() if ref.size else 0.0
    n2 = np.linalg.norm(ref)
    e_max = np.abs(d).max() / mx if mx > 0 else np.abs(d).max()
    e_2 = np.linalg.norm(d) / n2 if n2 > 0 else np.linalg.norm(d)
    return float(e_max), float(e_2)


def assert_close(x, ref, tol=TOL_FP32, name=""):
    e_max, e_2 = rel_errors(x, ref)
    assert e_max <= tol and e_2 <= tol, f"{name}: max-rel {e_max:.3e}, 2-rel {e_2:.3e} > {tol:.1e}"
    return e_max, e_2
