"""Tolerance rules shared by the GPU parity tests.

Floating-point outputs: per tensor, max|x - ref| <= tol * max|ref| and
||x - ref||_2 <= tol * ||ref||_2 (tol = 1e-5 for the FP32 path).  Integer
outputs (bins, flags, hash rows): exact equality."""
from __future__ import annotations

import numpy as np

TOL_FP32 = 1e-5
# ReLU-stability check: how far each perturbation moves a value, as a
# fraction of the sum of the absolute terms that formed it (and, for the
# parameters, of their own size), and the largest share of rays a gradient
# check may leave out.  Scales: the FP32 trilinear weights (products of
# rounded fractions) put an encoded feature within a few 1e-7 of those terms;
# FP32 products and sums put an FP32 pre-activation within about 1e-6; sums of
# exact 16-bit products put a reduced-precision pre-activation within far
# less.  A ray carries 2048 encoded features and 4096 to 16384
# pre-activations, so a few percent of rays hold one that arithmetic at those
# scales can decide either way (measured 0-3.5% for 64-wide networks, 4-7%
# for 128-wide ones with two hidden layers).
KINK_FEATURES = 3e-7
KINK_REL_FP32 = 1e-6
KINK_REL_LOWP = 2e-8
MAX_KINK_SHARE = 0.10


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


def relu_stable_rays(arch, params, geo, rng, *, emulate=False, rel=None, features=KINK_FEATURES, trials=8):
    """Rays whose oracle ReLU pattern survives `trials` perturbations, each
    moving every parameter by a random relative amount of up to `rel`, every
    MLP pre-activation by up to `rel` and every encoded feature by up to
    `features` times the sum of the absolute terms that formed it (the
    oracle's jitter).  The kernels and the oracle differ by FP32 against FP64
    arithmetic, errors within those sizes; only a ray that fails this check
    can take a different ReLU decision (or, in the reduced-precision form,
    round an operand to a neighbouring 16-bit value) on the two sides, which
    changes one sample's unit delta by O(1)."""
    import oracle as orc
    if rel is None:
        rel = KINK_REL_LOWP if emulate else KINK_REL_FP32
    sig = orc.render_fwd(arch, params, *geo, want_relu_signature=True, emulate=emulate)["relu_signature"]
    keep = np.ones(sig.shape[0], bool)
    for k in range(trials):
        sgn = rng.choice([-1.0, 1.0], params.size)
        pp = params.astype(np.float64) * (1.0 + rel * sgn * rng.uniform(0.5, 1.0, params.size))
        keep &= orc.render_fwd(arch, pp.astype(np.float32), *geo, want_relu_signature=True, emulate=emulate,
                               jitter=rel, jitter_features=features,
                               jitter_seed=int(rng.integers(1, 2**62)))["relu_signature"] == sig
    return keep
