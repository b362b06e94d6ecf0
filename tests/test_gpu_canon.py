"""Canonical yaw search on the GPU (Sec. III-B, "Object State
Canonicalization", Eq. (3)) against the oracle: scores within 1e-12 (FP64,
sums in another order), extents and centres within 1e-13, and the chosen yaw
a maximum of the oracle's scores (equal to the oracle's choice whenever the
top two scores are apart by more than the tolerance)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as orc
from parity_util import assert_close
from test_oracle_pins import l_shape_points, l_shape_prior, rot_z

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-12


def say(*a):
    print(*a, flush=True)


def gpu_yaw(P, F, K):
    from paper_2503_01582_amd import api
    r = api.prenom_canonical_yaw(torch.as_tensor(P).cuda(), torch.as_tensor(F).cuda(), K)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if k != "best" else int(v.item())) for k, v in r.items()}


def check(got, ref):
    assert_close(got["scores"], ref["scores"], TOL, "scores")
    assert_close(got["extents"], ref["extents"], 1e-13, "extents")
    assert_close(got["centers"], ref["centers"], 1e-13, "centers")
    s = ref["scores"]
    top = s.max()
    assert s[got["best"]] >= top - TOL * abs(top), "GPU choice is not a maximum of the oracle's scores"
    runner_up = np.sort(s)[-2] if s.size > 1 else -np.inf
    if runner_up < top - 10 * TOL * abs(top):   # a clear maximum: the same index
        assert got["best"] == ref["best"]


@pytest.mark.parametrize("n,K,R", [(1, 1, 2), (17, 2, 9), (4096, 72, 17), (4097, 360, 64), (100003, 97, 33)])
def test_yaw_matches_oracle(n, K, R):
    say(f"test_yaw_matches_oracle[n={n}, K={K}, R={R}]")
    rng = np.random.default_rng(n + K + R)
    P = (rng.normal(size=(n, 3)) * [0.4, 0.25, 0.3] + [1.0, -2.0, 0.3]).astype(np.float32)
    F = rng.uniform(0, 2, (R, R, R)).astype(np.float32)
    check(gpu_yaw(P, F, K), orc.canonical_yaw(P, F, K))


@pytest.mark.parametrize("k0", [0, 13, 41, 70])
def test_yaw_recovers_known_rotation(k0):
    say(f"test_yaw_recovers_known_rotation[{k0}]")
    rng = np.random.default_rng(k0 + 100)
    K = 72
    P = l_shape_points(rng, 20000) @ rot_z(-2 * math.pi * k0 / K).T
    P = (P * 0.8 + np.array([-1.0, 4.0, 0.2])).astype(np.float32)
    F = l_shape_prior(64)
    got = gpu_yaw(P, F, K)
    assert got["best"] == k0
    check(got, orc.canonical_yaw(P, F, K))


def test_yaw_degenerate_clouds():
    """A repeated point (every extent 0) and a flat cloud (z extent 0)."""
    say("test_yaw_degenerate_clouds")
    rng = np.random.default_rng(3)
    F = rng.uniform(0, 1, (9, 9, 9)).astype(np.float32)
    P = np.tile(np.float32([[0.3, -0.1, 0.2]]), (5000, 1))
    got = gpu_yaw(P, F, 36)
    check(got, orc.canonical_yaw(P, F, 36))
    assert got["best"] == 0 and np.all(got["extents"] == 0)
    flat = rng.normal(size=(3000, 3)).astype(np.float32)
    flat[:, 2] = 0.5
    check(gpu_yaw(flat, F, 40), orc.canonical_yaw(flat, F, 40))


def test_yaw_large_cloud_sampled():
    """2^22 points, 360 yaws, the 64^3 grid: the yaws 45 m (m = 0..7) are the
    oracle's yaws 2 pi m / 8, compared one by one."""
    say("test_yaw_large_cloud_sampled")
    rng = np.random.default_rng(11)
    n = 1 << 22
    P = (rng.normal(size=(n, 3)) * [0.4, 0.25, 0.3]).astype(np.float32)
    F = rng.uniform(0, 1, (64, 64, 64)).astype(np.float32)
    got = gpu_yaw(P, F, 360)
    ref = orc.canonical_yaw(P, F, 8)
    assert_close(got["scores"][::45], ref["scores"], TOL, "scores at 8 yaws")
    assert_close(got["extents"][::45], ref["extents"], 1e-13, "extents at 8 yaws")
    say(f"  scores range [{got['scores'].min():.6e}, {got['scores'].max():.6e}], best {got['best']}")


def test_yaw_argument_errors():
    say("test_yaw_argument_errors")
    from paper_2503_01582_amd import api
    P = torch.zeros((10, 3), device="cuda")
    F = torch.zeros((4, 4, 4), device="cuda")
    for K in (0, 4097):
        with pytest.raises(Exception):
            api.prenom_canonical_yaw(P, F, K)
    with pytest.raises(Exception):
        api.prenom_canonical_yaw(torch.zeros((0, 3), device="cuda"), F, 8)
    with pytest.raises(Exception):
        api.prenom_canonical_yaw(P, torch.zeros((1, 1, 1), device="cuda"), 8)
