"""Host logic of the architecture search (Sec. III-A, "Architecture
Optimization"): Pareto fronts against the definition of dominance by brute
force, a hand-worked crowding distance, survival, the knee of a known convex
decreasing curve, and the whole genetic loop on a mixed-variable problem
whose Pareto set is known.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2503_01582_amd.archsearch import (Var, crowding_distance, curve_knee, fit_convex_decreasing,
                                              knee_point, non_dominated_fronts, nsga_search, survivors)


def brute_fronts(F):
    """Peel fronts by the definition: a point is in the current front when no
    remaining point is at most as large in every objective and smaller in one."""
    left = list(range(len(F)))
    out = []
    while left:
        cur = [i for i in left
               if not any(np.all(F[j] <= F[i]) and np.any(F[j] < F[i]) for j in left if j != i)]
        out.append(sorted(cur))
        left = [i for i in left if i not in cur]
    return out


@pytest.mark.parametrize("seed", range(6))
def test_fronts_match_brute_force(seed):
    rng = np.random.default_rng(seed)
    F = rng.integers(0, 6, (60, 2 + seed % 2)).astype(np.float64)   # many ties and duplicates
    assert [f.tolist() for f in non_dominated_fronts(F)] == brute_fronts(F)


def test_crowding_distance_hand_worked():
    """Points (0,4), (1,2), (2,1), (4,0): both extremes of each objective are
    infinite; (1,2): (2-0)/4 + (4-1)/4 = 1.25; (2,1): (4-1)/4 + (2-0)/4 = 1.25."""
    F = np.array([[0, 4], [1, 2], [2, 1], [4, 0]], np.float64)
    d = crowding_distance(F)
    assert np.isinf(d[0]) and np.isinf(d[3])
    np.testing.assert_allclose(d[1:3], [1.25, 1.25], rtol=0, atol=1e-15)


def test_survivors_keep_fronts_then_spread():
    """Front 0 = {(0,3), (1,1.5), (1.2,1.4), (3,0)}, front 1 = {(2,2)}: asking
    for 3 keeps the two extremes and the interior point of larger crowding."""
    F = np.array([[0, 3], [1, 1.5], [1.2, 1.4], [3, 0], [2, 2]], np.float64)
    keep = sorted(survivors(F, 3).tolist())
    d = crowding_distance(F[[0, 1, 2, 3]])
    interior = 1 if d[1] > d[2] else 2
    assert keep == sorted([0, 3, interior])
    assert sorted(survivors(F, 5).tolist()) == [0, 1, 2, 3, 4]


def test_knee_of_a_known_curve():
    """Points on y = exp(-6 x): scaled to [0, 1] this is a exp(-c x) + d with
    c = 6, so the fit recovers c and its knee equals the largest-curvature
    point of the known curve, found here by a dense numerical search."""
    x = np.linspace(0, 1, 40)
    y = np.exp(-6 * x)
    yn = (y - y.min()) / (y.max() - y.min())
    a, c, d = fit_convex_decreasing(x, yn)
    assert abs(c - 6) < 1e-6
    xs = np.linspace(0, 1, 200001)
    f = (np.exp(-6 * xs) - y.min()) / (y.max() - y.min())
    d1, d2 = np.gradient(f, xs), np.gradient(np.gradient(f, xs), xs)
    kappa = d2 / (1 + d1 ** 2) ** 1.5
    assert abs(curve_knee(a, c, d) - xs[np.argmax(kappa[10:-10]) + 10]) < 1e-3
    # the chosen member of a sampled front is the one nearest that x
    F = np.stack([x * 5 + 1, y * 3 + 2], 1)
    k = knee_point(F, np.arange(len(x)))
    assert abs(x[k] - curve_knee(a, c, d)) <= 0.5 / 39 + 1e-12


def test_knee_small_sets():
    """One or two points: the one closest to the ideal point after scaling."""
    assert knee_point(np.array([[1.0, 5.0]]), np.array([7])) == 7
    assert knee_point(np.array([[1.0, 5.0], [2.0, 1.0]]), np.array([3, 9])) in (3, 9)


def test_search_finds_a_known_pareto_set():
    """x in [0, 1] (real), k in {0, 1, 2, 3} (choice), m in 0..5 (integer);
    f1 = x, f2 = g (1 - sqrt(x / g)) with g = 1 + k + m.  The Pareto set is
    k = m = 0 with any x; the search must end there, spread over x."""
    space = (Var("x", "real", lo=0.0, hi=1.0), Var("k", "cat", (0, 1, 2, 3)), Var("m", "int", lo=0, hi=5))

    def evaluate(gs):
        out = []
        for x, k, m in gs:
            g = 1.0 + k + m
            out.append((x, g * (1.0 - math.sqrt(x / g))))
        return np.array(out)

    res = nsga_search(evaluate, pop_size=24, generations=25, seed=3, space=space, log=lambda *a: None)
    front = [res.genomes[i] for i in res.front]
    assert all(k == 0 and m == 0 for _, k, m in front)
    xs = sorted(x for x, _, _ in front)
    assert xs[0] < 0.1 and xs[-1] > 0.9 and len(front) >= 8
    assert res.knee in res.front.tolist()
