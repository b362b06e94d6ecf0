"""Architecture search with the GPU evaluator (Sec. III-A, "Architecture
Optimization"): a small search runs end to end; every evaluation yields a
finite step time and depth error, the reported Pareto set is non-dominated
among all evaluations, and the knee is one of its members."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_small_search_end_to_end():
    print("test_small_search_end_to_end", flush=True)
    from paper_2503_01582_amd.archsearch import GpuEvaluator, dominates, nsga_search
    ev = GpuEvaluator(n_train=8, n_test=1, n_tasks=2, n_meta=2, adapt_steps=3, timed_steps=3,
                      log=lambda *a: print(*a, flush=True))
    res = nsga_search(ev, pop_size=4, generations=1, seed=5, log=lambda *a: print(*a, flush=True))
    assert len(res.genomes) == 8 and res.F.shape == (8, 2)
    assert np.all(res.F[:, 0] > 0)
    front = res.front.tolist()
    assert res.knee in front
    for i in front:
        assert not any(dominates(res.F[j], res.F[i]) for j in range(len(res.F)))
    for r in ev.records:
        assert np.isfinite(r["step_ms"]) or not np.isfinite(r["depth_err"])
