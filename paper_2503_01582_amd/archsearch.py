"""Architecture optimisation (Sec. III-A, "Architecture Optimization"): a
multi-objective, mixed-variable genetic search over a category's NeRF
architecture alpha, its meta-learning settings and its loss weight, with
the objectives training time and reconstruction error; the final alpha is
the knee of the convex decreasing curve fitted to the Pareto set.

Host code: the genetic loop (fast non-dominated sorting, crowding distance,
binary tournaments, crossover and mutation per variable kind, elitist
survival) and the knee pick.  Every evaluation runs on the GPU through the
library: the candidate is meta-trained with Reptile on instances of the
category (ReptileTrainer), adapted with Adam on unseen instances, and one
training step of an object is timed.

Run a search:  python -m paper_2503_01582_amd.archsearch --pop 12 --gens 6
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------- search space


@dataclass(frozen=True)
class Var:
    name: str
    kind: str                       # "cat" (choices), "int" (lo..hi), "real" (lo..hi, log if log=True)
    choices: Tuple = ()
    lo: float = 0.0
    hi: float = 0.0
    log: bool = False

    def sample(self, rng):
        if self.kind == "cat":
            return self.choices[int(rng.integers(len(self.choices)))]
        if self.kind == "int":
            return int(rng.integers(int(self.lo), int(self.hi) + 1))
        if self.log:
            return float(math.exp(rng.uniform(math.log(self.lo), math.log(self.hi))))
        return float(rng.uniform(self.lo, self.hi))

    def mutate(self, v, rng):
        if self.kind == "cat":
            others = [c for c in self.choices if c != v]
            return others[int(rng.integers(len(others)))] if others else v
        if self.kind == "int":
            step = int(rng.choice([-1, 1]))
            return int(min(max(v + step, int(self.lo)), int(self.hi)))
        if self.log:
            x = math.log(v) + rng.normal(0.0, 0.2 * (math.log(self.hi) - math.log(self.lo)))
            return float(math.exp(min(max(x, math.log(self.lo)), math.log(self.hi))))
        x = v + rng.normal(0.0, 0.2 * (self.hi - self.lo))
        return float(min(max(x, self.lo), self.hi))

    def cross(self, a, b, rng):
        """Child gene from parents a, b: one of them for choices and integers,
        a uniform blend (extended by 25% on both sides, clipped) for reals."""
        if self.kind in ("cat", "int"):
            return a if rng.random() < 0.5 else b
        if self.log:
            la, lb = math.log(a), math.log(b)
            lo, hi = min(la, lb), max(la, lb)
            ext = 0.25 * (hi - lo)
            x = rng.uniform(lo - ext, hi + ext)
            return float(math.exp(min(max(x, math.log(self.lo)), math.log(self.hi))))
        lo, hi = min(a, b), max(a, b)
        ext = 0.25 * (hi - lo)
        return float(min(max(rng.uniform(lo - ext, hi + ext), self.lo), self.hi))


# Hash-grid and MLP hyper-parameters of the encoding (the MLP shapes the
# library is compiled for), the meta-learning settings q, eta, beta, and the
# depth-loss weight lambda_d.
SPACE: Tuple[Var, ...] = (
    Var("n_levels", "cat", (8, 12, 16)),
    Var("log2_table", "int", lo=14, hi=19),
    Var("base_res", "cat", (8, 16, 32)),
    Var("growth", "cat", ("1.25", "1.5", "2.0")),
    Var("width", "cat", (32, 64, 128)),
    Var("hidden", "int", lo=1, hi=2),
    Var("q", "int", lo=2, hi=16),
    Var("eta", "real", lo=10.0, hi=200.0, log=True),
    Var("beta", "real", lo=0.1, hi=1.0),
    Var("lambda_d", "real", lo=0.0, hi=0.5),
)

Genome = Tuple


def random_genome(rng, space: Sequence[Var] = SPACE) -> Genome:
    return tuple(v.sample(rng) for v in space)


def as_dict(g: Genome, space: Sequence[Var] = SPACE) -> Dict:
    return {v.name: x for v, x in zip(space, g)}


# ---------------------------------------------------------------- NSGA machinery

def dominates(a, b) -> bool:
    """a dominates b (minimisation): no worse in every objective, better in one."""
    return bool(np.all(a <= b) and np.any(a < b))


def non_dominated_fronts(F: np.ndarray) -> List[np.ndarray]:
    """Fronts of F [n, m] (minimise): front 0 holds the points no other point
    dominates, front k those dominated only by points of fronts < k."""
    n = F.shape[0]
    dominated_by = [[] for _ in range(n)]
    count = np.zeros(n, np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            if dominates(F[i], F[j]):
                dominated_by[i].append(j)
                count[j] += 1
            elif dominates(F[j], F[i]):
                dominated_by[j].append(i)
                count[i] += 1
    fronts = []
    cur = [i for i in range(n) if count[i] == 0]
    while cur:
        fronts.append(np.array(sorted(cur), np.int64))
        nxt = []
        for i in cur:
            for j in dominated_by[i]:
                count[j] -= 1
                if count[j] == 0:
                    nxt.append(j)
        cur = nxt
    return fronts


def crowding_distance(F: np.ndarray) -> np.ndarray:
    """Per point of one front F [k, m]: the sum over objectives of the gap
    between its two neighbours in that objective, divided by the objective's
    range; the extreme points of each objective get infinity."""
    k, m = F.shape
    d = np.zeros(k)
    if k <= 2:
        return np.full(k, np.inf)
    for j in range(m):
        order = np.argsort(F[:, j], kind="stable")
        span = F[order[-1], j] - F[order[0], j]
        d[order[0]] = d[order[-1]] = np.inf
        if span <= 0:
            continue
        for r in range(1, k - 1):
            d[order[r]] += (F[order[r + 1], j] - F[order[r - 1], j]) / span
    return d


def rank_and_crowding(F: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    rank = np.zeros(F.shape[0], np.int64)
    crowd = np.zeros(F.shape[0])
    for r, fr in enumerate(non_dominated_fronts(F)):
        rank[fr] = r
        crowd[fr] = crowding_distance(F[fr])
    return rank, crowd


def survivors(F: np.ndarray, n: int) -> np.ndarray:
    """Indices of the n best of F: whole fronts in order, the last one cut by
    decreasing crowding distance."""
    keep: List[int] = []
    for fr in non_dominated_fronts(F):
        if len(keep) + len(fr) <= n:
            keep.extend(fr.tolist())
            continue
        cd = crowding_distance(F[fr])
        order = np.argsort(-cd, kind="stable")
        keep.extend(fr[order[:n - len(keep)]].tolist())
        break
    return np.array(keep, np.int64)


def tournament(rank, crowd, rng) -> int:
    i, j = rng.integers(0, len(rank), 2)
    if rank[i] != rank[j]:
        return int(i if rank[i] < rank[j] else j)
    return int(i if crowd[i] >= crowd[j] else j)


def offspring(pop: List[Genome], F: np.ndarray, n: int, rng, space: Sequence[Var] = SPACE,
              seen: Optional[set] = None) -> List[Genome]:
    """n new genomes: tournament parents, per-gene crossover, and mutation of
    each gene with probability 1 / len(space); genomes already evaluated are
    redrawn (a bounded number of times)."""
    rank, crowd = rank_and_crowding(F)
    seen = set(pop) if seen is None else seen
    out: List[Genome] = []
    tries = 0
    while len(out) < n:
        a, b = pop[tournament(rank, crowd, rng)], pop[tournament(rank, crowd, rng)]
        child = [v.cross(x, y, rng) for v, x, y in zip(space, a, b)]
        for k, v in enumerate(space):
            if rng.random() < 1.0 / len(space):
                child[k] = v.mutate(child[k], rng)
        g = tuple(child)
        tries += 1
        if g in seen and tries < 50 * n:
            continue
        seen.add(g)
        out.append(g)
    return out


@dataclass
class SearchResult:
    genomes: List[Genome]
    F: np.ndarray                       # [n, 2] objectives of every evaluated genome
    front: np.ndarray                   # indices of the final Pareto set
    knee: int                           # index of the chosen genome
    history: List[Dict] = field(default_factory=list)


def nsga_search(evaluate: Callable[[List[Genome]], np.ndarray], pop_size: int, generations: int, seed: int = 0,
                space: Sequence[Var] = SPACE, log=print) -> SearchResult:
    """Elitist multi-objective search: an initial random population of
    pop_size, then `generations` rounds of pop_size offspring; survivors by
    front and crowding.  evaluate(genomes) -> objectives [len, 2] (minimise)."""
    rng = np.random.default_rng(seed)
    pop = []
    while len(pop) < pop_size:
        g = random_genome(rng, space)
        if g not in pop:
            pop.append(g)
    F = np.asarray(evaluate(pop), np.float64)
    all_g, all_F = list(pop), [F]
    seen = set(pop)
    history = []
    for gen in range(generations):
        kids = offspring(pop, F, pop_size, rng, space, seen)
        Fk = np.asarray(evaluate(kids), np.float64)
        all_g += kids
        all_F.append(Fk)
        merged_g, merged_F = pop + kids, np.concatenate([F, Fk])
        keep = survivors(merged_F, pop_size)
        pop, F = [merged_g[i] for i in keep], merged_F[keep]
        front0 = non_dominated_fronts(F)[0]
        history.append(dict(generation=gen + 1, front_size=int(len(front0)),
                            best=[float(F[:, j].min()) for j in range(F.shape[1])]))
        log(f"generation {gen + 1}: front of {len(front0)}, best objectives {history[-1]['best']}")
    FA = np.concatenate(all_F)
    front = non_dominated_fronts(FA)[0]
    return SearchResult(all_g, FA, front, knee_point(FA[front], front), history)


# ---------------------------------------------------------------- knee

def fit_convex_decreasing(x: np.ndarray, y: np.ndarray) -> Tuple[float, float, float]:
    """Least-squares fit of y = a exp(-c x) + d with a >= 0, c > 0: a convex,
    decreasing curve."""
    from scipy.optimize import curve_fit
    f = lambda t, a, c, d: a * np.exp(-c * t) + d
    best = None
    for c0 in (0.5, 2.0, 8.0, 32.0):
        try:
            p, _ = curve_fit(f, x, y, p0=(max(y.max() - y.min(), 1e-6), c0, y.min()),
                             bounds=([0.0, 1e-3, -np.inf], [np.inf, 1e3, np.inf]), maxfev=20000)
        except RuntimeError:
            continue
        r = float(np.sum((f(x, *p) - y) ** 2))
        if best is None or r < best[0]:
            best = (r, p)
    if best is None:
        raise RuntimeError("no convex decreasing fit")
    return tuple(float(v) for v in best[1])


def curve_knee(a: float, c: float, d: float) -> float:
    """x in [0, 1] of largest curvature of y = a exp(-c x) + d: with
    y' = -a c e^{-cx} and y'' = a c^2 e^{-cx}, kappa = y'' / (1 + y'^2)^{3/2}
    peaks where (a c e^{-cx})^2 = 1/2, i.e. x = ln(sqrt(2) a c) / c, clipped
    to [0, 1]."""
    if a * c <= 0:
        return 0.0
    x = math.log(math.sqrt(2.0) * a * c) / c
    return min(max(x, 0.0), 1.0)


def knee_point(F_front: np.ndarray, idx: np.ndarray) -> int:
    """The knee of a two-objective Pareto set: both objectives scaled to [0, 1]
    over the set, the convex decreasing curve fitted (error against time),
    the point of largest curvature of the fit, and the member of the set
    closest to it in time.  Sets of one or two points: the member closest to
    the ideal point (0, 0)."""
    F_front = np.asarray(F_front, np.float64)
    lo, hi = F_front.min(0), F_front.max(0)
    span = np.where(hi > lo, hi - lo, 1.0)
    N = (F_front - lo) / span
    if len(N) < 3:
        return int(idx[int(np.argmin(np.hypot(N[:, 0], N[:, 1])))])
    order = np.argsort(N[:, 0], kind="stable")
    a, c, d = fit_convex_decreasing(N[order, 0], N[order, 1])
    xk = curve_knee(a, c, d)
    return int(idx[int(np.argmin(np.abs(N[:, 0] - xk)))])


# ---------------------------------------------------------------- GPU evaluator

class GpuEvaluator:
    """Objectives of a genome on the GPU: (training step time in ms, held-out
    depth error).

    * error: theta meta-trained from the random initialisation by Reptile
      (n_meta meta-iterations of n_tasks tasks x rays rays, the genome's q,
      eta, beta), then adapted with Adam for adapt_steps steps on each unseen
      instance (the genome's lambda_d); the objective is the mean absolute
      depth error on the object pixels of held-out views (the stand-in for
      the paper's Chamfer distance: meshes are not extracted here), the
      colour PSNR is recorded;
    * time: one training step of an object (sample, render, backward, Adam)
      at rays rays x 32 uniform samples, by HIP events over timed steps."""

    def __init__(self, category: int = 2, n_train: int = 16, n_test: int = 2, rays: int = 4096, n_tasks: int = 4,
                 n_meta: int = 12, adapt_steps: int = 20, timed_steps: int = 10, seed: int = 0, log=print):
        import torch
        from synth.category import category_pools, stratification
        from synth.workloads import SampleSpec, eval_views
        self.torch = torch
        self.rays, self.n_tasks, self.n_meta, self.adapt_steps = rays, n_tasks, n_meta, adapt_steps
        self.timed_steps, self.seed, self.log = timed_steps, seed, log
        self.spec = SampleSpec(n_coarse=0, n_fine=32, include_coarse=False, uniform_only=True)
        self.train = category_pools(category, n_train, 4 * rays)
        self.test = category_pools(category, n_test, 4 * rays, first_instance=100)
        self.views = [eval_views(p.scene, n_views=3, seed=300 + j, res=40) for j, p in enumerate(self.test)]
        self.dev = {f: torch.stack([torch.as_tensor(getattr(p, f)) for p in self.train]).cuda()
                    for f in ("rays_o", "rays_d", "tgt_rgb", "tgt_depth", "mask")}
        self.xi = torch.as_tensor(stratification(seed, 0, 4 * rays, self.spec.n_fine)).cuda()
        self.records: List[Dict] = []

    def arch(self, g: Dict):
        from synth.arch import Arch
        return Arch(n_levels=g["n_levels"], log2_table=g["log2_table"], base_res=g["base_res"], growth=g["growth"],
                    width=g["width"], hidden=g["hidden"])

    def _meta_train(self, arch, g: Dict) -> np.ndarray:
        from synth.params import init_params
        from synth.workloads import LossSpec, nocs_affine
        from .meta import ReptileTrainer
        torch, n, B = self.torch, self.rays, self.n_tasks
        tr = ReptileTrainer(arch, init_params(arch, self.seed), B, n, self.spec, LossSpec(lambda_d=g["lambda_d"]),
                            inner_lr=g["eta"], beta=g["beta"], world_to_obj=nocs_affine().reshape(3, 4))
        n_inst = self.dev["rays_o"].shape[0]
        for i in range(self.n_meta):
            ids = torch.as_tensor([(i * B + b) % n_inst for b in range(B)]).cuda()
            for k in range(g["q"]):
                lo = ((i * g["q"] + k) * n) % (3 * n)
                sl = slice(lo, lo + n)
                tr.load_rays(self.dev["rays_o"][ids, sl].reshape(-1, 3), self.dev["rays_d"][ids, sl].reshape(-1, 3),
                             self.xi[sl].repeat(B, 1), self.dev["tgt_rgb"][ids, sl].reshape(-1, 3),
                             self.dev["tgt_depth"][ids, sl].reshape(-1), self.dev["mask"][ids, sl].reshape(-1))
                tr.step()
            tr.outer()
        theta = tr.theta.cpu().numpy()
        del tr
        return theta

    def _adapt_and_score(self, arch, theta, g: Dict) -> Tuple[float, float, float]:
        """Mean depth error, mean PSNR over the unseen instances, and the step
        time (ms) of the last instance's training."""
        from synth.workloads import LossSpec, nocs_affine
        from . import api
        from .trainer import DeviceBatch, Trainer
        torch, n = self.torch, self.rays
        derr, psnrs, ms = [], [], None
        for j, pool in enumerate(self.test):
            tr = Trainer(arch, theta, self.spec, LossSpec(lambda_d=g["lambda_d"]))
            t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)

            def batch(k):
                lo = (k * n) % (3 * n)
                sl = slice(lo, lo + n)
                return DeviceBatch(rays_o=t(pool.rays_o[sl]), rays_d=t(pool.rays_d[sl]), xi=self.xi[sl],
                                   tgt_rgb=t(pool.tgt_rgb[sl]), tgt_depth=t(pool.tgt_depth[sl]),
                                   mask=t(pool.mask[sl], torch.uint8), world_to_obj=nocs_affine(), prior=None, bg=None)
            for k in range(self.adapt_steps):
                tr.step(batch(k))
            torch.cuda.synchronize()
            for o, d, col, depth, hit in self.views[j]:
                m = o.shape[0]
                xi = torch.full((m, self.spec.n_fine), 0.5, device="cuda")
                samp = api.prenom_sample(self.spec, t(o), t(d), xi, nocs_affine(), None)
                ws = api.Workspace().get(arch, m, self.spec.n_samples)
                out = api.prenom_render_fwd(tr.model, samp, None, ws, want_loss=False)
                rgb, dep = out["rgb"].cpu().numpy(), out["depth"].cpu().numpy()
                psnrs.append(-10.0 * math.log10(max(float(((rgb - col) ** 2).mean()), 1e-12)))
                obj = hit == 1
                derr.append(float(np.abs(dep[obj] - depth[obj]).mean()) if obj.any() else 0.0)
            if j == len(self.test) - 1:   # time steps of this object's training
                db = batch(0)
                for _ in range(3):
                    tr.step(db)
                torch.cuda.synchronize()
                s = torch.cuda.current_stream()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(self.timed_steps):
                    tr.step(db)
                e1.record(s)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / self.timed_steps
            del tr
        return float(np.mean(derr)), float(np.mean(psnrs)), float(ms)

    def __call__(self, genomes: List[Genome]) -> np.ndarray:
        out = []
        for gtuple in genomes:
            g = as_dict(gtuple)
            arch = self.arch(g)
            t0 = time.perf_counter()
            if max(arch.resolutions) >= 1 << 20:   # outside the library's grid limits: dominated by everything
                self.log(f"  {g} -> finest resolution {max(arch.resolutions)} not supported")
                self.records.append(dict(genome=g, step_ms=float("inf"), depth_err=float("inf"), psnr=float("nan"),
                                         eval_s=0.0))
                out.append((float("inf"), float("inf")))
                continue
            theta = self._meta_train(arch, g)
            if not np.all(np.isfinite(theta)):
                err, psnr, ms = float("inf"), float("nan"), float("inf")
            else:
                err, psnr, ms = self._adapt_and_score(arch, theta, g)
                if not math.isfinite(err):
                    err = float("inf")
            rec = dict(genome=g, step_ms=ms, depth_err=err, psnr=psnr, eval_s=time.perf_counter() - t0)
            self.records.append(rec)
            self.log(f"  {g} -> step {ms:.3f} ms, depth error {err:.4f}, PSNR {psnr:.2f} dB")
            out.append((ms, err))
        return np.array(out, np.float64)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pop", type=int, default=12)
    ap.add_argument("--gens", type=int, default=6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--meta", type=int, default=12, help="meta-iterations per evaluation")
    ap.add_argument("--out", default=None, help="write the evaluated genomes and the front as JSON")
    args = ap.parse_args()
    ev = GpuEvaluator(n_meta=args.meta, seed=args.seed, log=lambda *a: print(*a, flush=True))
    t0 = time.perf_counter()
    res = nsga_search(ev, args.pop, args.gens, seed=args.seed, log=lambda *a: print(*a, flush=True))
    wall = time.perf_counter() - t0
    print(f"{len(res.genomes)} evaluations in {wall:.1f} s ({wall / len(res.genomes):.2f} s each)")
    for i in sorted(res.front.tolist(), key=lambda i: res.F[i, 0]):
        mark = "  <- knee" if i == res.knee else ""
        print(f"  front: step {res.F[i, 0]:.3f} ms, depth error {res.F[i, 1]:.4f}  {as_dict(res.genomes[i])}{mark}")
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(records=ev.records, front=res.front.tolist(), knee=res.knee, history=res.history,
                           wall_s=wall), f, indent=1, default=str)


if __name__ == "__main__":
    main()
