"""Search strategies over the variant space.

All strategies see the space only through an evaluator (measure or replay a
variant, returning mean and standard deviation of the score and the benchmark
cost in seconds) and stop once their benchmark budget is spent:

  exhaustive   every variant (the ground truth);
  random       variants in a seeded random order;
  pagsa        the paper's genetic simulated annealing: parents drawn from the
               database at a random temperature, children by mutation,
               crossover or triangulation with probability 1/3 each;
  mlp          an ensemble of MLP cost models, trained on the GPU on what has
               been measured so far, proposes the next variants to benchmark
               (each member picks one of a batch: Thompson-style sampling).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import space as sp


@dataclass
class Trace:
    strategy: str
    evaluated: list = field(default_factory=list)   # (key, mu, cost) in order
    spent: float = 0.0
    best_key: str | None = None
    best_mu: float = 0.0

    def record(self, k: str, mu: float, cost: float):
        self.evaluated.append((k, mu, cost))
        self.spent += cost
        if mu > self.best_mu:
            self.best_mu, self.best_key = mu, k

    def anytime(self, optimum: float, budget: float) -> float:
        """Mean over the budget of the best-so-far fraction of the optimum (area under the
        best-so-far curve, benchmark seconds on the x axis, normalised to 1)."""
        area, t, best = 0.0, 0.0, 0.0
        for _, mu, cost in self.evaluated:
            step = min(cost, max(budget - t, 0.0))
            area += best * step
            t += step
            best = max(best, mu / optimum)
        area += best * max(budget - t, 0.0)
        return area / budget


class ReplayEvaluator:
    """Answers from a database of measured individuals (exhaustive run)."""

    def __init__(self, db):
        self.db = db

    def __call__(self, variant: dict) -> dict:
        r = self.db.get(sp.key(variant))
        if r is None:
            raise KeyError(sp.key(variant))
        return {"mu": r["mu"] if r["valid"] else 0.0, "sigma": r.get("sigma", 0.0), "cost": r["cost"],
                "valid": r["valid"]}


class LiveEvaluator:
    """Benchmarks on the GPU and appends every individual to the database."""

    def __init__(self, bench, db, ndim: int, log=None):
        self.bench, self.db, self.ndim = bench, db, ndim
        self.log = log or (lambda s: None)

    def __call__(self, variant: dict, parents=None, birth=None) -> dict:
        k = sp.key(variant)
        r = self.db.get(k)
        if r is None:
            res = self.bench.measure(variant)
            r = self.db.add({"key": k, "genome": sp.encode(variant, self.ndim), "variant": variant,
                             "parents": parents, "birth": birth, **res})
            self.log(f"{k}: valid={r['valid']} mu={r['mu'] / 1e9:.3f} Gcups sigma={r['sigma'] / 1e9:.3f} "
                     f"cost={r['cost']:.2f}s {r.get('reason', '')}")
        return {"mu": r["mu"] if r["valid"] else 0.0, "sigma": r.get("sigma", 0.0), "cost": r["cost"],
                "valid": r["valid"]}


def candidates(ndim: int, esize: int, manifest: bool = False) -> list:
    return [v for v in sp.enumerate_space(ndim, manifest) if sp.statically_valid(v, ndim, esize)]


def exhaustive(cands, evaluate) -> Trace:
    tr = Trace("exhaustive")
    for v in cands:
        r = evaluate(v)
        tr.record(sp.key(v), r["mu"], r["cost"])
    return tr


def random_search(cands, evaluate, budget: float, rng: np.random.Generator) -> Trace:
    tr = Trace("random")
    for i in rng.permutation(len(cands)):
        if tr.spent >= budget:
            break
        r = evaluate(cands[i])
        tr.record(sp.key(cands[i]), r["mu"], r["cost"])
    return tr


# ---- PAGSA -------------------------------------------------------------------------------

def draw_weights(mus: np.ndarray, sigmas: np.ndarray, T: float) -> np.ndarray:
    """Draw probabilities at temperature T.  The weight of individual I is
    exp(-(mu_top - mu_I + s_top + s_I) / (T + s_top + s_I)), I_top the best
    individual: low temperatures prefer high scores, differences small
    against the deviations are ignored.  (The exponent's sign is printed
    positive in the paper; the negative sign is the one that makes low
    temperatures prefer high scores, as the text states.)"""
    top = int(np.argmax(mus))
    mt, st = mus[top], sigmas[top]
    z = -(mt - mus + st + sigmas) / (T + st + sigmas)
    z -= z.max()
    w = np.exp(z)
    return w / w.sum()


def draw_temperature(mus, sigmas, rng) -> float:
    """log T uniform between log sigma_top and log mu_top."""
    top = int(np.argmax(mus))
    lo = math.log(max(sigmas[top], 1e-12 * max(mus[top], 1.0)))
    hi = math.log(max(mus[top], 1e-300))
    if hi <= lo:
        return math.exp(hi)
    return math.exp(rng.uniform(lo, hi))


def triangulate(base: str, secondary: str, primary: str) -> str:
    """Bit-wise three-parent crossover: a bit takes the change if the Primary
    or the Secondary changed it from the Base (binary table of the paper)."""
    out = []
    for b, s, p in zip(base, secondary, primary):
        out.append(p if p != b else s)
    return "".join(out)


def mutate(g: str, rng) -> str:
    bits = list(g)
    n = 1 + int(rng.integers(0, 2))
    for i in rng.choice(len(bits), size=n, replace=False):
        bits[i] = "1" if bits[i] == "0" else "0"
    return "".join(bits)


def crossover(a: str, b: str, rng) -> str:
    """Split both genomes at two random points and exchange the middle segment."""
    L = len(a)
    i, j = sorted(rng.choice(L + 1, size=2, replace=False))
    return a[:i] + b[i:j] + a[j:]


BIRTHS = ("mutation", "crossover", "triangulation")


def pagsa_birth(known: dict, rng, taken=()):
    """One birth of the paper's genetic simulated annealing.  `known` maps the
    genomes in the database to (mu, sigma) (mu = 0 for invalid ones); at a
    random temperature, one to three distinct parents are drawn by the draw
    weights and combined by mutation, crossover or triangulation (probability
    1/3 each; triangulation orders its parents Base < Secondary < Primary by
    score).  A child already known, or in `taken` (being benchmarked
    elsewhere), is redrawn at a 1.2 times higher temperature.  Returns
    (child genome, parent genomes, method) or None after 200 draws.  The
    caller makes sure some mu is positive."""
    genomes = list(known)
    mus = np.array([known[g][0] for g in genomes])
    sig = np.array([known[g][1] for g in genomes])
    T = draw_temperature(mus, sig, rng)
    method = int(rng.integers(0, 3))
    need = (1, 2, 3)[method]
    for _ in range(200):
        w = draw_weights(mus, sig, T)
        idx = rng.choice(len(genomes), size=need, replace=True, p=w)
        if len(set(idx.tolist())) < need:
            continue  # two parents coincide: draw again
        par = [genomes[i] for i in idx]
        if method == 0:
            c = mutate(par[0], rng)
        elif method == 1:
            c = crossover(par[0], par[1], rng)
        else:
            base, sec, prim = sorted(par, key=lambda g: known[g][0])
            c = triangulate(base, sec, prim)
        if c in known or c in taken:
            T *= 1.2  # duplicate genome: retry at a higher temperature
            continue
        return c, par, BIRTHS[method]
    return None


def pagsa(cands, evaluate, budget: float, rng, ndim: int, seed_variants) -> Trace:
    tr = Trace("pagsa")
    valid_keys = {sp.key(v) for v in cands}
    known = {}  # genome -> (mu, sigma)

    def run(v, parents=None, birth=None):
        g = sp.encode(v, ndim)
        if sp.key(v) in valid_keys:
            r = evaluate(v)
            tr.record(sp.key(v), r["mu"], r["cost"])
            known[g] = (r["mu"], r["sigma"])
        else:
            known[g] = (0.0, 0.0)  # cannot run on this hardware: score 0, no benchmark cost

    for v in seed_variants:
        if tr.spent >= budget:
            break
        run(v, birth="seed")
    while tr.spent < budget:
        if max(m for m, _ in known.values()) <= 0:
            break
        child = pagsa_birth(known, rng)
        if child is None:
            # every draw produced a known genome; fall back to an unseen random one
            unseen = [v for v in cands if sp.encode(v, ndim) not in known]
            if not unseen:
                break
            child = (sp.encode(unseen[int(rng.integers(0, len(unseen)))], ndim), [], "random")
        run(sp.decode(child[0], ndim), parents=child[1], birth=child[2])
    return tr


# ---- MLP-guided --------------------------------------------------------------------------

def mlp_guided(cands, evaluate, budget: float, rng, ndim: int, esize: int, init: int = 8, batch: int = 8,
               epochs: int = 200, ensemble: int = 8, model_seed: int = 0) -> Trace:
    """Model-guided search.  After `init` random variants, rounds of: fit an
    ensemble of networks (different initial weights) to the standardised log
    speed of everything measured, then benchmark `batch` unmeasured variants,
    the b-th being the best predicted by member b mod `ensemble`.  The members
    agree where the data pin the model down and disagree elsewhere, so the
    batch mixes exploitation with exploration of regions still uncertain
    (a cheap form of Thompson sampling); a single greedy model tends to
    settle on the first good region it finds."""
    from .model import CostModel
    tr = Trace("mlp")
    F = np.array([sp.features(v, ndim, esize) for v in cands], dtype=np.float64)
    mean, std = F.mean(axis=0), F.std(axis=0)
    std[std == 0] = 1.0
    Fn = (F - mean) / std
    measured = {}
    order = rng.permutation(len(cands))
    for i in order[:init]:
        if tr.spent >= budget:
            break
        r = evaluate(cands[i])
        measured[int(i)] = r["mu"]
        tr.record(sp.key(cands[i]), r["mu"], r["cost"])
    models = [CostModel(F.shape[1], 64, seed=model_seed * 16 + e) for e in range(ensemble)]
    while tr.spent < budget and len(measured) < len(cands):
        idx = np.array(sorted(measured))
        y = np.array([measured[i] for i in idx])
        ok = y > 0
        if ok.sum() < 2:
            pick = [int(i) for i in order if int(i) not in measured][:batch]
        else:
            ly = np.log(np.where(ok, y, y[ok].min() * 0.5))
            mu_y, sd_y = ly.mean(), ly.std() + 1e-9
            preds = []
            for m in models:
                m.fit(Fn[idx], (ly - mu_y) / sd_y, epochs=epochs)
                preds.append(m.predict(Fn))
            pick = []
            for b in range(batch):
                for i in np.argsort(-preds[b % ensemble]):
                    if int(i) not in measured and int(i) not in pick:
                        pick.append(int(i))
                        break
        for i in pick:
            if tr.spent >= budget:
                break
            r = evaluate(cands[i])
            measured[i] = r["mu"]
            tr.record(sp.key(cands[i]), r["mu"], r["cost"])
    return tr
