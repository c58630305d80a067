"""Tuner logic without a GPU: genome codec, the paper's birth operators and draw rule,
budgets, database resume and failure handling (a broken variant scores 0)."""
import json
import math

import numpy as np
import pytest

from paper_1204_4779_amd.tuner import search
from paper_1204_4779_amd.tuner import space as sp
from paper_1204_4779_amd.tuner.db import DB


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_genome_round_trip(ndim):
    seen = set()
    for v in sp.enumerate_space(ndim):
        g = sp.encode(v, ndim)
        assert len(g) == sp.genome_bits(ndim)
        assert sp.decode(g, ndim) == v
        seen.add(g)
    assert len(seen) == 4 ** ndim * 16 + {1: 0, 2: 32, 3: 128}[ndim]


def test_triangulation_table():
    # Base / Secondary / Primary -> Child, the paper's binary operation table
    table = {("0", "0", "0"): "0", ("0", "0", "1"): "1", ("0", "1", "0"): "1", ("0", "1", "1"): "1",
             ("1", "0", "0"): "0", ("1", "0", "1"): "0", ("1", "1", "0"): "0", ("1", "1", "1"): "1"}
    for (b, s, p), c in table.items():
        assert search.triangulate(b, s, p) == c
    assert search.triangulate("0011", "0101", "1001") == "1101"


def test_draw_weights_temperature():
    mus = np.array([10.0, 9.0, 5.0, 1.0])
    sig = np.array([0.1, 0.1, 0.1, 0.1])
    cold = search.draw_weights(mus, sig, 1e-3)
    hot = search.draw_weights(mus, sig, 1e6)
    assert cold[0] > 0.99                      # low temperature: the best individual
    assert np.all(np.abs(hot - 0.25) < 1e-3)   # high temperature: score hardly matters
    # differences small against the deviations are ignored
    even = search.draw_weights(np.array([10.0, 9.99]), np.array([1.0, 1.0]), 1e-3)
    assert abs(even[0] - even[1]) < 0.01
    assert np.all(np.diff(search.draw_weights(mus, sig, 2.0)) <= 0)


def test_temperature_range():
    rng = np.random.default_rng(0)
    mus, sig = np.array([100.0, 50.0]), np.array([2.0, 1.0])
    Ts = [search.draw_temperature(mus, sig, rng) for _ in range(2000)]
    assert min(Ts) >= 2.0 - 1e-9 and max(Ts) <= 100.0 + 1e-9
    logs = np.log(Ts)
    # log-uniform: mean of log T at the midpoint
    assert abs(np.mean(logs) - 0.5 * (math.log(2.0) + math.log(100.0))) < 0.1


def test_mutation_and_crossover_change_or_mix():
    rng = np.random.default_rng(1)
    g = "0101010101"
    for _ in range(100):
        assert search.mutate(g, rng) != g
        c = search.crossover("0000000000", "1111111111", rng)
        assert len(c) == 10 and set(c) <= {"0", "1"}


def _synthetic_db(ndim=3, esize=4, seed=3, broken=None):
    """A fake measured database: speed a smooth function of the features plus noise."""
    rng = np.random.default_rng(seed)
    db = DB()
    for v in sp.enumerate_space(ndim):
        k = sp.key(v)
        ok = sp.statically_valid(v, ndim, esize)
        t = v["tile"]
        mu = 0.0
        if ok:
            mu = 1e9 * (1 + 3 * v["lds"]) * (1 + 0.5 * v["fuse"] * v["lds"]) / (1 + 4 * v["fuse"] * (1 - v["lds"]))
            mu *= math.exp(-0.3 * abs(math.log2(t[0]) - 4) - 0.2 * abs(math.log2(t[1]) - 3))
            mu *= 1 + 0.05 * rng.normal()
        valid = ok and k != broken
        db.add({"key": k, "genome": sp.encode(v, ndim), "variant": v, "valid": valid,
                "mu": mu if valid else 0.0, "sigma": 0.01 * mu, "cost": 1.0 + (5.0 if not v["lds"] else 0.0)})
    return db


def test_budget_and_determinism():
    db = _synthetic_db()
    cands = search.candidates(3, 4)
    ev = search.ReplayEvaluator(db)
    a = search.random_search(cands, ev, 60.0, np.random.default_rng(5))
    b = search.random_search(cands, ev, 60.0, np.random.default_rng(5))
    assert a.evaluated == b.evaluated
    assert a.spent - a.evaluated[-1][2] < 60.0
    p = search.pagsa(cands, ev, 60.0, np.random.default_rng(7), 3, cands[:8])
    keys = [k for k, _, _ in p.evaluated]
    assert len(keys) == len(set(keys))          # every child is a new genome
    assert p.spent - p.evaluated[-1][2] < 60.0


def test_pagsa_improves_on_its_seeds():
    db = _synthetic_db()
    cands = search.candidates(3, 4)
    ev = search.ReplayEvaluator(db)
    rng = np.random.default_rng(11)
    seeds = [cands[int(i)] for i in rng.permutation(len(cands))[:8]]
    tr = search.pagsa(cands, ev, 200.0, rng, 3, seeds)
    seed_best = max(ev(v)["mu"] for v in seeds)
    assert tr.best_mu >= seed_best
    births = {r for r in (k for k, _, _ in tr.evaluated)}
    assert len(births) > 8


def test_broken_variant_scores_zero_and_is_never_best():
    cands = search.candidates(3, 4)
    clean = _synthetic_db()
    best = search.exhaustive(cands, search.ReplayEvaluator(clean)).best_key
    db = _synthetic_db(broken=best)
    tr = search.exhaustive(cands, search.ReplayEvaluator(db))
    assert tr.best_key != best
    assert dict((k, mu) for k, mu, _ in tr.evaluated)[best] == 0.0


def test_db_resume_skips_measured(tmp_path):
    path = str(tmp_path / "db.jsonl")
    calls = []

    class FakeBench:
        def measure(self, v):
            calls.append(sp.key(v))
            return {"valid": True, "mu": 1e9, "sigma": 1e7, "cost": 0.5, "reason": "ok"}

    cands = search.candidates(2, 4)[:10]
    ev = search.LiveEvaluator(FakeBench(), DB(path), 2)
    for v in cands[:6]:
        ev(v)
    # a forced stop: reopen the database and continue
    ev2 = search.LiveEvaluator(FakeBench(), DB(path), 2)
    for v in cands:
        ev2(v)
    assert calls == [sp.key(v) for v in cands[:6]] + [sp.key(v) for v in cands[6:]]
    rows = [json.loads(l) for l in open(path)]
    assert len(rows) == 10 and len({r["key"] for r in rows}) == 10


def test_static_validity_examples():
    big = sp.make_variant((64, 64, 64), 1, 1, 0, 3)
    assert not sp.statically_valid(big, 3, 4)
    ok = sp.make_variant((16, 8, 8), 1, 0, 0, 3)
    assert sp.statically_valid(ok, 3, 4)
    assert sp.statically_valid(sp.make_variant((64, 64, 64), 0, 1, 5, 3), 3, 4)


class _NumpyCostModel:
    """The cost model with the oracle's FP64 MLP in place of the GPU kernels."""

    def __init__(self, in_dim, hidden=64, seed=0, lr=3e-3):
        from oracle import mlp as om
        self.om, self.in_dim, self.hidden, self.lr = om, in_dim, hidden, lr
        rng = np.random.default_rng(seed)
        self.p = rng.normal(scale=0.3, size=om.n_params(in_dim, hidden))
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0

    def fit(self, X, y, epochs=200):
        for _ in range(epochs):
            _, g = self.om.loss_grad(X, y, self.p, self.in_dim, self.hidden)
            self.t += 1
            self.p, self.m, self.v = self.om.adam(self.p, g, self.m, self.v, self.lr, 0.9, 0.999, 1e-8, self.t)

    def predict(self, X):
        return self.om.forward(X, self.p, self.in_dim, self.hidden)[0]


def test_mlp_guided_ensemble_loop(monkeypatch):
    from paper_1204_4779_amd.tuner import model
    monkeypatch.setattr(model, "CostModel", _NumpyCostModel)
    db = _synthetic_db()
    cands = search.candidates(3, 4)
    ev = search.ReplayEvaluator(db)
    truth = search.exhaustive(cands, ev)
    budget = 0.1 * truth.spent
    tr = search.mlp_guided(cands, ev, budget, np.random.default_rng(4), 3, 4, epochs=60, ensemble=4, batch=4)
    keys = [k for k, _, _ in tr.evaluated]
    assert len(keys) == len(set(keys))                   # nothing benchmarked twice
    assert tr.spent - tr.evaluated[-1][2] < budget       # stops once the budget is spent
    assert tr.best_mu >= 0.9 * truth.best_mu             # the smooth synthetic optimum is found


# ---- component attribution (artificial crossover) -----------------------------------

def _product_db(ndim, c_of, m_of):
    """A database whose score is a product of a launch-configuration factor and a
    storage-choice factor: no synergy by construction."""
    db = DB(None)
    for v in search.candidates(ndim, 4, manifest=True):
        mu = 1e9 * c_of(v) * m_of(v)
        db.add({"key": sp.key(v), "variant": v, "valid": True, "mu": mu, "sigma": 0.0, "cost": 0.01})
    return db


def test_attribution_separates_independent_parts():
    from paper_1204_4779_amd.tuner import analysis
    c_of = lambda v: 1.0 + 0.01 * v["tile"][1] + 0.1 * (v["waves_per_eu"] == 3)
    m_of = lambda v: {0: 1.0, 1: 2.0, 2: 4.0}[v["lds"]] * (1.5 if v["fuse"] else 1.0) * (0.5 if v.get("manifest") else 1.0)
    db = _product_db(2, c_of, m_of)
    init = analysis.initial_individual(2)
    res = analysis.attribution([db], 2, init)
    best = db.best()["variant"]
    assert res["keys"]["best"] == sp.key(best)
    # two parts: moving C into the initial individual is removing M from the best
    assert res["keys"]["initial+C"] == res["keys"]["best-M"]
    assert res["keys"]["initial+M"] == res["keys"]["best-C"]
    assert res["add_M"] == pytest.approx(m_of(best) / m_of(init) - 1.0)
    # multiplicative parts: the single-part log gains add up to the whole
    assert res["log_additive_explained"] == pytest.approx(1.0)
    assert res["speedup"] == pytest.approx(c_of(best) * m_of(best) / (c_of(init) * m_of(init)))


def test_attribution_detects_synergy_and_missing_rows():
    from paper_1204_4779_amd.tuner import analysis
    # the launch configuration only matters once the storage choice is right
    db = DB(None)
    for v in search.candidates(2, 4):
        mu = 1e9 * (3.0 * (1 + 0.02 * v["tile"][1]) if v["lds"] == 2 else 1.0)
        db.add({"key": sp.key(v), "variant": v, "valid": True, "mu": mu, "sigma": 0.0, "cost": 0.01})
    res = analysis.attribution([db], 2, analysis.initial_individual(2))
    assert res["add_C"] == pytest.approx(0.0)
    assert res["log_additive_explained"] < 1.0
    # a crossover nobody measured is reported, not guessed
    empty = DB(None)
    for k in ("initial", "best"):
        v = analysis.initial_individual(2) if k == "initial" else db.best()["variant"]
        empty.add({"key": sp.key(v), "variant": v, "valid": True, "mu": 1e9 if k == "initial" else 2e9,
                   "sigma": 0.0, "cost": 0.01})
    res = analysis.attribution([empty], 2, analysis.initial_individual(2))
    assert res["scores"]["initial+C"] is None and res["add_C"] is None
    assert "log_additive_explained" not in res


def test_manifest_axis_keys_and_lds_budget():
    base = sp.make_variant((32, 16), 1, 0, 0, 2)
    kept = sp.make_variant((32, 16), 1, 0, 0, 2, manifest=2)
    assert sp.key(kept) == sp.key(base) + "_m2" and "manifest" not in base
    assert sp.lds_bytes(kept, 2, 4) - sp.lds_bytes(base, 2, 4) == 4 * 4 * 2 * (36 * 20)
    assert sp.make_variant((64, 16), 2, 1, 0, 2, manifest=1).get("manifest") is None
    assert len(search.candidates(2, 4, manifest=True)) > len(search.candidates(2, 4))
