"""Family-tree analyses of tuning databases (tuner/lineage.py): hand-built
trees for the contribution distance and the ranks, scipy for the
chi-squared statistic, synthetic word bags for the Markov tests."""
import numpy as np
import pytest

from paper_1204_4779_amd.tuner import lineage as ln
from paper_1204_4779_amd.tuner.db import DB


def _fam(spec):
    """spec: list of (name, mu, sigma, birth, parents)."""
    db = DB(None)
    for i, (g, mu, sig, birth, par) in enumerate(spec):
        db.add({"key": g, "genome": g, "variant": {"tile": (8, 8, 1)}, "valid": True, "mu": mu, "sigma": sig,
                "birth": birth, "parents": par, "cost": 0.0, "id": i})
    return ln.family([db])


TREE = [
    ("A", 10.0, 0.5, "seed", []),
    ("B", 12.0, 0.5, "seed", []),
    ("Z", 1.0, 0.5, "seed", []),
    ("C", 20.0, 0.5, "crossover", ["A", "B"]),
    ("D", 30.0, 1.0, "mutation", ["C"]),             # the best individual
    ("E", 5.0, 0.5, "mutation", ["A"]),
    ("F", 4.0, 0.5, "mutation", ["E"]),
    ("G", 29.5, 0.5, "triangulation", ["E", "F", "B"]),  # within sigma_top of the best
    ("H", 3.0, 0.5, "crossover", ["F", "E"]),
    ("I", 2.0, 0.5, "mutation", ["H"]),
    ("J", 0.5, 0.5, "mutation", ["Z"]),
]


def test_contribution_distance_by_hand():
    d = ln.contribution_distance(_fam(TREE))
    assert {g for g, v in d.items() if v == 0} == {"A", "B", "C", "D", "E", "F", "G"}
    assert d["H"] == 1 and d["I"] == 2
    assert d["Z"] is None and d["J"] is None      # no line to a champion, no parents


def test_ranks_by_hand():
    fam = _fam(TREE)
    assert ln.rank(fam, "C") == "A"     # far above both parents
    assert ln.rank(fam, "E") == "D"     # far below its only parent
    assert ln.rank(fam, "H") == "D"
    assert ln.rank(fam, "A") is None
    fam2 = _fam([("P", 10.0, 1.0, "seed", []), ("Q", 4.0, 1.0, "seed", []),
                 ("R", 10.5, 1.0, "crossover", ["P", "Q"]),     # level with its best parent
                 ("S", 7.0, 1.0, "crossover", ["P", "Q"])])     # between its parents
    assert ln.rank(fam2, "R") == "B" and ln.rank(fam2, "S") == "C"


def test_chi2_matches_scipy():
    from scipy.stats import chi2_contingency
    rng = np.random.default_rng(3)
    for _ in range(20):
        pop = list(range(int(rng.integers(20, 200))))
        a = {x: rng.random() < 0.4 for x in pop}
        b = {x: (rng.random() < 0.3) or (a[x] and rng.random() < 0.5) for x in pop}
        r = ln.chi2_2x2(pop, a.get, b.get)
        t = np.array(r["table"])
        if (t.sum(0) == 0).any() or (t.sum(1) == 0).any():
            continue
        want = chi2_contingency(t, correction=False)[0]
        assert r["x2"] == pytest.approx(want, rel=1e-12)
    r = ln.chi2_2x2(range(100), lambda x: x < 50, lambda x: x < 50)
    assert r["sign"] == 1 and r["significant"] and r["x2"] == pytest.approx(100.0)


def test_words_along_family_lines():
    fam = _fam(TREE)
    d = ln.contribution_distance(fam)
    w2 = sorted(ln.words(fam, d, 2))
    # D <- C (mutation after crossover), G <- E, F (triangulation after mutations),
    # F <- E, E <- A(seed: no letter), C <- A, B (seeds)
    assert w2 == sorted([(2, 1), (1, 3), (1, 3), (1, 1)])


def _markov_words(P, n, rng, length):
    out = []
    for _ in range(n):
        w = [int(rng.integers(1, 4))]
        for _ in range(length - 1):
            w.append(int(rng.choice([1, 2, 3], p=P[w[-1] - 1])))
        out.append(tuple(w))
    return out


def test_markov_tests_recognise_the_order_of_a_chain():
    rng = np.random.default_rng(11)
    iid = [[1 / 3] * 3] * 3
    chain = [[0.8, 0.1, 0.1], [0.1, 0.8, 0.1], [0.1, 0.1, 0.8]]
    r = ln.markov_x2(_markov_words(iid, 3000, rng, 2), _markov_words(iid, 3000, rng, 3))
    assert r["order0"]["p"] > 1e-3 and r["order1"]["p"] > 1e-3
    r = ln.markov_x2(_markov_words(chain, 3000, rng, 2), _markov_words(chain, 3000, rng, 3))
    assert r["order0"]["p"] < 1e-3 and r["order1"]["p"] > 1e-3     # first order, not zeroth
    assert r["order0"]["repeats"]["3->3"] > 0
    assert r["order0"]["dof"] == 4 and r["order1"]["dof"] == 12


def test_asynchronous_service_over_a_shared_database(tmp_path):
    # three worker processes answer from the measured KH database, sleeping a
    # scaled copy of each benchmark's cost so that they interleave
    import os
    from paper_1204_4779_amd.tuner import service
    from paper_1204_4779_amd.tuner import space as sp
    measured = os.path.join(os.path.dirname(ln.__file__), "data", "kh2048_f32.jsonl")
    out = str(tmp_path / "svc.jsonl")
    res = service.run_service(out, 3, 2, 4, ("replay", measured, 0.05), budget=0.6, seed=5)
    assert len(res) == 3 and all(r["evaluated"] > 0 for r in res)
    rows = [r for r in service.SharedDB(out).snapshot()]
    results = [r for r in rows if "mu" in r]
    claims = [r for r in rows if "claim" in r]
    keys = [r["key"] for r in results]
    assert len(keys) == len(set(keys))                       # no individual benchmarked twice
    assert sorted(r["id"] for r in results) == list(range(len(results)))
    assert {r["key"] for r in claims} == set(keys)           # every result was claimed first
    assert len({r["worker"] for r in results}) == 3          # all workers contributed
    pos = {r["genome"]: r["id"] for r in results}
    for r in results:
        assert r["birth"] in ("seed", "random", "mutation", "crossover", "triangulation")
        assert len(r["parents"]) == {"seed": 0, "random": 0, "mutation": 1, "crossover": 2,
                                     "triangulation": 3}[r["birth"]]
        for p in r["parents"]:
            assert pos[p] < r["id"]                          # parents were measured before the child
        assert sp.key(sp.decode(r["genome"], 2)) == r["key"]
    assert any(r["birth"] in ("crossover", "triangulation") for r in results)
    from paper_1204_4779_amd.tuner.db import DB
    rep = ln.report([DB(out)])
    assert rep["individuals"] == len(results) and rep["d0"] >= 1
