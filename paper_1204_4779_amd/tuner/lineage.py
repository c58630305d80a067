"""Family-tree analyses of a tuning database (section "Analysis on the
Automated Tuning Experiments").

Rows with a birth method and parents (mutation: 1 parent, crossover: 2,
triangulation: 3) form a family tree.  On it:

  contribution distance d(I): 0 for the best individuals (mu(I) > mu_top -
      sigma_top) and every ancestor of one; otherwise 1 + the smallest d of
      its parents (None for parentless individuals off the champions' trees);
  rank: A if significantly faster than every parent, D if significantly
      slower than every parent, B if within one combined deviation
      sigma(I, P) = (sigma(I)^2 + sigma(P)^2)^(1/2) of its fastest parent,
      C otherwise;
  Pearson's chi-squared test of independence of two predicates over a
      population (2 x 2 table, no continuity correction; 10.83 is the 1e-3
      point for one degree of freedom), signed by the direction of the
      correlation;
  Markov analysis of the birth methods along the champions' family lines:
      every way of tracing a d = 0 individual back n generations gives an
      n-letter word (oldest first, the individual's own method last); the
      bag of 2-letter words is tested against independence of consecutive
      letters (0th order, p(ab) = p(a) p(b)) and the bag of 3-letter words
      against a first-order chain (p(abc) = p(ab) p(bc) / p(b)).

Individuals are identified by their genome; parents are stored as genomes.
"""
from __future__ import annotations

import math
from collections import Counter, defaultdict

METHODS = {"mutation": 1, "crossover": 2, "triangulation": 3}
X2_1E3 = 10.83   # chi-squared, 1 degree of freedom, significance 1e-3


def _rows(dbs):
    rows = []
    for db in dbs:
        rows += [r for r in db.rows if "mu" in r and r.get("genome")]
    rows.sort(key=lambda r: r.get("id", 0))
    return rows


def family(dbs) -> dict:
    """genome -> record {mu, sigma, parents (genomes), birth, id}, first occurrence kept."""
    out = {}
    for r in _rows(dbs):
        g = r["genome"]
        if g in out:
            continue
        mu = r["mu"] if r.get("valid") else 0.0
        out[g] = {"mu": mu, "sigma": r.get("sigma", 0.0) if r.get("valid") else 0.0,
                  "parents": [p for p in (r.get("parents") or [])], "birth": r.get("birth"),
                  "id": r.get("id", len(out))}
    return out


def contribution_distance(fam: dict) -> dict:
    """d(I) for every genome (None where undefined)."""
    top = max(fam, key=lambda g: fam[g]["mu"])
    mt, st = fam[top]["mu"], fam[top]["sigma"]
    d = {g: None for g in fam}
    stack = [g for g in fam if g == top or fam[g]["mu"] > mt - st]
    while stack:   # the best individuals and all their ancestors
        g = stack.pop()
        if d[g] == 0:
            continue
        d[g] = 0
        stack += [p for p in fam[g]["parents"] if p in fam]
    for g in sorted(fam, key=lambda x: fam[x]["id"]):   # parents are older than children
        if d[g] == 0:
            continue
        ds = [d[p] for p in fam[g]["parents"] if p in fam and d[p] is not None]
        d[g] = 1 + min(ds) if ds else None
    return d


def rank(fam: dict, g: str):
    """'A', 'B', 'C', 'D' for an individual with parents, else None."""
    me = fam[g]
    par = [fam[p] for p in me["parents"] if p in fam]
    if not par:
        return None
    comb = lambda p: math.sqrt(me["sigma"] ** 2 + p["sigma"] ** 2)
    if all(me["mu"] < p["mu"] - comb(p) for p in par):
        return "D"
    if all(me["mu"] > p["mu"] + comb(p) for p in par):
        return "A"
    best = max(par, key=lambda p: p["mu"])
    if abs(me["mu"] - best["mu"]) < comb(best):
        return "B"
    return "C"


def chi2_2x2(population, pred_a, pred_b) -> dict:
    """Pearson's X^2 of independence of two predicates over `population`;
    sign +1 if they co-occur more often than independence predicts."""
    n = [[0, 0], [0, 0]]
    for x in population:
        n[1 if pred_a(x) else 0][1 if pred_b(x) else 0] += 1
    total = sum(map(sum, n))
    rows = [sum(n[i]) for i in range(2)]
    cols = [n[0][j] + n[1][j] for j in range(2)]
    x2 = 0.0
    for i in range(2):
        for j in range(2):
            e = rows[i] * cols[j] / total if total else 0.0
            if e > 0:
                x2 += (n[i][j] - e) ** 2 / e
    e11 = rows[1] * cols[1] / total if total else 0.0
    return {"x2": x2, "sign": 1 if n[1][1] > e11 else (-1 if n[1][1] < e11 else 0), "table": n,
            "significant": x2 > X2_1E3}


def words(fam: dict, d: dict, length: int) -> list:
    """Every birth-method word of `length` letters along the family lines of d = 0 individuals."""
    out = []

    def back(g, suffix):
        m = METHODS.get(fam[g]["birth"])
        if m is None:
            return
        w = [m] + suffix
        if len(w) == length:
            out.append(tuple(w))
            return
        for p in fam[g]["parents"]:
            if p in fam:
                back(p, w)

    for g in fam:
        if d.get(g) == 0:
            back(g, [])
    return out


def markov_x2(w2: list, w3: list, letters=(1, 2, 3)) -> dict:
    """X^2 of the 0th-order hypothesis on 2-letter words and of the
    1st-order hypothesis on 3-letter words, with degrees of freedom, p-values
    and the signed single-cell contributions of repeated letters."""
    from scipy.stats import chi2 as chi2dist
    letters = sorted(set(letters) | {a for w in w2 + w3 for a in w})
    K = len(letters)
    out = {}
    if w2:
        n = Counter(w2)
        first = Counter(w[0] for w in w2)
        second = Counter(w[1] for w in w2)
        tot = len(w2)
        x2 = 0.0
        cells = {}
        for a in letters:
            for b in letters:
                e = first[a] * second[b] / tot
                if e > 0:
                    c = (n[(a, b)] - e) ** 2 / e
                    x2 += c
                    if a == b:
                        cells[f"{a}->{a}"] = math.copysign(c, n[(a, b)] - e)
        dof = (K - 1) ** 2
        out["order0"] = {"x2": x2, "dof": dof, "p": float(chi2dist.sf(x2, dof)), "words": tot, "repeats": cells}
    if w3:
        n3 = Counter(w3)
        ab = Counter((w[0], w[1]) for w in w3)
        bc = Counter((w[1], w[2]) for w in w3)
        b_ = Counter(w[1] for w in w3)
        x2 = 0.0
        cells = {}
        for a in letters:
            for b in letters:
                for c in letters:
                    if b_[b] == 0:
                        continue
                    e = ab[(a, b)] * bc[(b, c)] / b_[b]
                    if e > 0:
                        contrib = (n3[(a, b, c)] - e) ** 2 / e
                        x2 += contrib
                        if a == b == c:
                            cells[f"{a}{a}->{a}"] = math.copysign(contrib, n3[(a, b, c)] - e)
        dof = K * (K - 1) ** 2
        out["order1"] = {"x2": x2, "dof": dof, "p": float(chi2dist.sf(x2, dof)), "words": len(w3), "repeats": cells}
    return out


def markov_tests(fam: dict, d: dict) -> dict:
    """markov_x2 on the words of the champions' family lines."""
    return markov_x2(words(fam, d, 2), words(fam, d, 3))


def report(dbs) -> dict:
    """The distance and rank distributions per birth method and the paper's
    predicate-pair tests."""
    fam = family(dbs)
    d = contribution_distance(fam)
    rk = {g: rank(fam, g) for g in fam}
    npar = {g: len([p for p in fam[g]["parents"] if p in fam]) for g in fam}
    born = [g for g in fam if npar[g] > 0]
    dist = defaultdict(Counter)
    ranks = defaultdict(Counter)
    for g in born:
        m = fam[g]["birth"]
        dist[m][d[g] if d[g] is not None else "none"] += 1
        ranks[m][rk[g]] += 1
    d0 = lambda g: d[g] == 0
    tests = {
        "mutation & d=0": chi2_2x2(born, lambda g: npar[g] == 1, d0),
        "crossover & d=0": chi2_2x2(born, lambda g: npar[g] == 2, d0),
        "triangulation & d=0": chi2_2x2(born, lambda g: npar[g] == 3, d0),
        "rank A & d=0": chi2_2x2(born, lambda g: rk[g] == "A", d0),
        "rank B & d=0": chi2_2x2(born, lambda g: rk[g] == "B", d0),
        "rank C & d=0": chi2_2x2(born, lambda g: rk[g] == "C", d0),
        "rank D & d=0": chi2_2x2(born, lambda g: rk[g] == "D", d0),
        "triangulation & d=0, within crossover or triangulation":
            chi2_2x2([g for g in born if npar[g] >= 2], lambda g: npar[g] == 3, d0),
        "rank A & crossover, within the elite":
            chi2_2x2([g for g in born if npar[g] >= 2 and rk[g] in ("A", "B")], lambda g: rk[g] == "A",
                     lambda g: npar[g] == 2),
        "id ends in 7 & d=0 (control)": chi2_2x2(born, lambda g: fam[g]["id"] % 10 == 7, d0),
        "id ends in 13 & d!=0 (control)": chi2_2x2(born, lambda g: fam[g]["id"] % 100 == 13, lambda g: not d0(g)),
    }
    top = max(fam, key=lambda g: fam[g]["mu"])
    return {"individuals": len(fam), "born": len(born), "best": top, "best_mu": fam[top]["mu"],
            "d0": sum(1 for g in fam if d[g] == 0),
            "distance_by_birth": {m: dict(c) for m, c in dist.items()},
            "rank_by_birth": {m: dict(c) for m, c in ranks.items()},
            "chi2": {k: {"x2": round(v["x2"], 3), "sign": v["sign"], "significant": v["significant"],
                         "table": v["table"]} for k, v in tests.items()},
            "markov": markov_tests(fam, d)}
