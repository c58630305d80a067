"""Component-wise attribution of a tuned variant (artificial crossover).

After the paper's analysis of its genome parts ("Contributions of The Three
Genome Parts"): take an initial individual I and the best individual B,
move one part of B's genome into I (or take one part of I into B) and
score the result, so that each part's own contribution and their synergy
can be read off.  The paper's parts are the kernel execution configuration
(C), the Manifest/Delayed choices (M) and the synchronisation points (S).
Here C is the tile and the waves-per-EU hint (the workgroup size follows
from them) and M is the staging family, RK-stage fusion and the LDS
kernels' Manifest choice; S has no counterpart (barriers follow from LDS
correctness).  Scores come from benchmark databases, so the analysis runs
anywhere; a crossover that no database holds is reported as missing.
"""
from __future__ import annotations

import math

from . import space as sp

PARTS = {"C": ("tile", "waves_per_eu"), "M": ("lds", "fuse", "manifest")}


def initial_individual(ndim: int) -> dict:
    """The paper's starting point: as few stored intermediates as possible
    (every cell recomputes its faces from global memory, one launch per
    stage), with a plain square tile."""
    tile = (32, 32) if ndim == 2 else (32, 8, 8)
    return sp.make_variant(tile[:ndim], 0, 0, 0, ndim)


def cross(base: dict, donor: dict, part: str, ndim: int) -> dict:
    """`base` with the genes of `part` taken from `donor`."""
    g = {"tile": base["tile"], "lds": base["lds"], "fuse": base["fuse"],
         "waves_per_eu": base["waves_per_eu"], "manifest": base.get("manifest", 0)}
    for name in PARTS[part]:
        g[name] = donor["tile"] if name == "tile" else donor.get(name, 0)
    # (the march forces 64 columns; its tiles are legal tiles of every other family)
    return sp.make_variant(list(g["tile"][:ndim]), g["lds"], g["fuse"], g["waves_per_eu"], ndim, g["manifest"])


def _score(dbs, variant: dict):
    k = sp.key(variant)
    for db in dbs:
        r = db.get(k)
        if r is not None:
            return r["mu"] if r.get("valid") and r.get("mu", 0) > 0 else 0.0
    return None


def attribution(dbs, ndim: int, initial: dict, best: dict | None = None) -> dict:
    """Scores of I, B and the four single-part crossovers, the relative
    changes, and how much of log(B/I) the sum of the two single-part log
    gains explains (1 = no synergy)."""
    if best is None:
        rows = [r for db in dbs for r in db.valid_rows()]
        best = max(rows, key=lambda r: r["mu"])["variant"]
    v = {"initial": initial, "best": best}
    for part in PARTS:
        v[f"initial+{part}"] = cross(initial, best, part, ndim)
        v[f"best-{part}"] = cross(best, initial, part, ndim)
    scores = {name: _score(dbs, var) for name, var in v.items()}
    out = {"keys": {name: sp.key(var) for name, var in v.items()}, "scores": scores}
    s_i, s_b = scores["initial"], scores["best"]
    if not s_i or not s_b:
        out["error"] = "initial or best individual not in the databases"
        return out
    gains = {}
    for part in PARTS:
        a, r = scores[f"initial+{part}"], scores[f"best-{part}"]
        out[f"add_{part}"] = None if a is None else a / s_i - 1.0
        out[f"remove_{part}"] = None if r is None else 1.0 - r / s_b
        gains[part] = None if not a else math.log(a / s_i)
    total = math.log(s_b / s_i)
    out["speedup"] = s_b / s_i
    if all(g is not None for g in gains.values()) and total > 0:
        out["log_additive_explained"] = sum(gains.values()) / total
    return out


def table(result: dict) -> str:
    """Markdown rows: individual, key, score (G cell-updates/s)."""
    lines = ["| individual | variant | G cell-updates/s |", "|---|---|---|"]
    for name, k in result["keys"].items():
        s = result["scores"][name]
        lines.append(f"| {name} | `{k}` | {'missing' if s is None else f'{s / 1e9:.2f}'} |")
    return "\n".join(lines)
