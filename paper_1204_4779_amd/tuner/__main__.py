"""Tuner command line.

    python -m paper_1204_4779_amd.tuner measure --workload box512 --db DB.jsonl
        benchmark every statically valid variant on the GPU (resumes a partial DB)
    python -m paper_1204_4779_amd.tuner gain --db DB.jsonl [--seeds 15] [--frac 0.1]
        replay the database: MLP-guided vs random vs PAGSA search at the same budget
    python -m paper_1204_4779_amd.tuner attribution --db DB.jsonl [--db MORE.jsonl]
        component-wise artificial crossover between an initial individual and the
        best one: what the launch configuration (C) and the storage choices (M) add
    python -m paper_1204_4779_amd.tuner service --workload kh2048 --db OUT.jsonl --workers 3 --budget 20
        asynchronous PAGSA: worker processes over one shared database (live on the
        GPU, benchmarks serialised by a device lock; or --replay DB.jsonl)
    python -m paper_1204_4779_amd.tuner lineage --db OUT.jsonl
        family-tree analyses: contribution distance, ranks, chi-squared and Markov tests
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import analysis, lineage, measure, search, service
from . import space as sp
from .db import DB


def log(msg: str):
    print(msg, flush=True)


def cmd_measure(a):
    wl = measure.WORKLOADS[a.workload]
    db = DB(a.db)
    cands = search.candidates(wl.ndim, wl.esize, a.manifest)
    log(f"{wl.name}: {len(sp.enumerate_space(wl.ndim, a.manifest))} raw variants, {len(cands)} statically valid, "
        f"{sum(1 for v in cands if sp.key(v) in db)} already in the database")
    bench = measure.Bench(wl, log=log)
    ev = search.LiveEvaluator(bench, db, wl.ndim, log=log)
    # fast families first so the screening threshold is set early
    order = sorted(cands, key=lambda v: (-v["lds"], v["fuse"] and not v["lds"]))
    for v in order:
        ev(v)
    best = db.best()
    log(f"best: {best['key']} {best['mu'] / 1e9:.3f} Gcups; total benchmark cost {db.total_cost():.1f} s")
    bench.close()


def gain_study(db: DB, ndim: int, esize: int, seeds: int = 15, frac: float = 0.1, log=log) -> dict:
    cands = search.candidates(ndim, esize)
    ev = search.ReplayEvaluator(db)
    truth = search.exhaustive(cands, ev)
    budget = frac * truth.spent
    out = {"optimum_key": truth.best_key, "optimum_mu": truth.best_mu, "exhaustive_cost": truth.spent,
           "budget": budget, "runs": {}}
    for name in ("mlp", "random", "pagsa"):
        res = []
        for s in range(seeds):
            rng = np.random.default_rng(1000 + s)
            if name == "mlp":
                tr = search.mlp_guided(cands, ev, budget, rng, ndim, esize, model_seed=s)
            elif name == "random":
                tr = search.random_search(cands, ev, budget, rng)
            else:
                seedv = [cands[int(i)] for i in rng.permutation(len(cands))[:8]]
                tr = search.pagsa(cands, ev, budget, rng, ndim, seedv)
            res.append({"seed": s, "best_frac": tr.best_mu / truth.best_mu, "best_key": tr.best_key,
                        "anytime": tr.anytime(truth.best_mu, budget), "spent": tr.spent,
                        "evaluated": len(tr.evaluated)})
            log(f"{name} seed {s}: best {tr.best_mu / truth.best_mu:.4f} of optimum, anytime "
                f"{res[-1]['anytime']:.4f}, after {len(tr.evaluated)} benchmarks, {tr.spent:.1f} s")
        out["runs"][name] = res
        best = [r["best_frac"] for r in res]
        out[f"{name}_median"] = float(np.median(best))
        out[f"{name}_mean"] = float(np.mean(best))
        out[f"{name}_min"] = float(np.min(best))
        out[f"{name}_hits"] = int(sum(1 for b in best if b >= 1.0 - 1e-12))   # seeds that found the optimum
        out[f"{name}_anytime_median"] = float(np.median([r["anytime"] for r in res]))
    return out


def cmd_gain(a):
    db = DB(a.db)
    wl = measure.WORKLOADS[a.workload]
    out = gain_study(db, wl.ndim, wl.esize, a.seeds, a.frac)
    log(json.dumps({k: v for k, v in out.items() if k != "runs"}))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="paper_1204_4779_amd.tuner")
    sub = ap.add_subparsers(dest="cmd", required=True)
    m = sub.add_parser("measure")
    m.add_argument("--workload", default="box512", choices=sorted(measure.WORKLOADS))
    m.add_argument("--db", required=True)
    m.add_argument("--manifest", action="store_true", help="include the LDS kernels' Manifest choices")
    g = sub.add_parser("gain")
    g.add_argument("--workload", default="box512", choices=sorted(measure.WORKLOADS))
    g.add_argument("--db", required=True)
    g.add_argument("--seeds", type=int, default=15)
    g.add_argument("--frac", type=float, default=0.1)
    g.add_argument("--out", default=None)
    sv = sub.add_parser("service")
    sv.add_argument("--workload", default="kh2048", choices=sorted(measure.WORKLOADS))
    sv.add_argument("--db", required=True)
    sv.add_argument("--workers", type=int, default=3)
    sv.add_argument("--budget", type=float, default=20.0, help="benchmark seconds per worker")
    sv.add_argument("--seed", type=int, default=0)
    sv.add_argument("--replay", default=None, help="measured database to answer from instead of the GPU")
    sv.add_argument("--time-scale", type=float, default=0.0)
    ln = sub.add_parser("lineage")
    ln.add_argument("--db", action="append", required=True)
    t = sub.add_parser("attribution")
    t.add_argument("--workload", default="kh2048", choices=sorted(measure.WORKLOADS))
    t.add_argument("--db", action="append", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "measure":
        cmd_measure(a)
    elif a.cmd == "gain":
        cmd_gain(a)
    elif a.cmd == "service":
        wl = measure.WORKLOADS[a.workload]
        spec = ("replay", a.replay, a.time_scale) if a.replay else ("live", a.workload)
        t0 = time.time()
        res = service.run_service(a.db, a.workers, wl.ndim, wl.esize, spec, a.budget, a.seed)
        log(json.dumps({"workers": res, "wall_s": time.time() - t0}))
    elif a.cmd == "lineage":
        log(json.dumps(lineage.report([DB(p) for p in a.db]), indent=1))
    else:
        wl = measure.WORKLOADS[a.workload]
        dbs = [DB(p) for p in a.db]
        log(json.dumps(analysis.attribution(dbs, wl.ndim, analysis.initial_individual(wl.ndim)), indent=1))


if __name__ == "__main__":
    sys.exit(main())
