"""Parallel asynchronous genetic simulated annealing as a multi-worker service.

After the paper's tuner ("Parallel Asynchronous Genetic Simulated
Annealing"): workers share one database and never wait for a generation.
Each worker repeatedly reads the database as it stands, makes one child
(the first `init` individuals are random, then PAGSA births), claims it,
benchmarks it and appends the result with its parents and method of birth.

The database is a JSON-lines file shared through POSIX advisory locks:
appends and claims take an exclusive lock on `<db>.lock`, reads a shared
one, so a reader never sees half a line.  A claim row (no "mu") marks an
individual being benchmarked; other workers treat it as taken.  Result rows
get consecutive ids in the order they are appended.

Workers are processes.  Live workers (one GPU) benchmark under an exclusive
lock on `<db>.gpu`, so timings never overlap while births, claims, gate
checks and database work of the other workers proceed; replay workers look
scores up in a measured database and may sleep for a scaled copy of the
benchmark cost to emulate asynchrony.
"""
from __future__ import annotations

import fcntl
import json
import os
import time
from contextlib import contextmanager

import numpy as np

from . import search
from . import space as sp


@contextmanager
def _flock(path: str, mode: int):
    with open(path, "a+") as f:
        fcntl.flock(f.fileno(), mode)
        try:
            yield
        finally:
            fcntl.flock(f.fileno(), fcntl.LOCK_UN)


class SharedDB:
    def __init__(self, path: str):
        self.path = path
        self.lock = path + ".lock"
        if not os.path.exists(path):
            open(path, "a").close()

    def _read(self) -> list:
        rows = []
        with open(self.path) as f:
            for line in f:
                line = line.strip()
                if line:
                    rows.append(json.loads(line))
        return rows

    def _append(self, row: dict):
        with open(self.path, "a") as f:
            f.write(json.dumps(row) + "\n")
            f.flush()
            os.fsync(f.fileno())

    def snapshot(self) -> list:
        with _flock(self.lock, fcntl.LOCK_SH):
            return self._read()

    def claim(self, variant: dict, genome: str, worker: int) -> bool:
        """Mark `variant` as being benchmarked by `worker`; False if it is
        already measured or claimed."""
        k = sp.key(variant)
        with _flock(self.lock, fcntl.LOCK_EX):
            if any(r.get("key") == k for r in self._read()):
                return False
            self._append({"key": k, "genome": genome, "variant": variant, "claim": worker, "time": time.time()})
            return True

    def add(self, row: dict) -> dict:
        with _flock(self.lock, fcntl.LOCK_EX):
            row = dict(row, id=sum(1 for r in self._read() if "mu" in r), time=time.time())
            self._append(row)
            return row


def _state(rows):
    known, taken = {}, set()
    for r in rows:
        g = r.get("genome")
        if g is None:
            continue
        if "mu" in r:
            known[g] = (r["mu"] if r.get("valid") else 0.0, r.get("sigma", 0.0) if r.get("valid") else 0.0)
        else:
            taken.add(g)
    return known, taken - set(known)


def worker_loop(db_path: str, worker: int, ndim: int, esize: int, evaluate, budget: float, seed: int,
                init: int = 8, log=None) -> dict:
    """Births, claims and benchmarks until this worker has spent `budget`
    seconds of benchmark time (or the space is exhausted)."""
    db = SharedDB(db_path)
    rng = np.random.default_rng(seed)
    cands = search.candidates(ndim, esize)
    valid_keys = {sp.key(v) for v in cands}
    spent, done = 0.0, 0
    log = log or (lambda s: None)
    while spent < budget:
        known, taken = _state(db.snapshot())
        parents, birth = [], "seed"
        child = None
        if len(known) + len(taken) >= init and known and max(m for m, _ in known.values()) > 0:
            child = search.pagsa_birth(known, rng, taken)
            if child is not None:
                g, parents, birth = child
        if child is None:
            unseen = [v for v in cands if sp.encode(v, ndim) not in known and sp.encode(v, ndim) not in taken]
            if not unseen:
                break
            g = sp.encode(unseen[int(rng.integers(0, len(unseen)))], ndim)
            birth = "seed" if len(known) + len(taken) < init else "random"
            parents = []
        v = sp.decode(g, ndim)
        if not db.claim(v, g, worker):
            continue   # another worker got there first
        if sp.key(v) in valid_keys:
            res = evaluate(v)
        else:
            res = {"valid": False, "mu": 0.0, "sigma": 0.0, "cost": 0.0, "reason": "statically invalid"}
        row = db.add({"key": sp.key(v), "genome": g, "variant": v, "parents": parents, "birth": birth,
                      "worker": worker, **res})
        spent += res["cost"]
        done += 1
        log(f"worker {worker}: #{row['id']} {row['key']} {birth} mu={res['mu'] / 1e9:.3f} G")
    return {"worker": worker, "evaluated": done, "spent": spent}


# ---- evaluators (built inside each worker process) ------------------------------------------

class ReplayEval:
    def __init__(self, db_path: str, time_scale: float = 0.0):
        from .db import DB
        self.ev = search.ReplayEvaluator(DB(db_path))
        self.time_scale = time_scale

    def __call__(self, v):
        r = self.ev(v)
        if self.time_scale > 0:
            time.sleep(r["cost"] * self.time_scale)
        return {k: r[k] for k in ("valid", "mu", "sigma", "cost")}


class LiveEval:
    def __init__(self, workload: str, gpu_lock: str):
        from . import measure
        self.bench = measure.Bench(measure.WORKLOADS[workload])
        self.gpu_lock = gpu_lock

    def __call__(self, v):
        with _flock(self.gpu_lock, fcntl.LOCK_EX):
            return self.bench.measure(v)


def _worker_main(args):
    db_path, worker, ndim, esize, spec, budget, seed, init = args
    if spec[0] == "replay":
        ev = ReplayEval(spec[1], spec[2])
    else:
        ev = LiveEval(spec[1], db_path + ".gpu")
    log = (lambda s: print(s, flush=True)) if spec[0] == "live" else None
    return worker_loop(db_path, worker, ndim, esize, ev, budget, seed, init, log)


def run_service(db_path: str, workers: int, ndim: int, esize: int, spec: tuple, budget: float, seed: int = 0,
                init: int = 8) -> list:
    """Start `workers` processes on one shared database and wait for them.
    spec: ("replay", measured_db_path, time_scale) or ("live", workload_name)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    jobs = [(db_path, w, ndim, esize, spec, budget, seed * 1000 + w, init) for w in range(workers)]
    with ctx.Pool(workers) as pool:
        return pool.map(_worker_main, jobs)
