"""Append-only database of benchmarked individuals (JSON lines).

Every individual keeps its genome, variant, score mean and sample standard
deviation, benchmark cost, validity and, for evolved individuals, parents
and method of birth.  Nothing is overwritten: the paper's tuner keeps all
past individuals accessible in its database (section on parallel
asynchronous genetic simulated annealing).  Re-opening a file resumes.
"""
from __future__ import annotations

import json
import os
import time


class DB:
    def __init__(self, path: str | None = None):
        self.path = path
        self.rows = []
        self.by_key = {}
        if path and os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if not line:
                        continue
                    r = json.loads(line)
                    self._index(r)

    def _index(self, r: dict):
        r["variant"]["tile"] = tuple(r["variant"]["tile"])
        self.rows.append(r)
        self.by_key[r["key"]] = r

    def __contains__(self, k: str) -> bool:
        return k in self.by_key

    def get(self, k: str):
        return self.by_key.get(k)

    def add(self, row: dict) -> dict:
        row = dict(row)
        row.setdefault("id", len(self.rows))
        row.setdefault("time", time.time())
        if self.path:
            with open(self.path, "a") as f:
                f.write(json.dumps(row) + "\n")
                f.flush()
                os.fsync(f.fileno())
        self._index(row)
        return row

    def valid_rows(self):
        return [r for r in self.rows if r.get("valid") and r.get("mu", 0) > 0]

    def best(self):
        v = self.valid_rows()
        return max(v, key=lambda r: r["mu"]) if v else None

    def total_cost(self) -> float:
        return float(sum(r.get("cost", 0.0) for r in self.rows))
