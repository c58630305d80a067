"""Benchmark harness: score one variant on one workload on the GPU.

Protocol (after the paper's tuner, "Parallel Asynchronous Genetic Simulated
Annealing"): the individual is benchmarked repeatedly and scored by the mean
and sample standard deviation of its speed in cell-updates per second; it is
then tested briefly and scores 0 if the state holds a NaN or has not
developed.  Here the brief test runs one step of a small mesh of the same
workload and also compares it with the library's default variant (itself
checked against the FP64 oracle by the test suite) to the FP32 tolerance.

Timing follows the regime the library runs in.  Applying a variant captures
its six step graphs; each repetition is one paraiso_advance of a
multiple of six device-dt steps, so that every step is a graph replay: at
least `steps_per_rep`, and enough whole periods for about `rep_ms` of device
time (a few milliseconds, so that launch gaps and timer resolution stay
negligible).  Before the repetitions the GPU clock is settled with untimed
steps (at least `settle_ms` of device time).  paraiso_advance starts with the
CFL reduction of its input and ends with a host synchronisation; that fixed
part is timed on its own (a zero-step advance, median of three) and taken
out of every repetition, so a repetition's time is that of its steps.
Repetitions stop at `max_reps`, or once `time_cap` seconds of timed work have
accumulated after at least `min_reps`.  Variants whose first step is more
than `screen_factor` times slower than the best so far are scored from
single-period repetitions (flagged "screened").
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from .. import binding as pb
from .. import inputs
from . import space


@dataclass
class Workload:
    name: str
    ndim: int
    n: int
    dtype: str
    gamma: float
    gate_n: int

    @property
    def esize(self) -> int:
        return 4 if self.dtype == "f32" else 8

    @property
    def cells(self) -> int:
        return self.n ** self.ndim

    def problem(self, n: int, z_range=None):
        if self.ndim == 3:
            return inputs.turbulent_box_3d(n, seed=4779, gamma=self.gamma, z_range=z_range)
        return inputs.kelvin_helmholtz_2d(n, seed=1204, gamma=self.gamma)


WORKLOADS = {
    "box512": Workload("box512", 3, 512, "f32", 5.0 / 3.0, 64),
    "box256": Workload("box256", 3, 256, "f32", 5.0 / 3.0, 64),
    "box128": Workload("box128", 3, 128, "f32", 5.0 / 3.0, 48),
    "kh2048": Workload("kh2048", 2, 2048, "f32", 1.4, 128),
    "kh2048_f64": Workload("kh2048_f64", 2, 2048, "f64", 1.4, 128),
}


def _state_err(got: np.ndarray, ref: np.ndarray, gamma: float) -> float:
    d = ref.shape[0] - 2
    rho = ref[0]
    m2 = sum(ref[1 + a] ** 2 for a in range(d))
    p = (gamma - 1.0) * (ref[d + 1] - 0.5 * m2 / rho)
    c = np.sqrt(gamma * np.maximum(p, 0.0) / rho)
    mscale = float(np.max(rho * (np.sqrt(m2) / rho + c)))
    worst = 0.0
    for q in range(ref.shape[0]):
        scale = mscale if 1 <= q <= d else float(np.max(np.abs(ref[q])))
        worst = max(worst, float(np.max(np.abs(got[q] - ref[q]))) / scale)
    return worst


class Bench:
    def __init__(self, wl: Workload, steps_per_rep: int = 6, max_reps: int = 30, min_reps: int = 3,
                 time_cap: float = 1.5, screen_factor: float = 20.0, settle_ms: float = 40.0, rep_ms: float = 3.0,
                 log=None):
        if steps_per_rep < 6 or steps_per_rep % 6:
            raise ValueError("steps_per_rep must be a positive multiple of 6 (one graph period)")
        import torch
        self.torch = torch
        self.wl = wl
        self.steps_per_rep, self.max_reps, self.min_reps = steps_per_rep, max_reps, min_reps
        self.time_cap, self.screen_factor, self.settle_ms = time_cap, screen_factor, settle_ms
        self.rep_ms = rep_ms
        self.log = log or (lambda s: None)
        d = wl.ndim
        spec = pb.MeshSpec(d, (wl.n,) * d, wl.gamma, (0,) * 3)
        self.solver = pb.Solver(spec, wl.dtype)
        self._upload_full()
        self.initial = None
        # gate mesh and its reference result from the default variant
        gp = wl.problem(wl.gate_n)
        self.gate_problem = gp
        self.gate = pb.Solver(pb.MeshSpec(d, (wl.gate_n,) * d, wl.gamma, (0,) * 3), wl.dtype)
        self.gate.upload(gp.U)
        self.gate_dt = self.gate.cfl_dt(0.5)[0]
        self.gate_in = self._gate_state()
        self.gate.step(self.gate_dt)
        self.gate_ref = self._gate_state()
        self.best_step_s = math.inf

    def _upload_full(self):
        torch = self.torch
        wl = self.wl
        buf = self.solver.state()
        if wl.ndim == 3:
            for z0 in range(0, wl.n, 32):
                z1 = min(wl.n, z0 + 32)
                sl = wl.problem(wl.n, z_range=(z0, z1))
                buf[:, z0:z1].copy_(torch.from_numpy(sl.U).to(buf.dtype))
        else:
            buf.copy_(torch.from_numpy(wl.problem(wl.n).U).to(buf.dtype))
        torch.cuda.synchronize()
        self.reset_state = buf.clone()

    def _gate_state(self):
        self.torch.cuda.synchronize()
        return self.gate.state().double().cpu().numpy()

    def _restore(self):
        cur = self.solver.state()
        cur.copy_(self.reset_state)
        self.torch.cuda.synchronize()

    def gate_check(self, variant: dict) -> tuple:
        """(ok, reason): one explicit step of the gate mesh with this variant."""
        g = self.gate
        g.upload(self.gate_in)
        g.set_variant(variant)
        g.step(self.gate_dt)
        out = self._gate_state()
        if not np.all(np.isfinite(out)):
            return False, "NaN"
        if float(np.max(np.abs(out - self.gate_in))) == 0.0:
            return False, "state did not develop"
        err = _state_err(out, self.gate_ref, self.wl.gamma)
        tol = 1e-5 if self.wl.dtype == "f32" else 1e-12
        if err > tol:
            return False, f"differs from the reference variant ({err:.2e})"
        return True, f"gate err {err:.1e}"

    def measure(self, variant: dict) -> dict:
        torch = self.torch
        t0 = time.perf_counter()
        v = dict(variant)
        try:
            self.solver.set_variant(v)
        except pb.ParaisoError as e:
            return {"valid": False, "mu": 0.0, "sigma": 0.0, "cost": time.perf_counter() - t0,
                    "reason": f"unsupported: {e}"}
        ok, why = self.gate_check(v)
        if not ok:
            return {"valid": False, "mu": 0.0, "sigma": 0.0, "cost": time.perf_counter() - t0, "reason": why}
        self._restore()
        s = self.solver
        stream = s.stream
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)

        def timed(steps: int) -> float:
            ev0.record(stream)
            s.advance(float("inf"), 0.5, max_steps=steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1) / 1e3

        # one graph period, also the screening probe
        first = timed(6) / 6
        screened = first > self.screen_factor * self.best_step_s
        spr = 6 if screened else max(self.steps_per_rep, 6 * max(1, round(self.rep_ms / 1e3 / (6 * first))))
        # clock settle: untimed periods until settle_ms of device time have passed
        settled = 6 * first
        while not screened and settled * 1e3 < self.settle_ms:
            settled += timed(6)
        fixed = sorted(timed(0) for _ in range(3))[1]
        scores = []
        timed_s = 0.0
        for _ in range(self.max_reps):
            dt = max(timed(spr) - fixed, 1e-9)
            timed_s += dt
            scores.append(self.wl.cells * spr / dt)
            if len(scores) >= self.min_reps and timed_s >= self.time_cap:
                break
            if screened and len(scores) >= self.min_reps:
                break
        self.best_step_s = min(self.best_step_s, timed_s / (len(scores) * spr))
        mu = float(np.mean(scores))
        sigma = float(np.std(scores, ddof=1)) if len(scores) > 1 else 0.0
        return {"valid": True, "mu": mu, "sigma": sigma, "reps": len(scores), "steps_per_rep": spr,
                "screened": bool(screened), "fixed_ms": fixed * 1e3, "cost": time.perf_counter() - t0,
                "reason": why}

    def close(self):
        self.solver.close()
        self.gate.close()
