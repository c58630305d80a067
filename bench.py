#!/usr/bin/env python3
"""Benchmark: cell-updates per second of the Euler step on one MI355X.

Headline workload: 2D periodic Kelvin-Helmholtz, 2048 x 2048 cells, gamma = 1.4
(seeded 1% v_y perturbation), FP32, advanced with the device-resident CFL time
step (CFL 0.5) by paraiso_advance; one step = both Runge-Kutta stages plus the
CFL reduction of the new state.  Inputs are resident in HBM before timing.

Every run first settles the GPU clock (untimed steps until at least 60 ms of
device time have passed; reported as `clock_settle`), then takes the W warm-up
steps, then times exactly K steps with HIP events on the library's stream.

Prints one JSON line.  Besides the headline it reports (in `extra`) FP64 and
the untuned (per-cell, unfused, no LDS) variant of the headline workload and
the other configurations of the metric: Sod 1024 FP64 to t = 0.2 (time to
solution), the 3D periodic box at 256^3 and 512^3 (FP32, tuned and untuned),
and the batch of 512 uneven 2D meshes (FP32, tuned, the tuned kernel fed by
the persistent work queues, and untuned); the roofline
of the dominant kernel; and the FP64 CPU oracle timed on bounded samples on
the host, serially and on all host cores.

    python bench.py [--gpus 1] [--steps 500] [--warmup 500] [--no-cpu] [--no-extra] [--variant JSON]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 2048
CFL = 0.5
METRIC = "cell-updates/sec and % HBM roofline, FP32 vs FP64, tuned vs untuned"

# Floating-point operations of the method per cell-update (one step and the
# CFL term of its result), counted on a counting number type with every
# quantity formed once (oracle/method_flops.py; every face in the HLLC star
# branch, which is what the subsonic workloads take).  The oracle's own code
# recomputes on purpose (slopes twice per axis, conserved face states inside
# the physical flux, both sides' fluxes before the branch); its count, an
# upper bound, is reported beside.
FLOPS_PER_CELL_UPDATE = {1: 165.0, 2: 379.0, 3: 653.0}
FLOPS_ORACLE_CODE = {2: 730.6, 3: 1322.0}


# Algorithmic HBM bytes per cell-update: read U^n once, write U^{n+1} once.
def bytes_per_cell_update(ndim: int, esize: int) -> int:
    return 2 * (ndim + 2) * esize


HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, each scaled by the reading of a plain 512 MiB device copy
# (factors 2.000 and 1.000); valid only for the kernel sources they were taken
# on (hash of the device headers) and the variant named.
TRAFFIC = {"sources": "e39bf9b461bcc066",
           "variant": {"tile": [64, 20], "lds": 2, "fuse": 1, "waves_per_eu": 0, "threads": 256},
           "bytes_per_launch": 157.78e6}


def kernel_name(v: dict) -> str:
    """The dominant kernel of a 2D FP32 variant (one launch per fused step)."""
    w = v.get("waves_per_eu", 0)
    fused = "true" if v.get("fuse", 1) else "false"
    lds = v.get("lds", 1)
    if lds == 2:
        return f"k_march2d<float,{w},{fused}>"
    fam = {1: "fused_lds" if v.get("fuse", 1) else "stage_lds", 0: "fused_direct" if v.get("fuse", 1) else "stage_direct"}
    return f"k_{fam[lds]}<float,2,{w}>"


def _kernel_source_hash() -> str:
    """Hash of the device headers with comments and blank space removed, so
    that editing a comment does not invalidate the profiled figures."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1204_4779_amd", "csrc")
    digests = ""
    for f in ("euler_device.h", "euler_common.h", "euler_march2d.h"):
        with open(os.path.join(csrc, f)) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        code = " ".join(code.split())
        digests += hashlib.sha256(code.encode()).hexdigest() + "\n"
    return hashlib.sha256(digests.encode()).hexdigest()[:16]


# MI355X vector peaks: 256 CU x 2.4 GHz.  FP32 157.3 TFLOP/s is the published
# figure (packed FP32 or dual issue); this library compiles packed FP32 out,
# which leaves 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6.
ALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
ALU_PEAK_NONPACKED_TFLOPS = {"f32": 78.6, "f64": 78.6}
SETTLE_MS = 60.0

from paper_1204_4779_amd import variants  # noqa: E402

TUNED = {"f32": variants.tuned("kh2048", "f32"), "f64": variants.tuned("kh2048", "f64")}
UNTUNED = dict(variants.UNTUNED_2D)


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fractions(cups: float, ndim: int, dtype: str) -> dict:
    esz = 4 if dtype == "f32" else 8
    fl = FLOPS_PER_CELL_UPDATE[ndim] * cups / 1e12
    return {"hbm_frac": cups * bytes_per_cell_update(ndim, esz) / 1e9 / HBM_PEAK_GBS,
            "alu_frac": fl / ALU_PEAK_TFLOPS[dtype], "alu_frac_nonpacked": fl / ALU_PEAK_NONPACKED_TFLOPS[dtype]}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def settle(s, t, t_end=float("inf"), chunk: int = 60):
    """Untimed steps until SETTLE_MS of device time have passed (the GPU's clock ramps up
    under sustained load); returns (t, steps, ms)."""
    import torch
    steps, ms = 0, 0.0
    while ms < SETTLE_MS:
        a, b = _events()
        a.record(s.stream)
        t, _ = s.advance(t_end, CFL, max_steps=chunk, t0=t)
        b.record(s.stream)
        torch.cuda.synchronize()
        ms += a.elapsed_time(b)
        steps += chunk
    return t, steps, ms


def timed_advance(s, steps: int, warmup: int, t_end=float("inf")):
    """Clock settle, `warmup` untimed steps, then exactly `steps` timed steps (one
    paraiso_advance call between HIP events on the library's stream)."""
    import torch
    count = s.count
    t = [0.0] * count
    t, settle_steps, settle_ms = settle(s, t, t_end)
    if warmup:
        t, _ = s.advance(t_end, CFL, max_steps=warmup, t0=t)
    a, b = _events()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    a.record(s.stream)
    t, n = s.advance(t_end, CFL, max_steps=steps, t0=t)
    b.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    event_ms = a.elapsed_time(b)
    # the advance call's fixed part (the CFL reduction of its input, the control-block
    # set-up, the copies and the final synchronisation), timed on its own as a
    # zero-step advance (median of three): the step kernel's own time per launch is
    # the timed region less this
    fixed = []
    for _ in range(3):
        a, b = _events()
        a.record(s.stream)
        s.advance(t_end, CFL, max_steps=0, t0=t)
        b.record(s.stream)
        torch.cuda.synchronize()
        fixed.append(a.elapsed_time(b))
    return {"wall_s": wall, "event_ms": event_ms, "steps": n, "t": t, "advance_fixed_ms": sorted(fixed)[1],
            "clock_settle": {"steps": settle_steps, "ms": round(settle_ms, 3)}}


def audit(tot0, tot1) -> dict:
    """Conserved-total drift: mass and energy relative to themselves, momentum relative to
    the mass total (unit velocity scale)."""
    drift = {"mass": 0.0, "momentum": 0.0, "energy": 0.0}
    for a0, a1 in zip(tot0, tot1):
        nf = len(a0)
        drift["mass"] = max(drift["mass"], abs(a1[0] - a0[0]) / abs(a0[0]))
        drift["energy"] = max(drift["energy"], abs(a1[-1] - a0[-1]) / abs(a0[-1]))
        for q in range(1, nf - 1):
            drift["momentum"] = max(drift["momentum"], abs(a1[q] - a0[q]) / abs(a0[0]))
    return drift


def run_gpu(U, dtype: str, variant: dict, steps: int, warmup: int, specs=None, t_end=float("inf"), fill=None):
    """Advance `steps` device-dt steps after the clock settle and `warmup`; U is one state
    or a list (batch), or None with `fill(solver)` writing the state on the device."""
    import torch
    from paper_1204_4779_amd import binding as pb
    if specs is None:
        specs = [pb.MeshSpec(2, (N, N), 1.4, (0, 0))]
    s = pb.Solver(specs, dtype)
    s.set_variant(variant)
    if fill is not None:
        fill(s)
    else:
        s.upload(U)
    tot0 = s.totals()
    r = timed_advance(s, steps, warmup, t_end)
    r["mass_energy_drift"] = audit(tot0, s.totals())
    r["launches"] = steps * (1 if variant.get("fuse", 1) or variant.get("lds") == 3 else 2)
    s.close()
    del s
    torch.cuda.empty_cache()
    return r


def repetitions(U, dtype: str, variant: dict, reps: int = 10, steps_each: int = 48):
    """Mean and sample standard deviation of cell-updates/s over `reps` separately timed
    runs of `steps_each` device-dt steps (whole graph periods) after the clock settle."""
    import statistics
    import torch
    from paper_1204_4779_amd import binding as pb
    s = pb.Solver([pb.MeshSpec(2, (N, N), 1.4, (0, 0))], dtype)
    s.set_variant(variant)
    s.upload(U)
    t, _, _ = settle(s, [0.0])
    vals = []
    for _ in range(reps):
        a, b = _events()
        torch.cuda.synchronize()
        a.record(s.stream)
        t, _ = s.advance(float("inf"), CFL, max_steps=steps_each, t0=t)
        b.record(s.stream)
        torch.cuda.synchronize()
        vals.append(N * N * steps_each / (a.elapsed_time(b) / 1e3))
    s.close()
    return {"reps": reps, "steps_each": steps_each, "mean": statistics.mean(vals), "std": statistics.stdev(vals),
            "note": "each repetition is one paraiso_advance call (its initial CFL reduction and host sync "
                    "included), after the clock settle"}


# ---------------------------------------------------------------------------------------
# the other configurations of the metric
# ---------------------------------------------------------------------------------------

def box_fill(n: int, seed: int = 4779):
    """Write the seeded 3D box (lognormal density, Gaussian velocities, p = 1) into the
    solver's current buffer, generated on the device 32 planes at a time."""
    def fill(s):
        import torch
        from paper_1204_4779_amd import inputs
        st = s.state()
        for z in range(0, n, 32):
            z1 = min(n, z + 32)
            chunk = inputs.turbulent_box_3d_torch(n, seed, z_range=(z, z1), device=st.device)
            st[:, z:z1].copy_(chunk.to(st.dtype))
            del chunk
        torch.cuda.synchronize()
    return fill


def config_entry(r, cells: int, ndim: int, dtype: str, variant: dict) -> dict:
    k = r["steps"][0] if isinstance(r["steps"], list) else r["steps"]
    cups = cells * k / (r["event_ms"] / 1e3)
    out = {"value": cups, "ms_per_step": r["event_ms"] / k, "steps": k, "variant": variant,
           "clock_settle": r["clock_settle"]}
    out.update(fractions(cups, ndim, dtype))
    return out


def sod_entry(variant=None) -> dict:
    """Sod 1024 FP64, outflow, to t = 0.2: one paraiso_advance from t = 0 (time to solution)."""
    import torch
    from paper_1204_4779_amd import binding as pb
    from paper_1204_4779_amd import inputs
    pr = inputs.sod_1d(1024)
    spec = pb.MeshSpec(1, pr.n, pr.gamma, pr.bc)
    var = variant or variants.tuned("sod1024", "f64")
    s = pb.Solver([spec], "f64")
    s.set_variant(var)
    s.upload(pr.U)
    s.advance(0.2, CFL)                 # first run: clock and caches
    best = None
    for _ in range(5):
        s.upload(pr.U)
        a, b = _events()
        torch.cuda.synchronize()
        a.record(s.stream)
        t, k = s.advance(0.2, CFL, t0=[0.0])
        b.record(s.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    s.close()
    return {"value": 1024 * k[0] / (best / 1e3), "time_to_solution_ms": best, "steps": k[0], "t": t[0],
            "variant": var, "timing": "best of 5 runs from t = 0 after one untimed run"}


def box_entries(n: int, steps: int, warmup: int, untuned: bool = True) -> dict:
    from paper_1204_4779_amd import binding as pb
    spec = pb.MeshSpec(3, (n, n, n), 5.0 / 3.0, (0, 0, 0))
    out = {}
    name = "box256" if n == 256 else "box512"
    var = variants.tuned(name, "f32")
    r = run_gpu(None, "f32", var, steps, warmup, specs=[spec], fill=box_fill(n))
    out["f32_tuned"] = config_entry(r, n ** 3, 3, "f32", var)
    out["f32_tuned"]["audit_drift"] = r["mass_energy_drift"]
    if untuned:
        uv = dict(variants.UNTUNED_3D)
        r = run_gpu(None, "f32", uv, max(steps // 4, 6), min(warmup, 12), specs=[spec], fill=box_fill(n))
        out["f32_untuned"] = config_entry(r, n ** 3, 3, "f32", uv)
    # the other member of the fusion pair: one-stage march if the tuned one is fused, else the fused march
    other = dict(variants.ONE_STAGE_3D) if var.get("fuse") else dict(variants.FUSED_3D)
    r = run_gpu(None, "f32", other, steps, warmup, specs=[spec], fill=box_fill(n))
    out["f32_fused_march" if other["fuse"] else "f32_one_stage_march"] = config_entry(r, n ** 3, 3, "f32", other)
    return out


def batch_entries(steps: int, warmup: int, untuned: bool = True) -> dict:
    from paper_1204_4779_amd import binding as pb
    from paper_1204_4779_amd import inputs
    probs = inputs.blob_batch(512, seed=12044779)
    specs = [pb.MeshSpec(2, p.n, p.gamma, p.bc) for p in probs]
    cells = sum(p.n[0] * p.n[1] for p in probs)
    out = {"meshes": len(probs), "cells": cells}
    var = variants.tuned("batch512", "f32")
    r = run_gpu([p.U for p in probs], "f32", var, steps, warmup, specs=specs)
    out["f32_tuned"] = config_entry(r, cells, 2, "f32", var)
    out["f32_tuned"]["audit_drift"] = r["mass_energy_drift"]
    # the same kernel fed by the persistent per-XCD work queues instead of the plain grid
    qv = dict(var, persistent=1)
    r = run_gpu([p.U for p in probs], "f32", qv, steps, warmup, specs=specs)
    out["f32_persistent_queue"] = config_entry(r, cells, 2, "f32", qv)
    if untuned:
        uv = dict(variants.UNTUNED_2D)
        r = run_gpu([p.U for p in probs], "f32", uv, max(steps // 4, 6), min(warmup, 12), specs=specs)
        out["f32_untuned"] = config_entry(r, cells, 2, "f32", uv)
    return out


# ---------------------------------------------------------------------------------------
# the FP64 CPU oracle (bounded samples on the host: serial, and OpenMP on all cores)
# ---------------------------------------------------------------------------------------

def _oracle_steps(m, U, budget_s: float, max_steps: int = 1 << 30):
    import oracle
    dt = oracle.cfl_dt(m, U, CFL)
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        U = oracle.step(m, U, dt)
        dt = oracle.cfl_dt(m, U, CFL)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return k, time.perf_counter() - t0, U


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle(U, ndim: int, n: tuple, gamma: float, label: str, budget_s: float, parallel: bool,
               max_steps: int = 1 << 30) -> dict:
    """The oracle stepping the given state (CFL included) for about `budget_s` seconds."""
    import numpy as np
    import oracle
    oracle.use_openmp(parallel)
    try:
        m = oracle.Mesh(ndim, n, gamma, tuple([0] * ndim))
        cells = int(np.prod(n))
        k, el, _ = _oracle_steps(m, np.ascontiguousarray(U), budget_s, max_steps)
        cores = oracle.num_threads()
    finally:
        oracle.use_openmp(False)
    return {"value": cells * k / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} FP64 steps (+CFL) of {label}, {'OpenMP' if parallel else 'serial'} C, {el:.1f} s"}


def cpu_baselines(kh_U) -> dict:
    """The oracle on the host: KH 2048^2 serially (about 10 s) and on all cores (about 5 s,
    plus a check that one OpenMP step is bitwise the serial step); Sod 1024 to t = 0.2 in
    full; one step of the 3D box at 256^3 serially and on all cores; the 512^3 box on its
    first 32 planes (a periodic 512 x 512 x 32 sample) on all cores; the batch on its
    first 32 meshes serially."""
    import numpy as np
    import oracle
    from paper_1204_4779_amd import inputs
    out = {"host_cpu": _cpu_model(), "host_threads": os.cpu_count()}
    out["kh2048_serial"] = cpu_oracle(kh_U, 2, (N, N), 1.4, "the full 2048x2048 KH mesh", 10.0, False)
    out["kh2048_all_cores"] = cpu_oracle(kh_U, 2, (N, N), 1.4, "the full 2048x2048 KH mesh", 5.0, True)
    m = oracle.Mesh(2, (N, N), 1.4, (0, 0))
    dt = oracle.cfl_dt(m, kh_U, CFL)
    a = oracle.step(m, kh_U, dt)
    oracle.use_openmp(True)
    try:
        b = oracle.step(m, kh_U, dt)
    finally:
        oracle.use_openmp(False)
    out["kh2048_all_cores"]["bitwise_equal_to_serial"] = bool(np.array_equal(a, b))
    del a, b
    pr = inputs.sod_1d(1024)
    ms = oracle.Mesh(1, pr.n, pr.gamma, pr.bc)
    t0 = time.perf_counter()
    _, t, k = oracle.advance(ms, pr.U, CFL, 0.2)
    el = time.perf_counter() - t0
    out["sod1024_serial"] = {"value": 1024 * k / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                             "time_to_solution_ms": el * 1e3, "steps": k,
                             "sample": f"the whole run to t = 0.2 ({k} steps), serial C"}
    box = inputs.turbulent_box_3d(256, seed=4779).U
    out["box256_serial"] = cpu_oracle(box, 3, (256, 256, 256), 5.0 / 3.0, "the 256^3 box", 0.0, False, 1)
    out["box256_all_cores"] = cpu_oracle(box, 3, (256, 256, 256), 5.0 / 3.0, "the 256^3 box", 0.0, True, 1)
    del box
    slab = inputs.turbulent_box_3d(512, seed=4779, z_range=(0, 32)).U
    out["box512_all_cores"] = cpu_oracle(slab, 3, (512, 512, 32), 5.0 / 3.0,
                                         "the 512^3 box's first 32 planes (periodic sample)", 0.0, True, 1)
    del slab
    probs = inputs.blob_batch(32, seed=12044779)
    t0 = time.perf_counter()
    cells = 0
    for p in probs:
        mb = oracle.Mesh(2, p.n, p.gamma, p.bc)
        _oracle_steps(mb, p.U, 0.0, 1)
        cells += p.n[0] * p.n[1]
    el = time.perf_counter() - t0
    out["batch512_serial"] = {"value": cells / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                              "sample": f"one FP64 step (+CFL) of each of the first 32 meshes ({cells} cells), "
                                        f"serial C, {el:.1f} s"}
    return out


def calibration_copy():
    """Three plain device copies of 512 MiB: known bytes that scale the HBM counters."""
    import torch
    src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("calibration copy: 536870912 bytes read and written per launch, 3 launches")


def other_workload(name: str, steps: int, warmup: int, sizes=None, with_cpu: bool = True):
    """Cell-updates/s of the other configurations (one JSON line each, not the headline)."""
    if name == "sod1024":
        e = sod_entry()
        return dict(e, workload="sod_1d_1024_outflow_fp64_to_t0.2", unit="cell-updates/s", dtype="f64")
    if name in ("box256", "box512"):
        n = 256 if name == "box256" else 512
        es = box_entries(n, steps, warmup, untuned=False)
        out = dict(es["f32_tuned"], workload=f"box3d_{n}^3_periodic_fp32", unit="cell-updates/s", dtype="f32")
        for k in ("f32_fused_march", "f32_one_stage_march"):
            if k in es:
                out[k] = es[k]
        return out
    if name == "batch512":
        e = batch_entries(steps, warmup, untuned=False)
        return dict(e["f32_tuned"], workload="batch_512_uneven_2d_periodic_fp32", unit="cell-updates/s",
                    dtype="f32", cells=e["cells"], persistent_queue=e["f32_persistent_queue"])
    if name == "wave":
        return wave_workload(with_cpu)
    if name == "manifest":
        return manifest_table(steps, warmup)
    if name == "convergence":
        return convergence_study(tuple(sizes) if sizes else (16, 32, 64, 128, 256, 512, 1024), with_cpu)
    raise SystemExit(f"unknown workload {name}")


# Linear-wave kernel: flops per cell-update of the scheme and its energy term,
# with the per-line constants folded (c^2 dt/dx^2, 1/(2dx), dx/2, c^2):
# f update 2, g update 5, central difference 2, c^2 (df/dx)^2 2, mean of g
# and its square 3, sum 1, times dx/2 1, accumulate 1.
WAVE_FLOPS_PER_CELL_UPDATE = 17.0
# LDS bytes per cell-update: f^{n+1} written once, both neighbours read.
WAVE_LDS_BYTES_PER_CELL_UPDATE = 24.0
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12   # 128 B per clock per CU


def wave_workload(with_cpu: bool = True, lines: int = 2048, n: int = 3072, steps: int = 2000):
    """The linear-wave example: (1) the paper's experiment, one line per
    n = 8 ... 3072 at c = 3.43, dt = dx / c, f = sin x, g = cos 3x, 10000
    steps, energy fluctuation per n; (2) throughput: `lines` lines of n cells
    (phases shifted per line) advanced `steps` steps in one launch."""
    import numpy as np
    import torch
    from paper_1204_4779_amd import binding as pb
    c = 3.43
    fluct = {}
    sizes = [8 << k for k in range(9)] + [3072]
    fs, gs = [], []
    for m in sizes:
        x = np.arange(m) * (2 * math.pi / m)
        fs.append(np.sin(x))
        gs.append(np.cos(3 * x))
    dxs = [2 * math.pi / m for m in sizes]
    w = pb.WaveLines(fs, gs, c, dxs, [dx / c for dx in dxs], 10000)
    w.advance(10000)
    torch.cuda.synchronize()
    for m, e in zip(sizes, w.energy):
        e = e.cpu().numpy()
        fluct[str(m)] = float((e.max() - e.min()) / e[0])
    log(f"wave energy fluctuation over 10000 steps: {fluct}")
    del w
    # throughput
    dx = 2 * math.pi / n
    x = np.arange(n) * dx
    fs = [np.sin(x + 0.001 * k) for k in range(lines)]
    gs = [np.cos(3 * x + 0.002 * k) for k in range(lines)]
    w = pb.WaveLines(fs, gs, c, dx, dx / c, steps)
    w.prepare()
    w.run(200)                        # warm-up, also the clock ramp
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    w.run(steps)                      # one launch: `steps` steps of every line
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    cu = float(lines) * n * steps
    v = cu / (ms / 1e3)
    e = w.energy[0].cpu().numpy()
    achieved = v * WAVE_FLOPS_PER_CELL_UPDATE / 1e12
    out = {"workload": f"linear_wave_1d_{lines}x{n}_periodic_c3.43_fp64", "value": v, "unit": "cell-updates/s",
           "dtype": "f64", "steps": steps, "ms": ms,
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS["f64"],
                        "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS["f64"], 4), "traffic": None,
                        "kernel": "k_wave1d", "flops_per_cell_update": WAVE_FLOPS_PER_CELL_UPDATE},
           "lds_roofline": {"achieved": round(v * WAVE_LDS_BYTES_PER_CELL_UPDATE / 1e12, 3), "peak": LDS_PEAK_TBS,
                            "unit": "TB/s"},
           "energy_fluctuation_line0": float((e.max() - e.min()) / e[0]),
           "paper_experiment_energy_fluctuation": fluct}
    if with_cpu:
        import oracle.wave as ow
        f0, g0 = ow.paper_initial(n)
        t0 = time.perf_counter()
        k = 0
        f, g = f0, g0
        while time.perf_counter() - t0 < 10.0:
            f, g, _ = ow.step(f, g, c, dx, dx / c)
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * k / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"one line of {n} cells, {k} FP64 steps (numpy), {el:.1f} s"}
    return out


# The paper's hand-annotated individuals (table of codes annotated by hand):
# whether the results of the interpolation (face states) and of the Riemann
# solver (face fluxes) are stored and reused (Manifest) or recomputed where
# used (Delayed).  Here the stored values live in LDS within a tile; all four
# share one launch shape (32 x 16 cells, 256 threads, one launch per stage).
MANIFEST_POINTS = (
    ("Izanami (D,D)", dict(tile=(32, 16), lds=0, fuse=0, waves_per_eu=0, threads=256)),
    ("Iwatsuchibiko (M,D)", dict(tile=(32, 16), lds=1, fuse=0, waves_per_eu=0, threads=256, manifest=1)),
    ("Shinatsuhiko (D,M)", dict(tile=(32, 16), lds=1, fuse=0, waves_per_eu=0, threads=256, manifest=0)),
    ("Hayaakitsuhime (M,M)", dict(tile=(32, 16), lds=1, fuse=0, waves_per_eu=0, threads=256, manifest=2)),
)


def manifest_table(steps: int, warmup: int):
    """KH 2048^2 in FP32 and FP64 through the four Manifest/Delayed points."""
    from paper_1204_4779_amd import inputs
    pr = inputs.kelvin_helmholtz_2d(N, seed=1204)
    rows = []
    for name, var in MANIFEST_POINTS:
        row = {"individual": name, "variant": var}
        for dtype in ("f32", "f64"):
            r = run_gpu(pr.U, dtype, var, steps, warmup)
            v = N * N * r["steps"][0] / (r["event_ms"] / 1e3)
            row[dtype] = {"value": v, "ms_per_step": r["event_ms"] / r["steps"][0],
                          "alu_frac": v * FLOPS_PER_CELL_UPDATE[2] / 1e12 / ALU_PEAK_TFLOPS[dtype]}
            log(f"{name} {dtype}: {v / 1e9:.2f} G cell-updates/s")
        rows.append(row)
    best = max(rows, key=lambda r: r["f32"]["value"])
    return {"workload": "manifest_points_kelvin_helmholtz_2d_2048x2048", "value": best["f32"]["value"],
            "unit": "cell-updates/s", "dtype": "f32", "points": rows}


def convergence_study(sizes=(16, 32, 64, 128, 256, 512, 1024), with_cpu: bool = True):
    """The convergence tests on the unit square with analytic boundaries:
    entropy wave and sound wave (amplitude 1e-5) to t = 1, Sod's tube to
    t = 0.125, each coaxial and rotated by 60 degrees, N^2 cells for N in
    `sizes`, in FP64 and FP32.  Initial and reference states come from the
    library's exact-state kernel; the L1 norm of the density error is taken
    with torch.  Throughput: cell-updates of the largest-N runs over their
    device time (advance, CFL included)."""
    import torch
    from paper_1204_4779_amd import binding as pb
    problems = (("entropy", pb.ENTROPY_WAVE, 1.0), ("sound", pb.SOUND_WAVE, 1.0), ("sod", pb.SHOCK_TUBE, 0.125))
    table, perf = {}, {}
    for dtype in ("f64", "f32"):
        var = variants.TUNED.get(("convergence", dtype))
        big_cu, big_ms = 0.0, 0.0
        for pname, kind, t_end in problems:
            for tag, angle in (("coaxial", 0.0), ("oblique", math.pi / 3)):
                errs, steps = [], []
                for n in sizes:
                    s = pb.Solver(pb.MeshSpec(2, (n, n), 1.4, (pb.ANALYTIC, pb.ANALYTIC)), dtype)
                    s.set_analytic(kind, angle, 1e-5)
                    if var:
                        s.set_variant(var)
                    s.fill_exact(0.0)
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    a.record(s.stream)
                    t, k = s.advance(t_end, CFL)
                    b.record(s.stream)
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(b)
                    rho = s.state()[0].double().clone()
                    s.fill_exact(t_end)
                    exact = s.state()[0].double()
                    errs.append(float((rho - exact).abs().mean()))
                    steps.append(k[0])
                    if n == sizes[-1]:
                        big_cu += float(n * n * k[0])
                        big_ms += ms
                    s.close()
                orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
                table[f"{dtype}_{pname}_{tag}"] = {"N": list(sizes), "l1_rho": errs, "orders": orders, "steps": steps}
                log(f"{dtype} {pname} {tag}: L1 {['%.3e' % e for e in errs]} orders {['%.2f' % o for o in orders]}")
        v = big_cu / (big_ms / 1e3)
        esz = 4 if dtype == "f32" else 8
        perf[dtype] = {"value": v, "device_ms_n1024": big_ms, "variant": var or "library default",
                       "hbm_frac": v * bytes_per_cell_update(2, esz) / 1e9 / HBM_PEAK_GBS,
                       "alu_frac": v * FLOPS_PER_CELL_UPDATE[2] / 1e12 / ALU_PEAK_TFLOPS[dtype]}
    out = {"workload": f"convergence_tests_2d_unit_square_analytic_bc_N{sizes[0]}-{sizes[-1]}",
           "value": perf["f64"]["value"],
           "unit": "cell-updates/s", "dtype": "f64", "f32": perf["f32"], "f64": perf["f64"], "l1": table}
    if with_cpu:
        log("CPU oracle baseline (entropy wave, oblique, 128^2, to t = 1)")
        out["cpu_baseline"] = cpu_baseline_convergence()
    return out


def cpu_baseline_convergence(n: int = 128):
    """The FP64 oracle on one problem of the study: the oblique entropy wave
    on 128^2 cells with analytic boundaries, advanced to t = 1."""
    import numpy as np
    import oracle
    m = oracle.Mesh(2, (n, n), 1.4, (oracle.ANALYTIC, oracle.ANALYTIC))
    an = oracle.Analytic(oracle.ENTROPY_WAVE, math.pi / 3)
    U0 = np.ascontiguousarray(oracle.exact_state(m, an, 0.0))
    t0 = time.perf_counter()
    _, t, steps = oracle.advance(m, U0, CFL, 1.0, analytic=an)
    el = time.perf_counter() - t0
    return {"value": n * n * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oblique entropy wave, {n}x{n}, {steps} FP64 steps to t = 1, serial C, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # Every run first settles the clock (untimed, reported); the warm-up and the
    # timed steps then run at the steady clock.
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-extra", action="store_true", help="headline FP32 only")
    ap.add_argument("--variant", type=str, default=None, help="JSON variant for the headline run")
    ap.add_argument("--workload", default="kh2048",
                    choices=("kh2048", "sod1024", "box256", "box512", "batch512", "convergence", "manifest",
                             "wave"),
                    help="kh2048 is the headline; the others print their own line")
    ap.add_argument("--sizes", type=int, nargs="*", default=None,
                    help="convergence workload: mesh sizes N (default 16 32 ... 1024)")
    ap.add_argument("--prof", action="store_true",
                    help="profiling run: headline only, plus a 512 MiB device copy that calibrates HBM counters")
    ap.add_argument("--prof-fp64", action="store_true",
                    help="with --prof: run the FP64 tuned KH variant instead of the FP32 headline")
    args = ap.parse_args()
    if args.prof:
        args.no_cpu = args.no_extra = True
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the Euler step is measured "
                          "on a single MI355X; multi-GPU domain decomposition is not built"}))
        sys.exit(2)

    import torch
    from paper_1204_4779_amd import inputs
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload != "kh2048":
        out = other_workload(args.workload, args.steps, args.warmup, args.sizes, not args.no_cpu)
        out.update({"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "data": "synthetic"})
        if args.prof:
            calibration_copy()
        print(json.dumps(out))
        return
    log("generating KH 2048^2 input")
    pr = inputs.kelvin_helmholtz_2d(N, seed=1204)
    cells = N * N
    if args.prof and args.prof_fp64:
        r = run_gpu(pr.U, "f64", TUNED["f64"], args.steps, args.warmup)
        calibration_copy()
        print(json.dumps({"profiled": "kh2048 f64 tuned", "variant": TUNED["f64"], "steps": args.steps,
                          "ms_per_step": r["event_ms"] / args.steps}))
        return

    tuned32 = json.loads(args.variant) if args.variant else TUNED["f32"]
    log(f"FP32 tuned {tuned32}")
    r32 = run_gpu(pr.U, "f32", tuned32, args.steps, args.warmup)
    r32["steps"], r32["t"] = r32["steps"][0], r32["t"][0]
    ms = r32["event_ms"] / args.steps
    value = cells * args.steps / (r32["event_ms"] / 1e3)

    extra = {}
    if not args.no_extra:
        k_untuned = max(args.steps // 5, 6)
        log(f"FP64 tuned {TUNED['f64']}")
        r64 = run_gpu(pr.U, "f64", TUNED["f64"], args.steps, args.warmup)
        log(f"FP32 untuned {UNTUNED}")
        ru32 = run_gpu(pr.U, "f32", UNTUNED, k_untuned, min(args.warmup, 12))
        log(f"FP64 untuned {UNTUNED}")
        ru64 = run_gpu(pr.U, "f64", UNTUNED, k_untuned, min(args.warmup, 12))
        extra["kh2048"] = {
            "f32_tuned": config_entry(dict(r32, steps=[r32["steps"]]), cells, 2, "f32", tuned32),
            "f64_tuned": config_entry(r64, cells, 2, "f64", TUNED["f64"]),
            "f32_untuned": config_entry(ru32, cells, 2, "f32", UNTUNED),
            "f64_untuned": config_entry(ru64, cells, 2, "f64", UNTUNED)}
        log("FP32 tuned: 10 repetitions of 48 steps")
        extra["kh2048"]["f32_tuned_repetitions"] = repetitions(pr.U, "f32", tuned32)
        log("Sod 1024 FP64 to t = 0.2")
        extra["sod1024_f64"] = sod_entry()
        log("3D box 256^3 FP32")
        extra["box256"] = box_entries(256, args.steps, args.warmup)
        log("3D box 512^3 FP32")
        extra["box512"] = box_entries(512, args.steps, args.warmup)
        log("batch of 512 uneven 2D meshes FP32")
        extra["batch512"] = batch_entries(args.steps, args.warmup)

    # roofline of the dominant kernel (the fused step kernel: one launch per step): its
    # time per launch is the timed region less the advance call's fixed part, over the
    # launches (the gaps between the graph's kernels stay in); the figure with the fixed
    # part left in is reported beside it
    launch_ms_incl = r32["event_ms"] / r32["launches"]
    launch_ms = (r32["event_ms"] - r32["advance_fixed_ms"]) / r32["launches"]
    cells_per_launch = cells if tuned32.get("fuse", 1) else cells / 2.0
    flops = FLOPS_PER_CELL_UPDATE[2] * cells_per_launch
    achieved_tf = flops / (launch_ms / 1e3) / 1e12
    bytes_launch = bytes_per_cell_update(2, 4) * cells_per_launch
    achieved_gbs = bytes_launch / (launch_ms / 1e3) / 1e9
    traffic = None
    same_variant = all(tuple(tuned32.get(k, ())) == tuple(v) if isinstance(v, list) else tuned32.get(k) == v
                       for k, v in TRAFFIC["variant"].items())
    if _kernel_source_hash() == TRAFFIC["sources"] and same_variant:
        traffic = TRAFFIC["bytes_per_launch"]
    # At 379 flops per 32 bytes (11.8 flop/B) the published peaks put the ridge at
    # 157.3 / 8 = 19.7 flop/B: the roofline of this kernel is the HBM one.
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name(tuned32), "bytes_per_launch": bytes_launch, "launch_ms": round(launch_ms, 5),
                "launch_ms_incl_advance_fixed_part": round(launch_ms_incl, 5),
                "advance_fixed_ms": round(r32["advance_fixed_ms"], 4),
                "bytes_per_cell_update": bytes_per_cell_update(2, 4)}
    alu = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": ALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
           "frac": round(achieved_tf / ALU_PEAK_TFLOPS["f32"], 4),
           "peak_nonpacked": ALU_PEAK_NONPACKED_TFLOPS["f32"],
           "frac_nonpacked": round(achieved_tf / ALU_PEAK_NONPACKED_TFLOPS["f32"], 4),
           "flops_per_cell_update": FLOPS_PER_CELL_UPDATE[2],
           "flops_per_cell_update_oracle_code": FLOPS_ORACLE_CODE[2], "flops_per_launch": flops}

    if args.prof:
        calibration_copy()

    cpu, cpu_all = None, None
    if not args.no_cpu:
        log("CPU oracle baselines")
        cpu_all = cpu_baselines(pr.U)
        cpu = dict(cpu_all["kh2048_all_cores"])
        cpu["serial"] = cpu_all["kh2048_serial"]
        cpu["host_cpu"] = cpu_all["host_cpu"]

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "kelvin_helmholtz_2d_2048x2048_periodic_gamma1.4_seed1204", "cells": cells,
                   "cfl": CFL, "variant": tuned32, "hbm_frac": roofline["frac"]},
        "clock_settle": r32["clock_settle"],
        "roofline": roofline, "alu_roofline": alu, "cpu_baseline": cpu, "extra": extra,
        "cpu_oracle_all_configs": cpu_all,
        "audit": {"f32_conserved_total_drift": r32["mass_energy_drift"],
                  "steps": args.steps + args.warmup + r32["clock_settle"]["steps"], "t_end": r32["t"]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
