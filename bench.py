#!/usr/bin/env python3
"""Benchmark: cell-updates per second of the Euler step on one MI355X.

Workload: 2D periodic Kelvin-Helmholtz, 2048 x 2048 cells, gamma = 1.4 (seeded
1% v_y perturbation), advanced with the device-resident CFL time step
(CFL 0.5) by paraiso_advance; one step = both Runge-Kutta stages plus the CFL
reduction of the new state.  Inputs are resident in HBM before timing.

Prints one JSON line.  Besides the headline FP32 number it reports FP64, the
untuned (per-cell, unfused, no LDS) variant, the roofline of the dominant
kernel, and the FP64 CPU oracle timed on a bounded sample on the host.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--no-cpu] [--variant JSON]
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

# Algorithmic work per cell-update on this workload, counted by running the
# oracle's arithmetic on a counting number type (oracle/flopcount.cpp, via
# oracle.count_ops on the 256^2 version of this workload): adds+muls+divs+sqrts
# of one step and its CFL reduction.  Compares/min/max/abs (145) not counted.
FLOPS_PER_CELL_UPDATE = {2: 730.6}
# Algorithmic HBM bytes per cell-update: read U^n once, write U^{n+1} once.
def bytes_per_cell_update(ndim: int, esize: int) -> int:
    return 2 * (ndim + 2) * esize

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, each scaled by the reading of a plain 512 MiB device copy
# (factors 2.000 and 1.000); valid only for the kernel sources they were taken
# on (hash of the device headers) and the variant named.
TRAFFIC = {"sources": "569ff4b8b5c7391a", "variant": {"tile": [32, 32], "lds": 1, "fuse": 1},
           "bytes_per_launch": 137.1e6}


def _kernel_source_hash() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_1204_4779_amd", "csrc")
    digests = ""
    for f in ("euler_device.h", "euler_kernels.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            digests += hashlib.sha256(fh.read()).hexdigest() + "\n"
    return hashlib.sha256(digests.encode()).hexdigest()[:16]
# FP32 without packed math (compiled out): 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
ALU_PEAK_PACKED_F32 = 157.3

from paper_1204_4779_amd import variants  # noqa: E402

TUNED = {"f32": variants.tuned("kh2048", "f32"), "f64": variants.tuned("kh2048", "f64")}
UNTUNED = dict(variants.UNTUNED_2D)


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(U, dtype: str, variant: dict, steps: int, warmup: int):
    import torch
    from paper_1204_4779_amd import binding as pb
    spec = pb.MeshSpec(2, (N, N), 1.4, (0, 0))
    s = pb.Solver(spec, dtype)
    s.set_variant(variant)
    s.upload(U)
    tot0 = s.totals()[0]
    t = [0.0]
    if warmup:
        t, _ = s.advance(float("inf"), CFL, max_steps=warmup, t0=t)
    stream = s.stream
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record(stream)
    t, n = s.advance(float("inf"), CFL, max_steps=steps, t0=t)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ev_ms = start.elapsed_time(stop)
    tot1 = s.totals()[0]
    drift = max(abs(a - b) / max(abs(a), 1e-300) for a, b in zip(tot0, tot1) if abs(a) > 0)
    launches = steps * (1 if variant.get("fuse", 1) else 2)
    s.close()
    del s
    torch.cuda.empty_cache()
    return {"wall_s": wall, "event_ms": ev_ms, "steps": n[0], "t": t[0], "launches": launches,
            "mass_energy_drift": drift}


def cpu_baseline(U, budget_s: float = 12.0):
    import numpy as np
    import oracle
    m = oracle.Mesh(2, (N, N), 1.4, (0, 0))
    U = np.ascontiguousarray(U)
    dt = oracle.cfl_dt(m, U, CFL)
    t0 = time.perf_counter()
    steps = 0
    while True:
        U = oracle.step(m, U, dt)
        dt = oracle.cfl_dt(m, U, CFL)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": N * N * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 steps (+CFL) of the full 2048x2048 KH mesh, serial C, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="headline FP32 only")
    ap.add_argument("--variant", type=str, default=None, help="JSON variant for the headline run")
    ap.add_argument("--prof", action="store_true",
                    help="profiling run: headline only, plus a 512 MiB device copy that calibrates HBM counters")
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
    log("generating KH 2048^2 input")
    pr = inputs.kelvin_helmholtz_2d(N, seed=1204)
    cells = N * N

    tuned32 = json.loads(args.variant) if args.variant else TUNED["f32"]
    log(f"FP32 tuned {tuned32}")
    r32 = run_gpu(pr.U, "f32", tuned32, args.steps, args.warmup)
    ms = r32["event_ms"] / args.steps
    value = cells * args.steps / (r32["event_ms"] / 1e3)

    extra = {}
    if not args.no_extra:
        log(f"FP64 tuned {TUNED['f64']}")
        r64 = run_gpu(pr.U, "f64", TUNED["f64"], args.steps, args.warmup)
        log(f"FP32 untuned {UNTUNED}")
        ru32 = run_gpu(pr.U, "f32", UNTUNED, max(args.steps // 4, 10), min(args.warmup, 5))
        log(f"FP64 untuned {UNTUNED}")
        ru64 = run_gpu(pr.U, "f64", UNTUNED, max(args.steps // 4, 10), min(args.warmup, 5))
        for name, r, dt, var in (("f64_tuned", r64, "f64", TUNED["f64"]), ("f32_untuned", ru32, "f32", UNTUNED),
                                 ("f64_untuned", ru64, "f64", UNTUNED)):
            k = r["steps"]
            cups = cells * k / (r["event_ms"] / 1e3)
            esz = 4 if dt == "f32" else 8
            extra[name] = {"value": cups, "ms_per_step": r["event_ms"] / k, "variant": var,
                           "hbm_frac": cups * bytes_per_cell_update(2, esz) / 1e9 / HBM_PEAK_GBS,
                           "alu_frac": cups * FLOPS_PER_CELL_UPDATE[2] / 1e12 / ALU_PEAK_TFLOPS[dt]}

    # roofline of the dominant kernel (the fused step kernel: one launch per step)
    launch_ms = r32["event_ms"] / r32["launches"]
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
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": ALU_PEAK_TFLOPS["f32"],
                "unit": "TFLOP/s", "frac": round(achieved_tf / ALU_PEAK_TFLOPS["f32"], 4), "traffic": traffic,
                "kernel": "k_fused_lds<float,2>", "flops_per_launch": flops, "launch_ms": round(launch_ms, 5),
                "peak_packed_f32": ALU_PEAK_PACKED_F32}
    hbm = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": bytes_launch}

    if args.prof:
        # plain copy of known size: 512 MiB read + 512 MiB written
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 536870912 bytes read and written per launch, 3 launches")

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(pr.U)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "kelvin_helmholtz_2d_2048x2048_periodic_gamma1.4_seed1204", "cells": cells,
                   "cfl": CFL, "variant": tuned32, "hbm_frac": hbm["frac"]},
        "roofline": roofline, "hbm_roofline": hbm, "cpu_baseline": cpu, "extra": extra,
        "audit": {"f32_total_rel_drift": r32["mass_energy_drift"], "t_end": r32["t"]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
