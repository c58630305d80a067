"""Parity at the workloads' full sizes, in the launch configurations that are benchmarked.

KH 2048^2 (the benchmark workload), the 3D box at 256^3 and every cell of
the 512-mesh batch are compared cell by cell with the oracle (run on all host
cores; its OpenMP build is bitwise the serial one).  The 512^3 box is
compared on whole z-planes: the oracle steps a 512 x 512 x (2R+1) slab around
each sampled plane (R = 4, the reach of one fused step; periodic in x and y),
whose centre plane depends only on planes inside the slab.  The sampled
planes sit on both sides of the kernel's plane-chunk seams and at the
periodic wrap; every plane covers every strip and row-block seam.

Measures: every field normwise against its own maximum and density and
energy pointwise (`rel_err`); where momenta start at rest or as a small
perturbation (KH's v_y, the blobs) FP32 momenta are held against
max rho (|v| + c) (`state_err`), and the strict numbers are printed.
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs, variants

from gpu_util import (TOL, as_input, field_errs, gpu_solver, gpu_state, measures, oracle_mesh, rel_err, spec_of,
                      state_err)

pytestmark = pytest.mark.gpu

R = 4


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_kh2048_full_field(dtype):
    print(f"case kh2048 {dtype}", flush=True)
    pr = inputs.kelvin_helmholtz_2d(2048, seed=1204)
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    s = gpu_solver(spec_of(pr), dtype, variants.tuned("kh2048", dtype), pr.U)
    got_dt = s.cfl_dt(0.5)[0]
    assert abs(got_dt - dt) <= 1e-14 * dt
    s.step(dt)
    got = gpu_state(s)
    err = rel_err(got, ref) if dtype == "f64" else state_err(got, ref, pr.gamma)
    print(f"  kh2048 {dtype} err {err:.3e} {measures(got, ref, pr.gamma)}", flush=True)
    assert err <= TOL[dtype]
    tot_ref = oracle.totals(m, ref)
    tot = np.array(s.totals()[0])
    np.testing.assert_allclose(tot, oracle.totals(m, as_input(gpu_state(s), "f64")), rtol=1e-13, atol=1e-13)
    assert np.all(np.abs(tot - tot_ref) <= TOL[dtype] * np.abs(oracle.totals(m, np.abs(ref))))


def test_box256_full_field():
    # every cell of the 3D box at 256^3: tuned register march, fused LDS tile, fused register march
    print("case box256 f32 full field", flush=True)
    pr = inputs.turbulent_box_3d(256, seed=4779)
    U0 = as_input(pr.U, "f32")
    m = oracle_mesh(pr)
    oracle.use_openmp(True)
    try:
        dt = oracle.cfl_dt(m, U0, 0.5)
        ref = oracle.step(m, U0, dt)
    finally:
        oracle.use_openmp(False)
    del U0
    for v in (variants.tuned("box256", "f32"), dict(tile=(8, 8, 8), lds=1, fuse=1, threads=256),
              dict(tile=(64, 12, 64), lds=2, fuse=1)):
        s = gpu_solver(spec_of(pr), "f32", v, pr.U)
        got_dt = s.cfl_dt(0.5)[0]
        assert abs(got_dt - dt) <= 1e-14 * dt
        s.step(dt)
        got = gpu_state(s)
        s.close()
        err = rel_err(got, ref)
        print(f"  box256 {v} err {err:.3e} {measures(got, ref, pr.gamma)}", flush=True)
        assert err <= TOL["f32"]
        del got


def test_batch512_full():
    # every member compared cell by cell (33 M cells in all)
    print("case batch512 f32", flush=True)
    probs = inputs.blob_batch(512, seed=12044779)
    specs = [spec_of(p) for p in probs]
    U0s = [as_input(p.U, "f32") for p in probs]
    dts = [oracle.cfl_dt(oracle_mesh(p), u, 0.5) for p, u in zip(probs, U0s)]
    s = gpu_solver(specs, "f32", variants.tuned("batch512", "f32"), [p.U for p in probs])
    got_dts = s.cfl_dt(0.5)
    np.testing.assert_allclose(got_dts, dts, rtol=1e-14)
    s.step(dts)
    worst, worst_state, worst_k, worst_f = 0.0, 0.0, -1, None
    for k, p in enumerate(probs):
        ref = oracle.step(oracle_mesh(p), U0s[k], dts[k])
        got = gpu_state(s, k)
        e = rel_err(got, ref)
        if e > worst:
            worst, worst_k, worst_f = e, k, field_errs(got, ref)
        worst_state = max(worst_state, state_err(got, ref, p.gamma))
    print(f"  batch512 strict {worst:.3e} (mesh {worst_k}, n={probs[worst_k].n[0]}, per field {worst_f}); "
          f"state-scaled with pointwise rho, E {worst_state:.3e}", flush=True)
    assert worst_state <= TOL["f32"]
    # the same kernel fed by the persistent work queues: bitwise the plain grid's step
    print("case batch512 f32 persistent queue", flush=True)
    q = gpu_solver(specs, "f32", dict(variants.tuned("batch512", "f32"), persistent=1), [p.U for p in probs])
    q.step(dts)
    for k in range(len(probs)):
        assert np.array_equal(gpu_state(q, k), gpu_state(s, k)), k


def box512_planes(chunk: int) -> list:
    """z-planes to compare: both sides of every third plane-chunk seam, the
    periodic wrap, and a few between seams."""
    n = 512
    zs = {0, n - 1, 1, n - 2, 200, 333}
    for z in range(chunk, n, 3 * chunk):
        zs.update((z - 1, z))
    return sorted(zs)


@pytest.mark.slow
def test_box512_planes():
    import torch
    n = 512
    var = variants.tuned("box512", "f32")
    planes = box512_planes(var["tile"][2])
    print(f"case box512 f32 planes {planes}", flush=True)
    spec = pb.MeshSpec(3, (n, n, n), 5.0 / 3.0, (0, 0, 0))
    s = pb.Solver(spec, "f32")
    s.set_variant(var)
    buf = s.state()
    # the FP64 values of the (2R+1)-plane slab around each sampled plane
    slabs = {z: np.zeros((5, 2 * R + 1, n, n)) for z in planes}
    qmax = 0.0
    oracle.use_openmp(True)
    try:
        for z0 in range(0, n, 32):
            sl = inputs.turbulent_box_3d(n, seed=4779, z_range=(z0, z0 + 32))
            buf[:, z0:z0 + 32].copy_(torch.from_numpy(sl.U.astype(np.float32)))
            u32 = as_input(sl.U, "f32")
            m = oracle.Mesh(3, (n, n, 32), sl.gamma, (0, 0, 0), dx=(1.0 / n,) * 3)
            qmax = max(qmax, oracle.cfl_qmax(m, u32))
            for zc, slab in slabs.items():
                for zi, o in enumerate(range(-R, R + 1)):
                    z = (zc + o) % n
                    if z0 <= z < z0 + 32:
                        slab[:, zi] = u32[:, z - z0]
            del sl, u32
        torch.cuda.synchronize()
        dt = 0.5 / qmax
        got_dt = s.cfl_dt(0.5)[0]
        assert abs(got_dt - dt) <= 1e-14 * dt
        s.step(dt)
        torch.cuda.synchronize()
        m = oracle.Mesh(3, (n, n, 2 * R + 1), 5.0 / 3.0, (0, 0, 1), dx=(1.0 / n,) * 3)
        worst = 0.0
        for zc in planes:
            ref = oracle.step(m, slabs[zc], dt)[:, R]
            got = s.state()[:, zc].double().cpu().numpy()
            e = rel_err(got, ref)
            worst = max(worst, e)
            print(f"  box512 plane {zc}: err {e:.3e} {measures(got, ref, 5.0 / 3.0)}", flush=True)
            assert e <= TOL["f32"], zc
    finally:
        oracle.use_openmp(False)
    s.close()
    print(f"  box512 worst plane err {worst:.3e}", flush=True)
