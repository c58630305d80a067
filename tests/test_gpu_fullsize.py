"""Parity at the workloads' full sizes, in the launch configurations that are benchmarked.

KH 2048^2 (the benchmark workload) is compared cell by cell with the oracle.
The 3D boxes and the 512-mesh batch are compared on sampled cells: the oracle
steps a (2R+1)^d block around each sampled cell (R = 4, the reach of one fused
step), whose centre value depends only on cells inside the block.
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs, variants

from gpu_util import TOL, as_input, field_errs, gpu_solver, gpu_state, oracle_mesh, rel_err, spec_of, state_err

pytestmark = pytest.mark.gpu

R = 4


def local_oracle(U, pr, cells, dt):
    """Oracle one-step values at the given cells (x, y, z index tuples) of a periodic mesh."""
    d, nf = pr.ndim, pr.ndim + 2
    n = pr.n
    dx = tuple(1.0 / n[a] for a in range(d))
    m = oracle.Mesh(d, (2 * R + 1,) * d, pr.gamma, (1, 1, 1), dx=dx)
    out = np.empty((len(cells), nf))
    for k, c in enumerate(cells):
        idx = [(np.arange(-R, R + 1) + c[a]) % n[a] for a in range(d)]
        block = U[np.ix_(range(nf), *reversed(idx))]
        res = oracle.step(m, block, dt)
        out[k] = res[(slice(None),) + (R,) * d]
    return out


def sample_cells(rng, n, d, count):
    return [tuple(int(rng.integers(0, n[a])) for a in range(d)) for _ in range(count)]


def gather(U, cells, d):
    return np.array([U[(slice(None),) + tuple(reversed(c[:d]))] for c in cells])


def sampled_err(got, ref):
    scale = np.max(np.abs(ref), axis=0)
    return float(np.max(np.abs(got - ref) / np.where(scale > 0, scale, 1.0)))


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
    err = rel_err(gpu_state(s), ref)
    print(f"  kh2048 {dtype} rel err {err:.3e} per field {field_errs(gpu_state(s), ref)} "
          f"state-scaled {state_err(gpu_state(s), ref, pr.gamma):.3e}", flush=True)
    assert err <= TOL[dtype]
    tot_ref = oracle.totals(m, ref)
    tot = np.array(s.totals()[0])
    np.testing.assert_allclose(tot, oracle.totals(m, as_input(gpu_state(s), "f64")), rtol=1e-13, atol=1e-13)
    assert np.all(np.abs(tot - tot_ref) <= TOL[dtype] * np.abs(oracle.totals(m, np.abs(ref))))


def test_box256_sampled():
    print("case box256 f32", flush=True)
    pr = inputs.turbulent_box_3d(256, seed=4779)
    U0 = as_input(pr.U, "f32")
    dt = oracle.cfl_dt(oracle_mesh(pr), U0, 0.5)
    rng = np.random.default_rng(256)
    cells = sample_cells(rng, pr.n, 3, 96)
    ref = local_oracle(U0, pr, cells, dt)
    for v in (variants.tuned("box256", "f32"), dict(tile=(8, 8, 8), lds=1, fuse=1, threads=256)):
        s = gpu_solver(spec_of(pr), "f32", v, pr.U)
        s.step(dt)
        got = gather(gpu_state(s), cells, 3)
        err = sampled_err(got, ref)
        print(f"  box256 {v} sampled rel err {err:.3e}", flush=True)
        assert err <= TOL["f32"]
        s.close()


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
    print(f"  batch512 rel err {worst:.3e} (mesh {worst_k}, n={probs[worst_k].n[0]}, per field {worst_f}); "
          f"state-scaled {worst_state:.3e}", flush=True)
    assert worst_state <= TOL["f32"]


@pytest.mark.slow
def test_box512_sampled():
    print("case box512 f32", flush=True)
    import torch
    n = 512
    spec = pb.MeshSpec(3, (n, n, n), 5.0 / 3.0, (0, 0, 0))
    s = pb.Solver(spec, "f32")
    s.set_variant(variants.tuned("box512", "f32"))
    buf = s.state()
    rng = np.random.default_rng(5120)
    cells = sample_cells(rng, (n, n, n), 3, 48)
    blocks = np.zeros((len(cells), 5, 2 * R + 1, 2 * R + 1, 2 * R + 1))
    win = [((np.arange(-R, R + 1) + c[1]) % n, (np.arange(-R, R + 1) + c[0]) % n) for c in cells]
    qmax = 0.0
    for z0 in range(0, n, 32):
        sl = inputs.turbulent_box_3d(n, seed=4779, z_range=(z0, z0 + 32))
        buf[:, z0:z0 + 32].copy_(torch.from_numpy(sl.U.astype(np.float32)))
        u32 = as_input(sl.U, "f32")
        m = oracle.Mesh(3, (n, n, 32), sl.gamma, (0, 0, 0), dx=(1.0 / n,) * 3)
        qmax = max(qmax, oracle.cfl_qmax(m, u32))
        for k, c in enumerate(cells):
            for zi, o in enumerate(range(-R, R + 1)):
                z = (c[2] + o) % n
                if z0 <= z < z0 + 32:
                    iy, ix = win[k]
                    blocks[k][:, zi] = u32[:, z - z0][:, iy][:, :, ix]
    torch.cuda.synchronize()
    dt = 0.5 / qmax
    got_dt = s.cfl_dt(0.5)[0]
    assert abs(got_dt - dt) <= 1e-14 * dt
    m = oracle.Mesh(3, (2 * R + 1,) * 3, 5.0 / 3.0, (1, 1, 1), dx=(1.0 / n,) * 3)
    refs = np.array([oracle.step(m, blocks[k], dt)[:, R, R, R] for k in range(len(cells))])
    s.step(dt)
    torch.cuda.synchronize()
    got = np.array([s.state()[(slice(None), c[2], c[1], c[0])].double().cpu().numpy() for c in cells])
    err = sampled_err(got, refs)
    print(f"  box512 sampled rel err {err:.3e}", flush=True)
    assert err <= TOL["f32"]
