"""First-order (piecewise-constant) reconstruction on the GPU against the oracle.

The order-1 branch of the paper's interpolation listing: each face takes the
values of the two cells beside it.  It runs on the LDS-tile kernels (fused
and unfused, and the unfused one with analytic boundaries).  One step from
identical input with an explicit dt: FP64 within 1e-12 and FP32 within 1e-5,
on meshes that span several tiles and end in a ragged tile.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

from gpu_util import TOL, as_input, gpu_solver, gpu_state, rel_err, state_err

pytestmark = pytest.mark.gpu

SHAPES = {1: (203,), 2: (37, 21), 3: (19, 11, 10)}
TILES = {1: (64, 1, 1), 2: (16, 8, 1), 3: (8, 4, 4)}


def _spec(pr, order=1):
    return pb.MeshSpec(pr.ndim, pr.n, pr.gamma, pr.bc, order=order)


def _mesh(pr, order=1):
    return oracle.Mesh(pr.ndim, pr.n, pr.gamma, pr.bc, order=order)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("fuse", [0, 1, None])
def test_one_step_matches_oracle(dtype, ndim, bc, fuse):
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=300 + 10 * ndim + bc, rough=True, bc=(bc,) * ndim)
    m = _mesh(pr)
    U0 = as_input(pr.U, dtype)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    v = None if fuse is None else dict(tile=TILES[ndim], lds=1, fuse=fuse)
    s = gpu_solver(_spec(pr), dtype, v, U0)
    if fuse is None:
        assert s.variant()["lds"] == 1        # the library's own choice for order 1
    s.step(dt)
    err = rel_err(gpu_state(s), ref)
    s.close()
    assert err <= TOL[dtype], err


def test_first_order_differs_from_minbee():
    # the same input through both orders: the results differ by far more than rounding
    pr = inputs.random_state(2, (40, 24), seed=311, rough=True)
    dt = oracle.cfl_dt(_mesh(pr), pr.U, 0.5)
    out = {}
    for order in (1, 2):
        s = gpu_solver(_spec(pr, order), "f64", dict(tile=(16, 8), lds=1, fuse=1), pr.U)
        s.step(dt)
        out[order] = gpu_state(s)
        s.close()
        assert rel_err(out[order], oracle.step(_mesh(pr, order), pr.U, dt)) <= 1e-12
    assert rel_err(out[1], out[2]) > 1e-3


def test_advance_and_batch():
    probs = [inputs.blob_2d(n, 12044779, k) for k, n in enumerate((40, 72, 33))]
    specs = [_spec(p) for p in probs]
    b = gpu_solver(specs, "f64", dict(tile=(16, 16), lds=1, fuse=1, persistent=1), [p.U for p in probs])
    t, n = b.advance(0.01, 0.5, t0=[0.0, 0.0, 0.0])
    for k, p in enumerate(probs):
        ref, t_ref, n_ref = oracle.advance(_mesh(p), p.U, 0.5, 0.01)
        assert n[k] == n_ref and t[k] == t_ref
        assert rel_err(gpu_state(b, k), ref) < 1e-11
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_with_analytic_boundaries(dtype):
    an = oracle.Analytic(oracle.SHOCK_TUBE, math.pi / 3)
    m = oracle.Mesh(2, (37, 29), 1.4, (pb.ANALYTIC, pb.ANALYTIC), order=1)
    U0 = as_input(oracle.exact_state(m, an, 0.05), dtype)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt, 0.05, an)
    s = pb.Solver(pb.MeshSpec(2, (37, 29), 1.4, (pb.ANALYTIC, pb.ANALYTIC), order=1), dtype)
    s.set_analytic(an.kind, an.angle)
    assert (s.variant()["lds"], s.variant()["fuse"]) == (1, 0)
    s.upload(U0)
    s.set_time(0.05)
    s.step(dt)
    assert state_err(gpu_state(s), ref, 1.4) <= TOL[dtype]
    s.close()


def test_first_order_convergence_matches_oracle():
    # entropy wave with analytic boundaries to t = 1: first-order L1 convergence,
    # the GPU's error equal to the oracle's at N = 32
    an = oracle.Analytic(oracle.ENTROPY_WAVE, math.pi / 3)
    errs = []
    for n in (32, 64, 128, 256):
        s = pb.Solver(pb.MeshSpec(2, (n, n), 1.4, (pb.ANALYTIC, pb.ANALYTIC), order=1), "f64")
        s.set_analytic(an.kind, an.angle)
        s.fill_exact(0.0)
        t, _ = s.advance(1.0, 0.5)
        rho = gpu_state(s)[0]
        s.fill_exact(1.0)
        errs.append(float(np.mean(np.abs(rho - gpu_state(s)[0]))))
        s.close()
    m = oracle.Mesh(2, (32, 32), 1.4, (pb.ANALYTIC, pb.ANALYTIC), order=1)
    U, _, _ = oracle.advance(m, oracle.exact_state(m, an, 0.0), 0.5, 1.0, analytic=an)
    want = float(np.mean(np.abs(U[0] - oracle.exact_state(m, an, 1.0)[0])))
    assert abs(errs[0] - want) <= 1e-8 * want
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    print(f"  first order, oblique entropy wave: L1 {errs} orders {orders}", flush=True)
    assert all(0.75 < o < 1.15 for o in orders), (errs, orders)


def test_first_order_rejects_other_kernel_families():
    pr = inputs.random_state(2, (64, 64), seed=312)
    s = gpu_solver(_spec(pr), "f32", None, pr.U)
    for v in (dict(tile=(64, 8), lds=2, fuse=1, threads=256), dict(tile=(16, 8), lds=0, fuse=0)):
        with pytest.raises(pb.ParaisoError) as ei:
            s.set_variant(v)
        assert ei.value.code == pb.ERR_UNSUPPORTED
    s.close()
