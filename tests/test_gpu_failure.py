"""A state that turns non-physical part-way through paraiso_advance: the advance
stops after the step that produced it, as the oracle's advance does, and
reports NONFINITE with that step's time and count; the state buffers hold
that step's output.  Input: a cold, randomly stirred patch (seed 23,
amplitude 0.5, p = 1e-3) whose pressure goes negative in the output of step
3 in FP64 and FP32 alike, while every state that step's fluxes are computed
from stays physical: the oracle's minimum pressure is 2.3e-4 after step 2,
9.3e-5 in step 3's stage-1 state and -5.4e-5 after step 3, margins far above
either precision's rounding.  (A stage-1 state that is already non-physical
would make the failing step's output depend on how each side evaluates a
sound speed from a negative pressure, which no definition fixes.)"""
import math

import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

from gpu_util import TOL, as_input, field_errs, gpu_solver, gpu_state, oracle_mesh, spec_of

pytestmark = pytest.mark.gpu

FAMILIES = {
    "march_fused": dict(tile=(64, 8), lds=2, fuse=1, threads=128),
    "march": dict(tile=(64, 8), lds=2, fuse=0, threads=128),
    "lds_fused": dict(tile=(16, 8), lds=1, fuse=1),
    "lds": dict(tile=(16, 8), lds=1, fuse=0),
    "direct": dict(tile=(16, 8), lds=0, fuse=0),
}


def failing_problem():
    return inputs.cold_stirred_2d((40, 24), seed=23, amp=0.5)


def _pmin(U):
    m2 = U[1] ** 2 + U[2] ** 2
    return float(np.min(0.4 * (U[3] - 0.5 * m2 / U[0])))


def assert_stage1_physical(pr, U):
    """The failing step's inputs and its stage-1 state are physical by a wide margin; only
    its output is not (so the output is fixed by the scheme on both sides)."""
    m = oracle_mesh(pr)
    U2, _, k, ok = oracle.advance(m, U, 0.5, math.inf, max_steps=2, on_failure="return")
    assert ok and k == 2
    dt = oracle.cfl_dt(m, U2, 0.5)
    U1 = oracle.stage(m, U2, U2, 0.5 * dt)
    assert _pmin(U2) > 1e-4 and _pmin(U1) > 5e-5
    assert _pmin(oracle.stage(m, U1, U2, dt)) < -5e-5


@pytest.mark.parametrize("t_end", [math.inf, 1.0])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("family", sorted(FAMILIES))
def test_advance_stops_at_the_failing_step(family, dtype, t_end):
    pr = failing_problem()
    U = as_input(pr.U, dtype)
    ref, t_ref, k_ref, ok = oracle.advance(oracle_mesh(pr), U, 0.5, t_end, max_steps=20, on_failure="return")
    assert not ok and k_ref == 3
    assert_stage1_physical(pr, U)
    s = gpu_solver([spec_of(pr)], dtype, FAMILIES[family], pr.U)
    print(f"failure advance: {family} {dtype} t_end={t_end}", flush=True)
    with pytest.raises(pb.NonFiniteError) as ei:
        s.advance(t_end, 0.5, max_steps=20)
    assert ei.value.steps == [k_ref]
    assert abs(ei.value.t[0] - t_ref) <= (1e-13 if dtype == "f64" else 1e-6) * t_ref
    got = gpu_state(s)
    errs = field_errs(got, ref)
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert max(errs) <= tol, errs
    # a second advance from the failed state takes no step and fails again
    with pytest.raises(pb.NonFiniteError) as ei2:
        s.advance(t_end, 0.5, max_steps=20, t0=ei.value.t)
    assert ei2.value.steps == [0]
    assert np.array_equal(gpu_state(s), got)
    s.close()


def test_batch_failing_mesh_stops_others_continue():
    """Two meshes in one persistent launch per step: the failing mesh stops at its
    step 3, the other one takes all 12 steps (FP64)."""
    bad = failing_problem()
    good = inputs.random_state(2, (40, 24), seed=77, bc=(0, 0))
    specs = [spec_of(bad), spec_of(good)]
    s = gpu_solver(specs, "f64", dict(FAMILIES["march_fused"], persistent=1), [bad.U, good.U])
    with pytest.raises(pb.NonFiniteError) as ei:
        s.advance(math.inf, 0.5, max_steps=12)
    assert ei.value.steps == [3, 12]
    ref_bad, t_bad, k_bad, ok = oracle.advance(oracle_mesh(bad), bad.U, 0.5, math.inf, max_steps=12,
                                               on_failure="return")
    ref_good, t_good, k_good = oracle.advance(oracle_mesh(good), good.U, 0.5, math.inf, max_steps=12)
    assert (k_bad, k_good, ok) == (3, 12, False)
    assert abs(ei.value.t[0] - t_bad) <= 1e-13 * t_bad
    assert abs(ei.value.t[1] - t_good) <= 1e-13 * t_good
    assert max(field_errs(gpu_state(s, 0), ref_bad)) <= 1e-11
    assert max(field_errs(gpu_state(s, 1), ref_good)) <= 1e-11
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_resident_1d_advance_stops_at_the_failing_step(dtype):
    """The resident 1D kernel (the whole advance in one launch, its own CFL
    reduction per step): a cold stirred line of 200 cells (seed 14, amplitude
    0.5, p = 1e-3) whose pressure goes negative in the output of step 2 (the
    oracle's minimum pressure: 3.5e-4 after step 1, 9.1e-5 in step 2's
    stage-1 state, -6.0e-5 after step 2)."""
    pr = inputs.cold_stirred_1d(200, seed=14, amp=0.5)
    U = as_input(pr.U, dtype)
    ref, t_ref, k_ref, ok = oracle.advance(oracle_mesh(pr), U, 0.5, math.inf, max_steps=20, on_failure="return")
    assert not ok and k_ref == 2
    s = gpu_solver([spec_of(pr)], dtype, dict(tile=(200,), lds=3, fuse=1), pr.U)
    print(f"resident failure advance: {dtype}", flush=True)
    with pytest.raises(pb.NonFiniteError) as ei:
        s.advance(math.inf, 0.5, max_steps=20)
    assert ei.value.steps == [k_ref]
    assert abs(ei.value.t[0] - t_ref) <= (1e-13 if dtype == "f64" else 1e-6) * t_ref
    got = gpu_state(s)
    assert max(field_errs(got, ref)) <= (1e-11 if dtype == "f64" else 2e-5)
    with pytest.raises(pb.NonFiniteError) as ei2:
        s.advance(math.inf, 0.5, max_steps=20, t0=ei.value.t)
    assert ei2.value.steps == [0]
    assert np.array_equal(gpu_state(s), got)
    s.close()


# (FP32 variant, FP64 variant): the FP64 LDS tiles hold fewer cells
FAMILIES_3D = {
    "march": (dict(tile=(64, 4, 64), lds=2, fuse=0, waves_per_eu=3),) * 2,
    "march_fused": (dict(tile=(64, 12, 64), lds=2, fuse=1), dict(tile=(64, 6, 32), lds=2, fuse=1)),
    "lds_fused": (dict(tile=(8, 8, 8), lds=1, fuse=1), dict(tile=(8, 4, 4), lds=1, fuse=1)),
    "direct": (dict(tile=(16, 4, 4), lds=0, fuse=0),) * 2,
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("family", sorted(FAMILIES_3D))
def test_advance_3d_stops_at_the_failing_step(family, dtype):
    """A periodic box 20 x 16 x 12 (cold stirred, seed 7, amplitude 0.3, p = 1e-3)
    whose step 2 turns non-physical: the oracle's minimum pressure is 2.3e-4 after
    step 1 and -2.1e-5 already in step 2's stage-1 state, so step 2's output is not
    fixed by the scheme (a sound speed of a negative pressure), but both sides stop
    after step 2, at the time step 1's state fixes."""
    pr = inputs.cold_stirred_3d((20, 16, 12), seed=7, amp=0.3)
    U = as_input(pr.U, dtype)
    _, t_ref, k_ref, ok = oracle.advance(oracle_mesh(pr), U, 0.5, math.inf, max_steps=20, on_failure="return")
    assert not ok and k_ref == 2
    s = gpu_solver([spec_of(pr)], dtype, FAMILIES_3D[family][dtype == "f64"], pr.U)
    print(f"3D failure advance: {family} {dtype}", flush=True)
    with pytest.raises(pb.NonFiniteError) as ei:
        s.advance(math.inf, 0.5, max_steps=20)
    assert ei.value.steps == [k_ref]
    assert abs(ei.value.t[0] - t_ref) <= (1e-13 if dtype == "f64" else 1e-6) * t_ref
    got = gpu_state(s)
    with pytest.raises(pb.NonFiniteError) as ei2:
        s.advance(math.inf, 0.5, max_steps=20, t0=ei.value.t)
    assert ei2.value.steps == [0]
    assert np.array_equal(gpu_state(s), got, equal_nan=True)
    s.close()
