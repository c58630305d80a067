"""Analytic boundaries on the GPU: the convergence-test problems of section
"Tuning Experiments / Automated Tuning" (entropy wave, sound wave, Sod's
shock tube; coaxial and rotated by 60 degrees) with the exact solution in
the ghost cells, against the FP64 oracle.

One step from the oracle's exact state at t0 > 0 with an explicit dt: FP64
within 1e-12 and FP32 within 1e-5.  Density and energy are held pointwise
(every cell against its own value) and normwise.  In FP64 the momenta are
held against their own maximum too (a component that is zero in exact
arithmetic, such as the transverse momentum of a coaxial wave, holds only
rounding and is measured against max rho (|v| + c)), except the sound
wave's: its momentum is
of the order of the amplitude (1e-5) while its flux carries the O(1)
pressure, so the rounding of that pressure term, not the scheme, sets its
own-scale error; it is held, as every FP32 momentum is, against
max rho (|v| + c).  Meshes span several tiles and end in a ragged tile, so
interior tiles, edge tiles and corners all read ghosts.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb

from gpu_util import TOL, as_input, gpu_state, measures, state_err, strict_err

pytestmark = pytest.mark.gpu

A = pb.ANALYTIC
KINDS = {"entropy": pb.ENTROPY_WAVE, "sound": pb.SOUND_WAVE, "sod": pb.SHOCK_TUBE}
OBLIQUE = math.pi / 3
# the one-stage register march, ghost cells from the ghost arrays
MARCH = dict(tile=(64, 8), lds=2, fuse=0, threads=256)


def _err(got, ref, kind, dtype):
    """The bar's measure for this problem and precision (see the module docstring)."""
    if dtype == "f64" and kind != "sound":
        return strict_err(got, ref, 1.4)
    return state_err(got, ref, 1.4)


def _problem(kind, angle):
    return oracle.Analytic(KINDS[kind], angle, 1e-5)


def _solver(ndim, n, bc, dtype, an, variant=None):
    s = pb.Solver(pb.MeshSpec(ndim, n, 1.4, bc), dtype)
    s.set_analytic(an.kind, an.angle, an.amplitude)
    if variant is not None:
        s.set_variant(variant)
    return s


def _one_step(ndim, n, bc, dtype, an, t0, variant=None, nsteps=1):
    m = oracle.Mesh(ndim, n, 1.4, bc)
    U0 = as_input(oracle.exact_state(m, an, t0), dtype)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref, t = U0, t0
    for _ in range(nsteps):
        ref = oracle.step(m, ref, dt, t, an)
        t += dt
    s = _solver(ndim, n, bc, dtype, an, variant)
    s.upload(U0)
    s.set_time(t0)
    for _ in range(nsteps):
        s.step(dt)
    got = gpu_state(s)
    tg = s.time()[0]
    s.close()
    return got, ref, tg, t


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["entropy", "sound", "sod"])
@pytest.mark.parametrize("angle", [0.0, OBLIQUE])
def test_one_step_2d_matches_oracle(dtype, kind, angle):
    an = _problem(kind, angle)
    for variant in (None, dict(tile=(16, 8), lds=1, fuse=0, persistent=1), MARCH, dict(MARCH, tile=(64, 4))):
        got, ref, _, _ = _one_step(2, (37, 29), (A, A), dtype, an, 0.07, variant)
        err = _err(got, ref, kind, dtype)
        print(f"  {kind} angle {angle:.3f} {dtype} {variant}: {err:.3e} {measures(got, ref, 1.4)}", flush=True)
        assert err <= TOL[dtype], (variant, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["entropy", "sound", "sod"])
def test_one_step_1d_and_3d_match_oracle(dtype, kind):
    got, ref, _, _ = _one_step(1, (203,), (A,), dtype, _problem(kind, 0.0), 0.05,
                               dict(tile=(64, 1, 1), lds=1, fuse=0))
    print(f"  1D {kind} {dtype}: {measures(got, ref, 1.4)}", flush=True)
    assert _err(got, ref, kind, dtype) <= TOL[dtype]
    # 3D: the problem lives in the x-y plane; z periodic (the solution is z-independent)
    got, ref, _, _ = _one_step(3, (19, 11, 6), (A, A, pb.PERIODIC), dtype, _problem(kind, OBLIQUE), 0.05)
    print(f"  3D {kind} {dtype}: {measures(got, ref, 1.4)}", flush=True)
    assert _err(got, ref, kind, dtype) <= TOL[dtype]


def test_analytic_axis_mixes_with_periodic_and_outflow():
    # coaxial waves do not depend on y: the y axis may be periodic or outflow
    for bc in ((A, pb.PERIODIC), (A, pb.OUTFLOW), (pb.PERIODIC, A)):
        an = _problem("entropy", 0.0 if bc[0] == A else math.pi / 2)
        for variant in (None, MARCH):
            got, ref, _, _ = _one_step(2, (33, 18), bc, "f64", an, 0.11, variant)
            assert strict_err(got, ref, 1.4) <= 1e-12, (bc, variant)


def test_explicit_steps_carry_the_time():
    # three explicit steps: ghosts at t0 + k dt (and + dt/2 in stage 2); the
    # device time is the same sum of doubles as on the host
    for variant in (None, MARCH):
        got, ref, tg, t = _one_step(2, (40, 24), (A, A), "f64", _problem("sod", OBLIQUE), 0.02, variant, nsteps=3)
        assert tg == t
        assert strict_err(got, ref, 1.4) <= 1e-12


def test_time_survives_cfl_and_variant_changes():
    an = _problem("entropy", OBLIQUE)
    s = _solver(2, (24, 24), (A, A), "f64", an)
    s.fill_exact(0.0)
    assert s.time() == [0.0]
    s.set_time(0.25)
    dt = s.cfl_dt(0.5)[0]
    s.set_variant(dict(tile=(8, 8), lds=1, fuse=0))
    assert s.time() == [0.25]
    s.step(dt)
    assert s.time() == [0.25 + dt]
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_exact_state_fill_matches_oracle(dtype, ndim):
    n = {1: (131,), 2: (45, 38), 3: (13, 9, 5)}[ndim]
    bc = (A,) * ndim
    for kind in KINDS:
        for t in (0.0, 0.1):
            an = _problem(kind, OBLIQUE if ndim > 1 else 0.0)
            m = oracle.Mesh(ndim, n, 1.4, bc)
            ref = oracle.exact_state(m, an, t)
            s = _solver(ndim, n, bc, dtype, an)
            s.fill_exact(t)
            got = gpu_state(s)
            s.close()
            tol = 1e-14 if dtype == "f64" else 2e-7
            assert state_err(got, ref, 1.4) <= tol, (kind, t)


def test_advance_matches_oracle():
    for kind, angle, t_end in (("entropy", OBLIQUE, 0.05), ("sod", 0.0, 0.04), ("sound", OBLIQUE, 0.05)):
        an = _problem(kind, angle)
        m = oracle.Mesh(2, (40, 36), 1.4, (A, A))
        U0 = oracle.exact_state(m, an, 0.0)
        ref, t_ref, n_ref = oracle.advance(m, U0, 0.5, t_end, analytic=an)
        for variant in (None, MARCH):
            s = _solver(2, (40, 36), (A, A), "f64", an, variant)
            s.upload(U0)
            t, n = s.advance(t_end, 0.5)
            got = gpu_state(s)
            s.close()
            assert t == [t_end] and n == [n_ref], (kind, variant)
            print(f"  advance {kind} {variant}: {measures(got, ref, 1.4)}", flush=True)
            assert _err(got, ref, kind, "f64") < 1e-11, (kind, variant)


def _l1_gpu(kind, angle, n, t_end, dtype="f64", variant=None):
    an = _problem(kind, angle)
    s = _solver(2, (n, n), (A, A), dtype, an, variant)
    s.fill_exact(0.0)
    t, _ = s.advance(t_end, 0.5)
    assert t == [t_end]
    rho = gpu_state(s)[0]
    s.fill_exact(t_end)
    exact = gpu_state(s)[0]
    s.close()
    return float(np.mean(np.abs(rho - exact)))


@pytest.mark.parametrize("kind,angle", [("entropy", 0.0), ("entropy", OBLIQUE), ("sound", 0.0),
                                        ("sound", OBLIQUE), ("sod", 0.0), ("sod", OBLIQUE)])
def test_convergence_study(kind, angle):
    # the convergence tests on the unit square (to t = 1 for the waves and
    # t = 0.125 for the tube): the GPU's L1 density error equals the oracle's
    # at N = 32 and falls at second order for the smooth waves (minmod clips
    # their extrema, so slightly less) and at about first order for the tube
    t_end = 0.125 if kind == "sod" else 1.0
    an = _problem(kind, angle)
    m = oracle.Mesh(2, (32, 32), 1.4, (A, A))
    U, t, _ = oracle.advance(m, oracle.exact_state(m, an, 0.0), 0.5, t_end, analytic=an)
    want = float(np.mean(np.abs(U[0] - oracle.exact_state(m, an, t_end)[0])))
    sizes = (32, 64, 128, 256)
    errs = [_l1_gpu(kind, angle, n, t_end) for n in sizes]
    assert abs(errs[0] - want) <= 1e-8 * want, (errs[0], want)
    march = _l1_gpu(kind, angle, 32, t_end, variant=MARCH)
    assert abs(march - want) <= 1e-8 * want, (march, want)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"  {kind} angle {angle:.3f}: L1 {errs} orders {orders}", flush=True)
    lo = 0.7 if kind == "sod" else 1.6
    assert all(o > lo for o in orders), (errs, orders)


def test_analytic_errors():
    an = _problem("entropy", 0.0)
    s = pb.Solver(pb.MeshSpec(2, (16, 16), 1.4, (A, pb.PERIODIC)), "f64")
    with pytest.raises(pb.ParaisoError) as ei:       # stepping before the problem is set
        s.step(1e-3)
    assert ei.value.code == pb.ERR_INVALID_ARG
    with pytest.raises(pb.ParaisoError) as ei:
        s.advance(0.1, 0.5)
    assert ei.value.code == pb.ERR_INVALID_ARG
    with pytest.raises(pb.ParaisoError):
        s.fill_exact(0.0)
    for bad in (dict(kind=0), dict(kind=4), dict(kind=pb.SOUND_WAVE, amplitude=1.5),
                dict(kind=pb.SOUND_WAVE, amplitude=float("nan")), dict(kind=1, angle=float("inf"))):
        with pytest.raises(pb.ParaisoError) as ei:
            s.set_analytic(**bad)
        assert ei.value.code == pb.ERR_INVALID_ARG, bad
    with pytest.raises(pb.ParaisoError) as ei:
        s.set_analytic(an.kind, mesh=1)
    assert ei.value.code == pb.ERR_INVALID_ARG
    s.set_analytic(an.kind)
    assert s.variant()["lds"] == 2 and s.variant()["fuse"] == 0     # the one-stage march
    for v in (dict(tile=(16, 8), lds=1, fuse=1), dict(tile=(64, 8), lds=2, fuse=1),
              dict(tile=(16, 8), lds=0, fuse=0)):
        with pytest.raises(pb.ParaisoError) as ei:
            s.set_variant(v)
        assert ei.value.code == pb.ERR_UNSUPPORTED, v
    with pytest.raises(pb.ParaisoError) as ei:
        s.set_time(float("nan"))
    assert ei.value.code == pb.ERR_INVALID_ARG
    s.close()
    # a mesh without an analytic axis takes no problem; 1D takes no angle
    p = pb.Solver(pb.MeshSpec(2, (16, 16), 1.4, (pb.PERIODIC, pb.OUTFLOW)), "f64")
    with pytest.raises(pb.ParaisoError) as ei:
        p.set_analytic(pb.ENTROPY_WAVE)
    assert ei.value.code == pb.ERR_INVALID_ARG
    p.close()
    q = pb.Solver(pb.MeshSpec(1, (64,), 1.4, (A,)), "f64")
    with pytest.raises(pb.ParaisoError) as ei:
        q.set_analytic(pb.ENTROPY_WAVE, angle=0.5)
    assert ei.value.code == pb.ERR_INVALID_ARG
    q.close()


@pytest.mark.parametrize("variant", [dict(MARCH, persistent=1), dict(tile=(16, 8), lds=1, fuse=0, persistent=1)])
def test_batch_of_analytic_problems_equals_solo_runs(variant):
    # uneven meshes, each with its own problem, in one persistent launch per stage
    probs = [("entropy", OBLIQUE, (40, 36)), ("sod", 0.0, (64, 20)), ("sound", OBLIQUE, (33, 47))]
    specs = [pb.MeshSpec(2, n, 1.4, (A, A)) for _, _, n in probs]
    b = pb.Solver(specs, "f64")
    for k, (kind, angle, _) in enumerate(probs):
        an = _problem(kind, angle)
        b.set_analytic(an.kind, an.angle, an.amplitude, mesh=k)
        b.fill_exact(0.0, mesh=k)
    b.set_variant(variant)
    t, n = b.advance(0.03, 0.5, t0=[0.0] * 3)
    assert t == [0.03] * 3
    for k, (kind, angle, size) in enumerate(probs):
        an = _problem(kind, angle)
        s = _solver(2, size, (A, A), "f64", an, dict(variant, persistent=0))
        s.fill_exact(0.0)
        ts, ns = s.advance(0.03, 0.5)
        assert ns[0] == n[k]
        np.testing.assert_array_equal(gpu_state(b, k), gpu_state(s))
        s.close()
    b.close()
