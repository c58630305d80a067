"""HIP path vs the FP64 oracle, through the C ABI (paraiso_*).

One step from identical input with an explicit dt (the oracle's CFL step):
FP64 within 1e-12 and FP32 within 1e-5, normwise relative per field, for
every kernel variant, dimension and boundary condition, on meshes that span
several tiles and end in a ragged tile.
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

from gpu_util import (TOL, VARIANTS, as_input, default_tile, gpu_solver, gpu_state, oracle_mesh, rel_err,
                      spec_of)

pytestmark = pytest.mark.gpu

SHAPES = {1: (203,), 2: (37, 21), 3: (19, 11, 10)}


def _variant(name, ndim, tile=None):
    if VARIANTS[name] is None:
        return None
    v = dict(VARIANTS[name])
    v["tile"] = tile or default_tile(ndim)
    return v


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("vname", list(VARIANTS))
def test_one_step_matches_oracle(dtype, ndim, bc, vname):
    print(f"case dtype={dtype} ndim={ndim} bc={bc} variant={vname}", flush=True)
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=100 + 10 * ndim + bc, rough=(ndim != 3),
                             bc=(bc,) * 3)
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    s = gpu_solver(spec_of(pr), dtype, _variant(vname, ndim), pr.U)
    s.step(dt)
    got = gpu_state(s)
    err = rel_err(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= TOL[dtype], err
    # the step did something
    assert rel_err(ref, U0) > 1e-4


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_smooth_2d_many_tiles_and_persistent(dtype):
    pr = inputs.random_state(2, (133, 70), seed=7, bc=(0, 1))
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.4)
    ref = oracle.step(m, U0, dt)
    for v in (dict(tile=(32, 16), lds=1, fuse=1, persistent=1),
              dict(tile=(16, 16), lds=1, fuse=0, persistent=1, threads=128),
              dict(tile=(64, 8), lds=1, fuse=1, waves_per_eu=4, threads=512)):
        s = gpu_solver(spec_of(pr), dtype, v, pr.U)
        s.step(dt)
        assert rel_err(gpu_state(s), ref) <= TOL[dtype], v


@pytest.mark.parametrize("ndim,n", [(1, (1,)), (1, (3,)), (2, (5, 2)), (2, (1, 6)), (2, (6, 1)), (2, (1, 1)),
                                    (3, (3, 2, 5)), (3, (1, 1, 5)), (3, (4, 1, 1)), (3, (1, 3, 1))])
@pytest.mark.parametrize("bc", [0, 1])
def test_tiny_meshes(ndim, n, bc):
    print(f"case tiny ndim={ndim} n={n} bc={bc}", flush=True)
    pr = inputs.random_state(ndim, n, seed=3, bc=(bc,) * 3)
    m = oracle_mesh(pr)
    dt = 1e-3
    ref = oracle.step(m, pr.U, dt)
    variants = [(vname, _variant(vname, ndim)) for vname in VARIANTS]
    # the register marches beside the library's default choice: the one-stage
    # form (2D and 3D) and, on periodic meshes, the fused form
    if ndim == 2:
        variants.append(("march one-stage", dict(tile=(64, 8), lds=2, fuse=0, threads=256)))
        if bc == 0:
            variants.append(("march fused", dict(tile=(64, 8), lds=2, fuse=1, threads=256)))
    if ndim == 3:
        variants.append(("march one-stage", dict(tile=(64, 8, 16), lds=2, fuse=0)))
        if bc == 0:
            variants.append(("march fused", dict(tile=(64, 6, 16), lds=2, fuse=1)))
    for vname, v in variants:
        s = gpu_solver(spec_of(pr), "f64", v, pr.U)
        s.step(dt)
        assert rel_err(gpu_state(s), ref) <= 1e-12, vname


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_uniform_flow_bitwise(dtype, ndim):
    pr = inputs.uniform_flow(ndim, SHAPES[ndim], bc=(1, 0, 1))
    for vname in VARIANTS:
        s = gpu_solver(spec_of(pr), dtype, _variant(vname, ndim), pr.U)
        s.step(2e-3)
        np.testing.assert_array_equal(gpu_state(s), as_input(pr.U, dtype))


def test_zero_dt_is_identity():
    pr = inputs.random_state(2, (40, 30), seed=4, rough=True)
    for vname in VARIANTS:
        s = gpu_solver(spec_of(pr), "f64", _variant(vname, 2), pr.U)
        s.step(0.0)
        np.testing.assert_array_equal(gpu_state(s), pr.U)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_cfl_dt_matches_oracle(dtype, ndim):
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=17, rough=True)
    U0 = as_input(pr.U, dtype)
    want = oracle.cfl_dt(oracle_mesh(pr), U0, 0.5)
    s = gpu_solver(spec_of(pr), dtype, None, pr.U)
    got = s.cfl_dt(0.5)[0]
    assert abs(got - want) <= 1e-14 * want


def test_cfl_flags_nonphysical():
    pr = inputs.random_state(2, (30, 20), seed=5)
    bad = pr.U.copy()
    bad[0, 7, 3] = -0.5
    s = gpu_solver(spec_of(pr), "f64", None, bad)
    with pytest.raises(FloatingPointError):
        s.cfl_dt(0.5)
    bad = pr.U.copy()
    bad[3, 1, 1] = np.nan
    s = gpu_solver(spec_of(pr), "f32", None, bad)
    with pytest.raises(FloatingPointError):
        s.cfl_dt(0.5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_cfl_flags_nonpositive_pressure(dtype, ndim):
    # p < 0 (kinetic energy above the total) and p = 0 exactly (at rest, E = 0)
    # in one cell: the oracle's failure cases, which the GPU's CFL term must
    # report too (its sound speed goes through the reciprocal square root of
    # gamma rho p)
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=29)
    cell = (1,) * ndim
    for make in ("negative", "zero"):
        bad = pr.U.copy()
        if make == "negative":
            m2 = sum(bad[(1 + a,) + cell] ** 2 for a in range(ndim))
            bad[(ndim + 1,) + cell] = 0.25 * m2 / bad[(0,) + cell]
        else:
            for a in range(ndim):
                bad[(1 + a,) + cell] = 0.0
            bad[(ndim + 1,) + cell] = 0.0
        with pytest.raises(FloatingPointError):
            oracle.cfl_dt(oracle_mesh(pr), as_input(bad, dtype), 0.5)
        s = gpu_solver(spec_of(pr), dtype, None, bad)
        with pytest.raises(FloatingPointError):
            s.cfl_dt(0.5)
        s.close()


def _corrupt(U, ndim, cell, kind):
    """One non-physical cell of the given kind (rho <= 0, p <= 0 or a component
    that is not finite)."""
    E = (ndim + 1,) + cell
    if kind == "rho_zero":
        U[(0,) + cell] = 0.0
    elif kind == "rho_negzero":
        U[(0,) + cell] = -0.0
    elif kind == "rho_negative_energy_negative":  # gamma rho p > 0 although rho < 0
        U[(0,) + cell] = -1.0
        for a in range(ndim):
            U[(1 + a,) + cell] = 0.0
        U[E] = -2.0
    elif kind == "rho_inf":
        U[(0,) + cell] = np.inf
    elif kind == "energy_inf":
        U[E] = np.inf
    elif kind == "energy_neginf":
        U[E] = -np.inf
    elif kind == "momentum_inf":
        U[(1,) + cell] = np.inf
    elif kind == "momentum_nan":
        U[(ndim,) + cell] = np.nan
    else:
        raise ValueError(kind)
    return U


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("kind", ["rho_zero", "rho_negzero", "rho_negative_energy_negative", "rho_inf",
                                  "energy_inf", "energy_neginf", "momentum_inf", "momentum_nan"])
def test_cfl_flags_every_nonphysical_kind(dtype, ndim, kind):
    # the CFL term flags a cell by one class test of its quantity (anything
    # but a positive finite number); every kind the oracle reports must land
    # there, in the first cell of a block and in one inside it
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=31)
    for cell in ((0,) * ndim, tuple(min(3, n - 1) for n in reversed(SHAPES[ndim]))):
        bad = _corrupt(pr.U.copy(), ndim, cell, kind)
        with pytest.raises(FloatingPointError):
            oracle.cfl_dt(oracle_mesh(pr), as_input(bad, dtype), 0.5)
        s = gpu_solver(spec_of(pr), dtype, None, bad)
        with pytest.raises(FloatingPointError):
            s.cfl_dt(0.5)
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_totals_match_oracle(dtype, ndim):
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=23)
    U0 = as_input(pr.U, dtype)
    want = oracle.totals(oracle_mesh(pr), U0)
    s = gpu_solver(spec_of(pr), dtype, None, pr.U)
    got = np.array(s.totals()[0])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("vname", ["lds_fused", "lds", "direct"])
def test_sod_advance_matches_oracle_and_exact(vname):
    from oracle import exact_riemann as er
    pr = inputs.sod_1d(1024)
    ref, t_ref, steps_ref = oracle.advance(oracle_mesh(pr), pr.U, 0.5, 0.2)
    s = gpu_solver(spec_of(pr), "f64", _variant(vname, 1, tile=(256, 1, 1)), pr.U)
    t, steps = s.advance(0.2, 0.5)
    got = gpu_state(s)
    assert t[0] == 0.2 and steps[0] == steps_ref
    assert rel_err(got, ref) < 1e-10
    x = inputs.centres(1024)
    rho_ex = np.array([e[0] for e in er.sample_cells(1.4, er.Side(1, 0, 1), er.Side(0.125, 0, 0.1), 0.5, 0.2, x)])
    assert np.mean(np.abs(got[0] - rho_ex)) < 5e-3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_advance_graph_equals_eager_and_is_deterministic(dtype):
    pr = inputs.random_state(2, (96, 64), seed=31)
    spec = spec_of(pr)
    a = gpu_solver(spec, dtype, None, pr.U)
    ta, na = a.advance(float("inf"), 0.5, max_steps=12)   # two six-step graph replays
    b = gpu_solver(spec, dtype, None, pr.U)
    t = [0.0]
    for k in (5, 5, 2):                                    # eager launches only
        t, _ = b.advance(float("inf"), 0.5, max_steps=k, t0=t)
    c = gpu_solver(spec, dtype, None, pr.U)
    tc, _ = c.advance(float("inf"), 0.5, max_steps=12)
    assert na == [12]
    np.testing.assert_array_equal(gpu_state(a), gpu_state(c))
    assert ta == tc
    np.testing.assert_array_equal(gpu_state(a), gpu_state(b))
    assert ta == t


def test_advance_matches_oracle_steps_2d():
    pr = inputs.random_state(2, (48, 40), seed=41, bc=(1, 0))
    ref, t_ref, n_ref = oracle.advance(oracle_mesh(pr), pr.U, 0.5, 1e9, max_steps=10)
    for v in (dict(tile=(16, 8), lds=1, fuse=1), dict(tile=(16, 8), lds=1, fuse=0)):
        s = gpu_solver(spec_of(pr), "f64", v, pr.U)
        t, n = s.advance(1e9, 0.5, max_steps=10)
        assert n == [10]
        assert abs(t[0] - t_ref) <= 1e-13 * t_ref
        assert rel_err(gpu_state(s), ref) < 1e-11


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("family", ["lds_fused", "march_shared"])
def test_batch_members_equal_solo_runs(persistent, family):
    sizes = [(20, 17), (64, 64), (9, 31), (130, 70)]
    probs = [inputs.random_state(2, n, seed=60 + k) for k, n in enumerate(sizes)]
    specs = [spec_of(p) for p in probs]
    dts = [oracle.cfl_dt(oracle_mesh(p), as_input(p.U, "f32"), 0.5) for p in probs]
    v = {"lds_fused": dict(tile=(16, 8), lds=1, fuse=1, persistent=persistent),
         "march_shared": dict(tile=(64, 8), lds=2, fuse=1, threads=256, persistent=persistent)}[family]
    b = gpu_solver(specs, "f32", v, [p.U for p in probs])
    b.step(dts)
    for k, p in enumerate(probs):
        solo = gpu_solver(specs[k], "f32", v, p.U)
        solo.step(dts[k])
        np.testing.assert_array_equal(gpu_state(b, k), gpu_state(solo))
        ref = oracle.step(oracle_mesh(p), as_input(p.U, "f32"), dts[k])
        assert rel_err(gpu_state(b, k), ref) <= TOL["f32"]


def test_batch_advance_per_mesh_dt():
    probs = [inputs.blob_2d(n, 12044779, k) for k, n in enumerate((40, 72, 33))]
    specs = [spec_of(p) for p in probs]
    b = gpu_solver(specs, "f64", dict(tile=(16, 16), lds=1, fuse=1, persistent=1), [p.U for p in probs])
    t, n = b.advance(0.01, 0.5, t0=[0.0, 0.0, 0.0])
    for k, p in enumerate(probs):
        ref, t_ref, n_ref = oracle.advance(oracle_mesh(p), p.U, 0.5, 0.01)
        assert n[k] == n_ref and t[k] == t_ref
        assert rel_err(gpu_state(b, k), ref) < 1e-11


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_variant_round_trips(dtype):
    # whatever paraiso_get_variant reports, paraiso_set_variant takes back unchanged:
    # the library's defaults for every family and a few explicit choices
    P, O, A = pb.PERIODIC, pb.OUTFLOW, pb.ANALYTIC
    cases = [([pb.MeshSpec(1, (300,), 1.4, (O,))], None),                     # resident
             ([pb.MeshSpec(1, (300,), 1.4, (P,)), pb.MeshSpec(1, (70,), 1.4, (O,))], None),
             ([pb.MeshSpec(1, (5000,), 1.4, (P,))], None),                    # LDS tiles
             ([pb.MeshSpec(2, (70, 50), 1.4, (P, P))], None),                 # fused march
             ([pb.MeshSpec(2, (70, 50), 1.4, (O, P))], None),                 # LDS tiles
             ([pb.MeshSpec(2, (70, 50), 1.4, (A, P))], None),                 # one-stage march, ghosts
             ([pb.MeshSpec(2, (70, 50), 1.4, (P, P), order=1)], None),        # first order
             ([pb.MeshSpec(3, (40, 20, 10), 1.4, (P, O, P))], None),          # 3D march
             ([pb.MeshSpec(3, (40, 20, 10), 1.4, (P, P, P))], dict(tile=(64, 6, 16), lds=2, fuse=1)),
             ([pb.MeshSpec(2, (70, 50), 1.4, (P, P))], dict(tile=(32, 16), lds=1, fuse=1, manifest=2)),
             ([pb.MeshSpec(2, (70, 50), 1.4, (P, P))], dict(tile=(64, 4), lds=0, fuse=0, persistent=1))]
    for specs, v in cases:
        s = pb.Solver(specs, dtype)
        if v is not None:
            s.set_variant(v)
        else:   # init applied the library's default, not a fallback
            dv = pb.paraiso_default_variant(s.meshes).as_dict()
            assert {k: s.variant()[k] for k in dv if k != "threads"} == \
                {k: dv[k] for k in dv if k != "threads"}, (specs, dv, s.variant())
        got = s.variant()
        s.set_variant(got)
        assert s.variant() == got, (specs, got, s.variant())
        s.close()


def test_set_variant_rejects_oversized_lds():
    pr = inputs.random_state(3, (16, 16, 16), seed=1)
    s = gpu_solver(spec_of(pr), "f64", None, pr.U)
    with pytest.raises(pb.ParaisoError) as ei:
        s.set_variant(dict(tile=(64, 64, 64), lds=1, fuse=1))
    assert ei.value.code == pb.ERR_UNSUPPORTED
    # the previous variant is still in place and works
    s.step(1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("n", [(200, 77), (37, 21), (64, 64), (5, 9), (130, 3)])
def test_register_march_matches_oracle(dtype, fuse, n):
    pr = inputs.random_state(2, n, seed=300 + n[0], rough=True)
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    # rows per wave: a steady state shorter than, equal to and longer than
    # the six-push unrolled group, with and without a remainder
    for rows, threads in ((8, 256), (16, 64), (64, 128), (6, 192), (25, 256)):
        v = dict(tile=(64, rows), lds=2, fuse=fuse, threads=threads)
        s = gpu_solver(spec_of(pr), dtype, v, pr.U)
        s.step(dt)
        err = rel_err(gpu_state(s), ref)
        assert err <= TOL[dtype], (v, err)


def test_register_march_advance_and_batch():
    probs = [inputs.blob_2d(n, 12044779, k) for k, n in enumerate((40, 72, 33, 130))]
    specs = [spec_of(p) for p in probs]
    v = dict(tile=(64, 16), lds=2, fuse=1, persistent=1)
    b = gpu_solver(specs, "f64", v, [p.U for p in probs])
    t, n = b.advance(0.01, 0.5, t0=[0.0] * 4)
    for k, p in enumerate(probs):
        ref, t_ref, n_ref = oracle.advance(oracle_mesh(p), p.U, 0.5, 0.01)
        assert n[k] == n_ref and t[k] == t_ref
        assert rel_err(gpu_state(b, k), ref) < 1e-11


def test_register_march_rejects_unsupported():
    pr = inputs.random_state(2, (40, 30), seed=1, bc=(1, 0))
    s = gpu_solver(spec_of(pr), "f32", None, pr.U)
    with pytest.raises(pb.ParaisoError):
        s.set_variant(dict(tile=(64, 16), lds=2, fuse=1))      # fused march needs periodic
    pr3 = inputs.random_state(3, (8, 8, 8), seed=1)
    s3 = gpu_solver(spec_of(pr3), "f32", None, pr3.U)
    with pytest.raises(pb.ParaisoError):
        s3.set_variant(dict(tile=(64, 4, 16), lds=2, fuse=1))  # fused 3D march: 6..12 stage-1 rows
    with pytest.raises(pb.ParaisoError):
        s3.set_variant(dict(tile=(64, 14, 16), lds=2, fuse=1))
    with pytest.raises(pb.ParaisoError):
        s3.set_variant(dict(tile=(64, 2, 16), lds=2, fuse=0))  # 4 or 8 rows per block
    s3.set_variant(dict(tile=(64, 12, 16), lds=2, fuse=1))
    s3.set_variant(dict(tile=(64, 12, 16), lds=2, fuse=1, threads=768))  # the tuner names the threads
    with pytest.raises(pb.ParaisoError):
        s3.set_variant(dict(tile=(64, 12, 16), lds=2, fuse=1, threads=512))
    s3d = gpu_solver(spec_of(pr3), "f64", None, pr3.U)
    with pytest.raises(pb.ParaisoError):
        s3d.set_variant(dict(tile=(64, 8, 16), lds=2, fuse=1))  # FP64: the LDS holds 6 rows
    s3d.set_variant(dict(tile=(64, 6, 16), lds=2, fuse=1))
    pr3o = inputs.random_state(3, (8, 8, 8), seed=1, bc=(0, 1, 0))
    s3o = gpu_solver(spec_of(pr3o), "f32", None, pr3o.U)
    with pytest.raises(pb.ParaisoError):
        s3o.set_variant(dict(tile=(64, 8, 16), lds=2, fuse=1))  # fused 3D march needs periodic
    pr1 = inputs.random_state(1, (100,), seed=1)
    s1 = gpu_solver(spec_of(pr1), "f32", None, pr1.U)
    with pytest.raises(pb.ParaisoError):
        s1.set_variant(dict(tile=(64,), lds=2, fuse=0))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n", [(19, 11, 10), (70, 9, 7), (130, 20, 5), (5, 4, 3)])
def test_register_march_3d_matches_oracle(dtype, bc, n):
    pr = inputs.random_state(3, n, seed=400 + n[0] + bc, rough=True, bc=(bc,) * 3)
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    for rows, planes in ((4, 8), (8, 32), (4, 64)):
        v = dict(tile=(64, rows, planes), lds=2, fuse=0)
        s = gpu_solver(spec_of(pr), dtype, v, pr.U)
        s.step(dt)
        err = rel_err(gpu_state(s), ref)
        assert err <= TOL[dtype], (v, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(19, 11, 10), (70, 9, 7), (130, 20, 5), (5, 4, 3), (60, 26, 70), (120, 7, 2)])
def test_register_march_3d_fused_matches_oracle(dtype, n):
    # the fused 3D march: stage-1 rows 6..12 (FP64: 6, its LDS limit), plane
    # chunks of 1, 3, 16 and 64 planes (chunk seams inside the mesh and a
    # chunk longer than the mesh), meshes narrower and wider than a strip
    pr = inputs.random_state(3, n, seed=500 + n[0] + n[2], rough=True)
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    shapes = ((6, 16), (6, 1), (6, 64)) if dtype == "f64" else ((8, 16), (12, 3), (6, 64), (10, 1), (12, 64))
    for rows, planes in shapes:
        v = dict(tile=(64, rows, planes), lds=2, fuse=1)
        print(f"case fused 3D march {dtype} {n} {v}", flush=True)
        s = gpu_solver(spec_of(pr), dtype, v, pr.U)
        got_dt = s.cfl_dt(0.5)[0]
        assert abs(got_dt - dt) <= 1e-14 * dt
        s.step(dt)
        err = rel_err(gpu_state(s), ref)
        assert err <= TOL[dtype], (v, err)
        s.close()


def test_register_march_3d_fused_advance_matches_oracle():
    # device-resident dt through the six-step graphs, FP64 and FP32
    pr = inputs.random_state(3, (40, 24, 20), seed=78)
    ref, t_ref, n_ref = oracle.advance(oracle_mesh(pr), pr.U, 0.5, 1e9, max_steps=8)
    for dtype, rows in (("f64", 6), ("f32", 12)):
        s = gpu_solver(spec_of(pr), dtype, dict(tile=(64, rows, 16), lds=2, fuse=1), pr.U)
        t, n = s.advance(1e9, 0.5, max_steps=8)
        tol_t = 1e-13 if dtype == "f64" else 1e-6
        assert n == [8] and abs(t[0] - t_ref) <= tol_t * t_ref
        ref_in = oracle.advance(oracle_mesh(pr), as_input(pr.U, dtype), 0.5, 1e9, max_steps=8)[0]
        assert rel_err(gpu_state(s), ref_in) < (1e-11 if dtype == "f64" else 1e-4)
        s.close()


def test_register_march_2d_unfused_outflow():
    pr = inputs.random_state(2, (90, 41), seed=8, rough=True, bc=(1, 1))
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, pr.U, 0.5)
    ref = oracle.step(m, pr.U, dt)
    s = gpu_solver(spec_of(pr), "f64", dict(tile=(64, 16), lds=2, fuse=0), pr.U)
    s.step(dt)
    assert rel_err(gpu_state(s), ref) <= 1e-12


def test_register_march_3d_advance_matches_oracle():
    pr = inputs.random_state(3, (40, 24, 20), seed=77)
    ref, t_ref, n_ref = oracle.advance(oracle_mesh(pr), pr.U, 0.5, 1e9, max_steps=8)
    s = gpu_solver(spec_of(pr), "f64", dict(tile=(64, 8, 16), lds=2, fuse=0), pr.U)
    t, n = s.advance(1e9, 0.5, max_steps=8)
    assert n == [8] and abs(t[0] - t_ref) <= 1e-13 * t_ref
    assert rel_err(gpu_state(s), ref) < 1e-11


@pytest.mark.parametrize("vname", ["march2d", "lds_fused", "lds"])
def test_graph_replays_interleaved_with_eager_work(vname):
    # Each advance(6) replays one captured six-step graph; between replays run eager
    # explicit steps, reductions and host reads.  Every replay must equal the same
    # steps launched eagerly (advance with 5 + 1 steps never forms a graph).
    pr = inputs.random_state(2, (128, 70), seed=91)
    v = {"march2d": dict(tile=(64, 16), lds=2, fuse=1), "lds_fused": dict(tile=(32, 16), lds=1, fuse=1),
         "lds": dict(tile=(32, 16), lds=1, fuse=0)}[vname]
    g = gpu_solver(spec_of(pr), "f64", v, pr.U)
    e = gpu_solver(spec_of(pr), "f64", v, pr.U)
    tg, te = [0.0], [0.0]
    for rep in range(4):
        tg, ng = g.advance(float("inf"), 0.5, max_steps=6, t0=tg)
        for k in (5, 1):
            te, _ = e.advance(float("inf"), 0.5, max_steps=k, t0=te)
        assert ng == [6] and tg == te, rep
        np.testing.assert_array_equal(gpu_state(g), gpu_state(e))
        # eager work between replays on both contexts
        dt = g.cfl_dt(0.4)[0]
        assert dt == e.cfl_dt(0.4)[0]
        g.step(dt)
        e.step(dt)
        assert g.totals() == e.totals()


# the largest mesh the resident kernel holds: 4096 cells in FP32; in FP64 the
# primitive and flux planes (8 * (6n + 3) bytes) cap it at 3407 cells of 160 KiB LDS
RESIDENT_MAX = {"f32": 4096, "f64": 3407}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n", [1, 3, 203, 1024, 2048, 2049, "max"])
def test_resident_1d_step_matches_oracle(dtype, bc, n):
    n = RESIDENT_MAX[dtype] if n == "max" else n
    pr = inputs.random_state(1, (n,), seed=500 + n + bc, rough=True, bc=(bc,))
    U0 = as_input(pr.U, dtype)
    m = oracle_mesh(pr)
    dt = oracle.cfl_dt(m, U0, 0.5)
    ref = oracle.step(m, U0, dt)
    s = gpu_solver(spec_of(pr), dtype, dict(tile=(n,), lds=3, fuse=1), pr.U)
    # the workgroup follows the mesh: 512 threads up to 2048 cells, else 1024
    assert s.variant()["threads"] == (512 if n <= 2048 else 1024)
    s.step(dt)
    assert rel_err(gpu_state(s), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 203, 1024, 2048])
def test_resident_1d_workgroup_sizes_agree(dtype, n):
    # 512 and 1024 threads hold the same cells in different places: one
    # advance of 20 device-dt steps gives the same bits and the same time
    print(f"case resident workgroups {dtype} n={n}", flush=True)
    pr = inputs.random_state(1, (n,), seed=900 + n, bc=(1,))
    out = []
    for threads in (512, 1024):
        s = gpu_solver(spec_of(pr), dtype, dict(tile=(n,), lds=3, fuse=1, threads=threads), pr.U)
        assert s.variant()["threads"] == threads
        t, k = s.advance(1e9, 0.5, max_steps=20)
        out.append((gpu_state(s), t, k))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    assert out[0][1:] == out[1][1:] and out[0][2] == [20]


def test_resident_1d_sod_advance_and_batch():
    from oracle import exact_riemann as er
    pr = inputs.sod_1d(1024)
    ref, t_ref, steps_ref = oracle.advance(oracle_mesh(pr), pr.U, 0.5, 0.2)
    s = gpu_solver(spec_of(pr), "f64", dict(tile=(1024,), lds=3, fuse=1), pr.U)
    t, steps = s.advance(0.2, 0.5)
    assert t[0] == 0.2 and steps[0] == steps_ref
    assert rel_err(gpu_state(s), ref) < 1e-10
    # a batch of 1D meshes, one block each, different step counts
    probs = [inputs.sod_1d(n) for n in (256, 1000, 64)]
    b = gpu_solver([spec_of(p) for p in probs], "f64", dict(tile=(1024,), lds=3, fuse=1), [p.U for p in probs])
    tb, nb = b.advance(0.1, 0.5, t0=[0.0] * 3)
    for k, p in enumerate(probs):
        r, tr, nr = oracle.advance(oracle_mesh(p), p.U, 0.5, 0.1)
        assert nb[k] == nr and tb[k] == tr
        assert rel_err(gpu_state(b, k), r) < 1e-10
    # switching to a queue-driven persistent variant afterwards still covers every tile
    b.set_variant(dict(tile=(64,), lds=1, fuse=1, persistent=1))
    dts = [1e-4] * 3
    refs = [oracle.step(oracle_mesh(p), gpu_state(b, k), 1e-4) for k, p in enumerate(probs)]
    b.step(dts)
    for k in range(3):
        assert rel_err(gpu_state(b, k), refs[k]) < 1e-12


def test_resident_1d_rejects_large_and_2d():
    pr = inputs.random_state(1, (5000,), seed=1)
    s = gpu_solver(spec_of(pr), "f64", None, pr.U)
    with pytest.raises(pb.ParaisoError):
        s.set_variant(dict(tile=(5000,), lds=3, fuse=1))
    # one cell past the FP64 LDS limit
    pr1 = inputs.random_state(1, (RESIDENT_MAX["f64"] + 1,), seed=1)
    s1 = gpu_solver(spec_of(pr1), "f64", None, pr1.U)
    with pytest.raises(pb.ParaisoError):
        s1.set_variant(dict(tile=(RESIDENT_MAX["f64"] + 1,), lds=3, fuse=1))
    pr2 = inputs.random_state(2, (16, 16), seed=1)
    s2 = gpu_solver(spec_of(pr2), "f64", None, pr2.U)
    with pytest.raises(pb.ParaisoError):
        s2.set_variant(dict(tile=(16, 16), lds=3, fuse=1))
    # 512 threads hold at most 2048 cells; other workgroup sizes do not exist
    pr3 = inputs.random_state(1, (2049,), seed=1)
    s3 = gpu_solver(spec_of(pr3), "f64", None, pr3.U)
    with pytest.raises(pb.ParaisoError):
        s3.set_variant(dict(tile=(2049,), lds=3, fuse=1, threads=512))
    s3.set_variant(dict(tile=(2049,), lds=3, fuse=1, threads=1024))
    for bad in (256, 768):
        with pytest.raises(pb.ParaisoError):
            s3.set_variant(dict(tile=(2049,), lds=3, fuse=1, threads=bad))
