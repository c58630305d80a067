"""The LDS-tile kernels' Manifest choices against the default one and the oracle.

The paper's hand-annotated individuals differ in whether the results of the
interpolation (face states) and of the Riemann solver (face fluxes) are
stored and reused or recomputed where used.  Here an LDS tile keeps face
fluxes (manifest 0, the default), face states with each cell solving both
its faces (1), or both (2).  Storing and reloading a value does not change
it and the recomputed fluxes repeat the same arithmetic, so the three differ
only where the compiler contracts a product and a sum into one FMA in one
inlined copy of the flux and not in another (a few ulp); each is held to
the oracle bar and to the others within 1e-13 (FP64) / 2e-6 (FP32).
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

from gpu_util import TOL, as_input, gpu_solver, gpu_state, oracle_mesh, rel_err, spec_of

pytestmark = pytest.mark.gpu

SHAPES = {1: (203,), 2: (37, 21), 3: (19, 11, 10)}
AGREE = {"f64": 1e-13, "f32": 2e-6}
TILES = {1: (64, 1, 1), 2: (16, 8, 1), 3: (8, 4, 4)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("fuse", [0, 1])
def test_manifest_choices_agree(dtype, ndim, bc, fuse):
    pr = inputs.random_state(ndim, SHAPES[ndim], seed=400 + 10 * ndim + bc, rough=True, bc=(bc,) * ndim)
    U0 = as_input(pr.U, dtype)
    dt = oracle.cfl_dt(oracle_mesh(pr), U0, 0.5)
    ref = oracle.step(oracle_mesh(pr), U0, dt)
    out = {}
    for mf in (0, 1, 2):
        # kept face values triple the LDS region: a 3D fused FP64 tile must stay small
        tile = (2, 2, 2) if (ndim == 3 and fuse) else TILES[ndim]
        s = gpu_solver(spec_of(pr), dtype, dict(tile=tile, lds=1, fuse=fuse, manifest=mf), U0)
        assert s.variant()["manifest"] == mf
        s.step(dt)
        out[mf] = gpu_state(s)
        s.close()
        assert rel_err(out[mf], ref) <= TOL[dtype], mf
    assert rel_err(out[1], out[0]) <= AGREE[dtype]
    assert rel_err(out[2], out[0]) <= AGREE[dtype]


def test_manifest_advance_graphs_and_batch():
    probs = [inputs.blob_2d(n, 12044779, k) for k, n in enumerate((40, 72, 33))]
    specs = [spec_of(p) for p in probs]
    states = {}
    for mf in (0, 1, 2):
        b = gpu_solver(specs, "f32", dict(tile=(32, 16), lds=1, fuse=1, persistent=1, manifest=mf),
                       [p.U for p in probs])
        t, n = b.advance(float("inf"), 0.5, max_steps=13, t0=[0.0] * 3)
        states[mf] = [gpu_state(b, k) for k in range(3)]
        b.close()
    for k in range(3):
        # 13 steps compound the few-ulp differences of one step
        assert rel_err(states[1][k], states[0][k]) <= 5e-5
        assert rel_err(states[2][k], states[0][k]) <= 5e-5
        assert rel_err(states[0][k], oracle.advance(oracle_mesh(probs[k]), as_input(probs[k].U, "f32"),
                                                    0.5, float("inf"), max_steps=13)[0]) <= 5e-5


def test_manifest_rejections():
    pr = inputs.random_state(2, (32, 32), seed=401)
    s = gpu_solver(spec_of(pr), "f32", None, pr.U)
    for v in (dict(tile=(16, 8), lds=1, fuse=1, manifest=3), dict(tile=(16, 8), lds=1, fuse=1, manifest=-1),
              dict(tile=(64, 8), lds=2, fuse=1, manifest=1), dict(tile=(16, 8), lds=0, fuse=0, manifest=2)):
        with pytest.raises(pb.ParaisoError) as ei:
            s.set_variant(v)
        assert ei.value.code == pb.ERR_UNSUPPORTED, v
    s.close()
    a = pb.Solver(pb.MeshSpec(2, (32, 32), 1.4, (pb.ANALYTIC, pb.ANALYTIC)), "f32")
    with pytest.raises(pb.ParaisoError) as ei:
        a.set_variant(dict(tile=(16, 8), lds=1, fuse=0, manifest=1))
    assert ei.value.code == pb.ERR_UNSUPPORTED
    a.close()
    f = pb.Solver(pb.MeshSpec(2, (32, 32), 1.4, (0, 0), order=1), "f32")
    with pytest.raises(pb.ParaisoError) as ei:
        f.set_variant(dict(tile=(16, 8), lds=1, fuse=1, manifest=2))
    assert ei.value.code == pb.ERR_UNSUPPORTED
    f.close()
