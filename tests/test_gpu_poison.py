"""No kernel reads workspace it has not written: every kernel family runs
on a workspace filled with 0xFF bytes (NaN in FP32 and FP64) and on a
zero-filled one, and the states after explicit steps and after a
graph-replayed advance must agree bitwise."""
import math

import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

from gpu_util import gpu_state

pytestmark = pytest.mark.gpu

CASES = [
    # (ndim, n, bc, variant)
    (1, (203,), (1,), dict(tile=(64, 1, 1), lds=0, fuse=0)),
    (1, (203,), (0,), dict(tile=(64, 1, 1), lds=0, fuse=1)),
    (1, (500,), (1,), None),                                            # resident
    (2, (70, 45), (0, 1), dict(tile=(16, 8), lds=1, fuse=0)),
    (2, (70, 45), (0, 0), dict(tile=(16, 8), lds=1, fuse=1)),
    (2, (70, 45), (0, 0), dict(tile=(16, 8), lds=1, fuse=1, manifest=2)),
    (2, (70, 45), (1, 0), dict(tile=(16, 8), lds=1, fuse=0, manifest=1)),
    (2, (130, 90), (0, 0), dict(tile=(64, 8), lds=2, fuse=1, threads=256)),
    (2, (130, 90), (1, 1), dict(tile=(64, 8), lds=2, fuse=0, threads=256)),
    (3, (40, 20, 24), (0, 0, 0), dict(tile=(64, 4, 16), lds=2, fuse=0)),
    (3, (70, 20, 24), (0, 0, 0), dict(tile=(64, 6, 16), lds=2, fuse=1)),
    (3, (19, 11, 10), (1, 0, 0), dict(tile=(8, 4, 4), lds=1, fuse=1)),
]


def _run(pr, dtype, variant, fill, order=2, analytic=None):
    s = pb.Solver(pb.MeshSpec(pr.ndim, pr.n, pr.gamma, pr.bc, order=order), dtype, workspace_fill=fill)
    if analytic is not None:
        s.set_analytic(*analytic)
    if variant is not None:
        s.set_variant(variant)
    s.upload(pr.U)
    dt = s.cfl_dt(0.5)[0]
    s.step(dt)
    s.step(dt)
    a = gpu_state(s).copy()
    t, n = s.advance(float("inf"), 0.5, max_steps=13, t0=[0.1])
    b = gpu_state(s).copy()
    tot = s.totals()
    s.close()
    return a, b, t, tot


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_poisoned_workspace_changes_nothing(case, dtype):
    ndim, n, bc, variant = CASES[case]
    pr = inputs.random_state(ndim, n, seed=700 + case, rough=False, bc=bc)
    clean = _run(pr, dtype, variant, 0)
    dirty = _run(pr, dtype, variant, 0xFF)
    for x, y in zip(clean[:2], dirty[:2]):
        assert np.all(np.isfinite(y))
        np.testing.assert_array_equal(x, y)
    assert clean[2] == dirty[2] and clean[3] == dirty[3]


@pytest.mark.parametrize("variant", [None, dict(tile=(16, 8), lds=1, fuse=0)])
def test_poisoned_workspace_analytic_and_first_order(variant):
    an = oracle.Analytic(oracle.SHOCK_TUBE, math.pi / 3)
    m = oracle.Mesh(2, (70, 45), 1.4, (2, 2))
    U = oracle.exact_state(m, an, 0.0)
    pr = inputs.Problem("sod_oblique", 2, (70, 45, 1), 1.4, (2, 2), U)
    for order in (2, 1):
        v = variant if order == 2 else dict(tile=(16, 8), lds=1, fuse=0)
        clean = _run(pr, "f64", v, 0, order, (an.kind, an.angle))
        dirty = _run(pr, "f64", v, 0xFF, order, (an.kind, an.angle))
        for x, y in zip(clean[:2], dirty[:2]):
            np.testing.assert_array_equal(x, y)
