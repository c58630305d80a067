"""paraiso_cfl_dt_static, the entry point that allocates nothing, against
paraiso_cfl_dt on the same states: bit for bit, on two calls in a row whose
second has a smaller input (fewer, smaller meshes whose signal speeds are
lower, so a maximum left in the static scratch by the first call would show).
"""
import numpy as np
import pytest

from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd import inputs

pytestmark = pytest.mark.gpu


def _solver(shapes, ndim, dtype, seed, scale):
    """A context over random states (velocities scaled by `scale`) and its dt."""
    probs = [inputs.random_state(ndim, n, seed=seed + k, rough=True, bc=(0,) * ndim) for k, n in enumerate(shapes)]
    specs = [pb.MeshSpec(ndim, p.n, p.gamma, p.bc) for p in probs]
    states = []
    for p in probs:
        U = p.U.copy()
        U[1:1 + ndim] *= scale
        U[ndim + 1] += 0.5 * (scale ** 2 - 1.0) * sum(p.U[1 + a] ** 2 for a in range(ndim)) / p.U[0]
        states.append(U)
    s = pb.Solver(specs, dtype)
    s.upload(states)
    return s


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_static_cfl_equals_context_cfl_twice(dtype, ndim):
    import torch
    big = {2: [(200, 150), (97, 131), (64, 64), (300, 41), (33, 257)], 3: [(40, 36, 30), (17, 50, 23), (64, 8, 8)]}
    small = {2: [(30, 20), (17, 9)], 3: [(9, 7, 5)]}
    a = _solver(big[ndim], ndim, dtype, 900 + ndim, scale=3.0)
    b = _solver(small[ndim], ndim, dtype, 950 + ndim, scale=0.2)
    stream = torch.cuda.current_stream().cuda_stream
    for s in (a, b):
        ref = s.cfl_dt(0.5)
        print(f"case static cfl {dtype} {ndim}D meshes={len(s.meshes)}", flush=True)
        got = pb.paraiso_cfl_dt_static(s.meshes, s.current(), 0.5, stream)
        assert got == ref, (got, ref)
    # the small input's steps are longer: a stale maximum from the first call would shorten them
    assert min(b.cfl_dt(0.5)) > max(a.cfl_dt(0.5))
    # the other buffer after a step of the gentle input, then the first input again
    b.step(b.cfl_dt(0.5))
    torch.cuda.synchronize()
    assert b.current() == 1
    assert pb.paraiso_cfl_dt_static(b.meshes, b.current(), 0.5, stream) == b.cfl_dt(0.5)
    assert pb.paraiso_cfl_dt_static(a.meshes, a.current(), 0.5, stream) == a.cfl_dt(0.5)
    a.close()
    b.close()


def test_static_cfl_reports_nonphysical_state():
    import torch
    s = _solver([(40, 30)], 2, "f64", 77, scale=1.0)
    st = s.state()
    st[3, 5, 7] = -1.0  # E < 0: p < 0 in that cell
    torch.cuda.synchronize()
    with pytest.raises(pb.NonFiniteError):
        pb.paraiso_cfl_dt_static(s.meshes, s.current(), 0.5, torch.cuda.current_stream().cuda_stream)
    with pytest.raises(pb.NonFiniteError):
        s.cfl_dt(0.5)
    s.close()


def test_static_cfl_rejects_sizes_beyond_the_scratch():
    import torch
    s = _solver([(16, 16)], 2, "f32", 5, scale=1.0)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_cfl_dt_static(s.meshes * (pb.STATIC_MESHES + 1), 0, 0.5, stream)
    assert ei.value.code == pb.ERR_UNSUPPORTED
    # the full capacity is accepted and agrees with the context
    got = pb.paraiso_cfl_dt_static(s.meshes * pb.STATIC_MESHES, s.current(), 0.5, stream)
    assert got == s.cfl_dt(0.5) * pb.STATIC_MESHES
    s.close()
