"""Meshes at the size limits, through the C ABI: a mesh holds fewer than 2^31
cells, and the register marches address a row (2D) or a z-plane (3D) with
32-bit byte offsets, so a row or plane stays under 4 GiB.

Each case fills a seeded rough state on the device (density and pressure in
[0.5, 2], velocities in [-1.5, 1.5]) with one planted high-pressure cell
(p = 100 at rest, rho = 1) near the mesh's last cell, so the CFL maximum is
known to lie in a window the oracle can evaluate. It then checks:
  * the conserved totals: equal to FP64 sums of the fields taken by torch;
  * dt: the library's CFL step equals the oracle's on that window (the
    planted cell's q = d c = d sqrt(140), at least 23.6, exceeds every other
    cell's, at most d (1.5 + sqrt(5.6)) < 11.7, by construction);
  * one explicit step of every kernel family against the oracle, window by
    window: windows at the periodic wrap, across the 2 GiB and 4 GiB byte
    offsets of a field and at the mesh's end. The oracle steps each window
    with 8 extra cells on every side (outflow there, periodic along the
    axes a window spans whole) and only cells at least 8 from those edges
    are compared, beyond the 4-cell reach of a two-stage step.
"""
import gc
import traceback

import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import binding as pb

from gpu_util import TOL, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GAMMA = 1.4
MARGIN = 8
PLANTED_P = 100.0


def _fill_rough(st, seed: int, ndim: int):
    """Seeded rough primitive state written as conserved variables, field by field on the device."""
    import torch
    g = torch.Generator(device=st.device)
    g.manual_seed(seed)
    rho, E = st[0], st[ndim + 1]
    rho.uniform_(0.5, 2.0, generator=g)
    for a in range(ndim):
        st[1 + a].uniform_(-1.5, 1.5, generator=g)      # v_a, turned into m_a below
    E.uniform_(0.5, 2.0, generator=g)                   # p, turned into E below
    E.div_(GAMMA - 1.0)
    tmp = st[1] * st[1]
    for a in range(1, ndim):
        tmp.addcmul_(st[1 + a], st[1 + a])
    tmp.mul_(rho).mul_(0.5)
    E.add_(tmp)
    del tmp
    for a in range(ndim):
        st[1 + a].mul_(rho)
    torch.cuda.synchronize(st.device)


def _plant_cell(st, at: tuple, ndim: int):
    """rho = 1, v = 0, p = 100 at one cell (index tuple in array order)."""
    vals = [1.0] + [0.0] * ndim + [PLANTED_P / (GAMMA - 1.0)]
    for q, v in enumerate(vals):
        st[(q,) + at] = v


def _window(st, ranges) -> np.ndarray:
    """Cells of the given index ranges (array order, each wrapped periodically) as FP64 on the host."""
    import torch
    out = st
    for ax, idx in enumerate(ranges):
        out = torch.index_select(out, 1 + ax, torch.as_tensor(idx, device=st.device))
    return out.double().cpu().numpy()


def _ranges(lo_hi, shape):
    """Array-order index ranges [lo - MARGIN, hi + MARGIN) mod n per axis (None: the whole axis)."""
    out = []
    for ax, n in enumerate(shape):
        if lo_hi[ax] is None:
            out.append(np.arange(n))
        else:
            lo, hi = lo_hi[ax]
            out.append(np.arange(lo - MARGIN, hi + MARGIN) % n)
    return out


def _interior(a: np.ndarray, lo_hi) -> np.ndarray:
    sl = [slice(None)]
    for r in lo_hi:
        sl.append(slice(None) if r is None else slice(MARGIN, -MARGIN))
    return a[tuple(sl)]


def _oracle_window_mesh(ndim, lo_hi, win_shape):
    """Oracle mesh of a window: outflow on cut axes, periodic on whole ones; unit spacing."""
    n_xyz = tuple(reversed(win_shape))
    bc_xyz = tuple(reversed([oracle.PERIODIC if r is None else oracle.OUTFLOW for r in lo_hi]))
    return oracle.Mesh(ndim, n_xyz, GAMMA, bc_xyz, dx=(1.0,) * ndim)


def _run(ndim, n_xyz, dtype, windows, planted_at, families, seed):
    import torch
    print(f"case maxsize {ndim}D {dtype} n={n_xyz}: allocating", flush=True)
    spec = pb.MeshSpec(ndim, n_xyz, GAMMA, (pb.PERIODIC,) * ndim, dx=(1.0,) * ndim)
    s = pb.Solver([spec], dtype)
    failure = None
    try:
        _check(s, ndim, dtype, windows, planted_at, families, seed)
    except Exception:   # report it as text: a kept traceback would keep its frames' device tensors alive
        failure = traceback.format_exc()
    finally:            # free the device memory for the tests after this one
        s.close()
        del s
        gc.collect()
        torch.cuda.empty_cache()
    if failure:
        pytest.fail(failure, pytrace=False)


def _check(s, ndim, dtype, windows, planted_at, families, seed):
    import torch
    st = s.state()
    shape = tuple(st.shape[1:])
    _fill_rough(st, seed, ndim)
    _plant_cell(st, planted_at, ndim)
    u0 = st.clone()
    torch.cuda.synchronize()
    # conserved totals (unit cells) against torch's FP64 sums of the same fields
    print(f"  totals over {np.prod(tuple(st.shape[1:]))} cells", flush=True)
    tot = s.totals()[0]
    for q in range(ndim + 2):
        want = float(st[q].double().sum())
        assert abs(tot[q] - want) <= 1e-11 * abs(want), (q, tot[q], want)

    # oracle windows of the input, and their one-step references
    wins = []
    for lo_hi in windows:
        U = _window(u0, _ranges(lo_hi, shape))
        wins.append((lo_hi, U, _oracle_window_mesh(ndim, lo_hi, U.shape[1:])))
    # the CFL step: the planted cell's window decides it
    planted = [w for w in wins if all(r is None or r[0] <= i < r[1] for r, i in zip(w[0], planted_at))]
    assert len(planted) == 1
    lo_hi, U, m = planted[0]
    dt_ref = oracle.cfl_dt(m, U, 0.5)
    print(f"  cfl_dt over {np.prod(shape)} cells", flush=True)
    dt = s.cfl_dt(0.5)[0]
    assert abs(dt - dt_ref) <= 1e-14 * dt_ref, (dt, dt_ref)
    # the entry point without a context runs the same reduction
    stream = torch.cuda.current_stream().cuda_stream
    assert pb.paraiso_cfl_dt_static(s.meshes, s.current(), 0.5, stream) == [dt]
    refs = [_interior(oracle.step(m, U, dt_ref), lo_hi) for lo_hi, U, m in wins]
    for (lo_hi, U, _), ref in zip(wins, refs):
        assert rel_err(ref, _interior(U, lo_hi)) > 1e-4      # the step changes every window

    for name, v, queue in families:
        print(f"  family {name}: one step", flush=True)
        s.state().copy_(u0)
        s.set_variant(v)
        # a grid of one workgroup per item beyond 2^32 work-items takes the queue instead
        assert s.variant()["persistent"] == queue, (name, s.variant())
        s.step(dt_ref)
        torch.cuda.synchronize()
        out = s.state()
        for (lo_hi, _, _), ref in zip(wins, refs):
            got = _interior(_window(out, _ranges(lo_hi, shape)), lo_hi)
            err = rel_err(got, ref)
            print(f"    window {lo_hi}: rel err {err:.3e}", flush=True)
            assert err <= TOL[dtype], (name, lo_hi, err)


def test_2d_f32_rows_just_under_4_gib():
    # 2 rows of 2^30 - 64 cells: 4 GiB - 256 B per row of a field, 2^31 - 128 cells in all
    nx, ny = (1 << 30) - 64, 2
    windows = [(None, (0, 64)),                                  # x wrap
               (None, ((1 << 29) - 32, (1 << 29) + 32)),         # 2 GiB into a row
               (None, ((1 << 28) + 123, (1 << 28) + 187)),
               (None, (nx - 128, nx))]                           # the end, wrapping onto x = 0
    # workgroups of 256 threads, one per item: the marches' strips of 56 (fused)
    # and 60 columns, 19.2 M and 17.9 M, and the LDS tiles of 32 columns, 33.6 M,
    # pass 2^32 work-items and take the queue; the per-cell kernel's 64-column
    # tiles, 2^24 - 1 of them, stay just under it
    families = [("fused march", dict(tile=(64, 20), lds=2, fuse=1, threads=256), 1),
                ("one-stage march", dict(tile=(64, 8), lds=2, fuse=0, threads=256), 1),
                ("LDS tile, fused", dict(tile=(32, 16), lds=1, fuse=1), 1),
                ("per-cell", dict(tile=(64, 4), lds=0, fuse=0), 0)]
    _run(2, (nx, ny), "f32", windows, (1, nx - 100), families, seed=31)


def test_2d_f64_rows_just_under_4_gib():
    # FP64: 2 rows of 2^29 - 32 cells, 4 GiB - 256 B per row of a field
    nx, ny = (1 << 29) - 32, 2
    windows = [(None, (0, 64)),
               (None, ((1 << 28) - 32, (1 << 28) + 32)),         # 2 GiB into a row
               (None, (nx - 128, nx))]
    families = [("fused march", dict(tile=(64, 40), lds=2, fuse=1, threads=256), 0),
                ("one-stage march", dict(tile=(64, 8), lds=2, fuse=0, threads=256), 0)]
    _run(2, (nx, ny), "f64", windows, (0, nx - 70), families, seed=32)


def test_3d_f32_planes_just_under_4_gib():
    # 2 planes of 32768 x 32767 cells: 4 GiB - 128 KiB per plane of a field, 2^31 - 2^16 cells
    nx, ny, nz = 32768, 32767, 2
    windows = [(None, (0, 8), (0, 64)),                          # the (x, y) wrap corner
               (None, (16380, 16388), (0, 64)),                  # 2 GiB into a plane (y = 16384, x = 0)
               (None, (ny - 8, ny), (nx - 64, nx))]              # the last corner
    families = [("one-stage march", dict(tile=(64, 4, 64), lds=2, fuse=0, waves_per_eu=3), 0),
                ("fused march", dict(tile=(64, 12, 64), lds=2, fuse=1), 0),
                ("LDS tile, fused", dict(tile=(16, 8, 4), lds=1, fuse=1), 0),
                ("per-cell", dict(tile=(16, 4, 4), lds=0, fuse=0), 1)]   # 2^24 tiles x 256: the queue
    _run(3, (nx, ny, nz), "f32", windows, (1, ny - 3, nx - 10), families, seed=33)
