"""The linear-wave kernel (paraiso_wave_advance) against the FP64 oracle.

One step: f and g within a few ulp (the kernel fuses dt * g + f into one FMA),
the energy within 1e-13 relative (its sum runs in another order).  Long runs
at the paper's setting (c = 3.43, dt = dx / c, f = sin x, g = cos 3x) keep the
energy constant to rounding on the GPU too, and match the oracle's history.
"""
import math

import numpy as np
import pytest

from oracle import wave
from paper_1204_4779_amd import binding as pb

pytestmark = pytest.mark.gpu

C = 3.43


def _paper(n):
    dx = 2 * math.pi / n
    f, g = wave.paper_initial(n)
    return f, g, dx, dx / C


def _run(fs, gs, c, dx, dt, steps, record=True):
    import torch
    w = pb.WaveLines(fs, gs, c, dx, dt, steps)
    w.advance(steps, record_energy=record)
    torch.cuda.synchronize()
    return ([x.cpu().numpy() for x in w.f], [x.cpu().numpy() for x in w.g],
            [x.cpu().numpy()[:steps] for x in w.energy])


@pytest.mark.parametrize("n", [3, 8, 255, 256, 257, 1000, 3072, 4096])
def test_one_step_matches_oracle(n):
    rng = np.random.default_rng(n)
    f0, g0 = rng.normal(size=n), rng.normal(size=n)
    dx, dt = 0.37, 0.11
    f1, g1, e1 = wave.step(f0, g0, 1.7, dx, dt)
    f, g, e = _run([f0], [g0], 1.7, dx, dt, 1)
    np.testing.assert_allclose(f[0], f1, rtol=0, atol=4e-16 * np.max(np.abs(f1)))
    np.testing.assert_allclose(g[0], g1, rtol=0, atol=1e-14 * np.max(np.abs(g1)))
    assert abs(e[0][0] - e1) <= 1e-13 * abs(e1)


@pytest.mark.parametrize("n", [8, 64, 3072])
def test_paper_runs_keep_the_energy(n):
    f0, g0, dx, dt = _paper(n)
    steps = 1000
    fr, gr, er = wave.advance(f0, g0, C, dx, dt, steps)
    f, g, e = _run([f0], [g0], C, dx, dt, steps)
    e = e[0]
    assert (e.max() - e.min()) / e[0] < 1e-12
    np.testing.assert_allclose(e, er, rtol=1e-12)
    # a rounding difference in f^{n+1} (the kernel's FMA) reaches g through
    # k = c^2 dt / dx^2 (1677 at n = 3072): per step at most a few k eps |f|
    k = C * C * dt / (dx * dx)
    atol_g = 4.0 * steps * k * np.finfo(float).eps * np.max(np.abs(fr))
    np.testing.assert_allclose(g[0], gr, rtol=0, atol=max(atol_g, 1e-12))
    np.testing.assert_allclose(f[0], fr, rtol=0, atol=max(steps * dt * atol_g, 1e-12))


def test_batch_of_uneven_lines_equals_solo_runs_and_is_deterministic():
    ns = [8, 100, 3072, 17, 4096, 513]
    rng = np.random.default_rng(7)
    fs = [rng.normal(size=n) for n in ns]
    gs = [rng.normal(size=n) for n in ns]
    cs = [1.0 + 0.5 * k for k in range(len(ns))]
    dxs = [2 * math.pi / n for n in ns]
    dts = [0.9 * dx / c for dx, c in zip(dxs, cs)]
    f, g, e = _run(fs, gs, cs, dxs, dts, 50)
    f2, g2, e2 = _run(fs, gs, cs, dxs, dts, 50)
    for k, n in enumerate(ns):
        np.testing.assert_array_equal(f[k], f2[k])
        np.testing.assert_array_equal(e[k], e2[k])
        fs1, gs1, es1 = _run([fs[k]], [gs[k]], cs[k], dxs[k], dts[k], 50)
        np.testing.assert_array_equal(f[k], fs1[0])
        np.testing.assert_array_equal(g[k], gs1[0])
        np.testing.assert_array_equal(e[k], es1[0])
        fr, gr, er = wave.advance(fs[k], gs[k], cs[k], dxs[k], dts[k], 50)
        np.testing.assert_allclose(e[k], er, rtol=1e-12)
        np.testing.assert_allclose(g[k], gr, rtol=0, atol=1e-10 * np.max(np.abs(gr)))


def test_travelling_wave_returns_after_n_steps():
    n = 96
    dx = 2 * math.pi / n
    dt = dx / C
    s = np.sin(np.arange(n) * dx)
    f, _, _ = _run([s], [(np.roll(s, 1) - s) / dt], C, dx, dt, n, record=False)
    np.testing.assert_allclose(f[0], s, rtol=0, atol=1e-11)
    f7, _, _ = _run([s], [(np.roll(s, 1) - s) / dt], C, dx, dt, 7, record=False)
    np.testing.assert_allclose(f7[0], np.roll(s, 7), rtol=0, atol=1e-12)


def test_zero_steps_and_errors():
    f0, g0, dx, dt = _paper(64)
    f, g, _ = _run([f0], [g0], C, dx, dt, 0, record=False)
    np.testing.assert_array_equal(f[0], f0)
    np.testing.assert_array_equal(g[0], g0)
    w = pb.WaveLines([f0], [g0], C, dx, dt, 4)
    with pytest.raises(ValueError):
        w.advance(5)
    with pytest.raises(RuntimeError):   # run() before prepare(): no line table on the device yet
        w.run(1)
    big = pb.WaveLines([np.zeros(4097)], [np.zeros(4097)], C, dx, dt, 1)
    with pytest.raises(pb.ParaisoError) as ei:
        big.advance(1)
    assert ei.value.code == pb.ERR_INVALID_ARG and "line 0" in str(ei.value)


def test_lines_longer_than_the_launch_allows_are_untouched():
    import torch
    rng = np.random.default_rng(9)
    fs = [rng.normal(size=100), rng.normal(size=600)]
    gs = [rng.normal(size=100), rng.normal(size=600)]
    w = pb.WaveLines(fs, gs, 1.0, 0.1, 0.05, 3)
    w.prepare()
    pb.paraiso_wave_run(w.ws_ptr, 2, 3, 256, torch.cuda.current_stream().cuda_stream)   # one cell per thread
    torch.cuda.synchronize()
    np.testing.assert_array_equal(w.f[1].cpu().numpy(), fs[1])
    np.testing.assert_array_equal(w.g[1].cpu().numpy(), gs[1])
    fr, gr, er = wave.advance(fs[0], gs[0], 1.0, 0.1, 0.05, 3)
    np.testing.assert_allclose(w.g[0].cpu().numpy(), gr, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w.energy[0].cpu().numpy()[:3], er, rtol=1e-13)
