"""The library from C alone: tests/c_abi_consumer.c (hipMalloc'd buffers, a
256 x 192 periodic shear layer in FP64, ten steps of paraiso_advance,
paraiso_totals before and after) compiled with gcc against include/paraiso.h
and libparaiso.so, run, and checked against the oracle's advance of the same
initial state: same step count and time, state within 1e-12, mass and
momentum conserved."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

from gpu_util import rel_err

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_1204_4779_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _initial_state(nx=256, ny=192, gamma=1.4):
    """The consumer's initial state, written out the same way (rational values)."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    y = (j + 0.5) / ny
    mid = (y >= 0.25) & (y < 0.75)
    rho = np.where(mid, 2.0, 1.0)
    vx = np.where(mid, 0.5, -0.5)
    vy = 0.01 * ((i % 7) - 3) / 3.0
    E = 2.5 / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, E])


def test_c_program_advances_through_the_abi(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = tmp_path / "c_abi_consumer"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-O2", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
                        os.path.join(HERE, "c_abi_consumer.c"), "-o", str(exe), "-L", PKG, "-lparaiso",
                        "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                        f"-Wl,-rpath,{PKG}:{os.path.join(ROCM, 'lib')}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = tmp_path / "state.bin"
    print("running the C consumer", flush=True)
    r = subprocess.run([str(exe), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    fields = r.stdout.split()
    steps, t = int(fields[0]), float(fields[1])
    tot0 = np.array([float(v) for v in fields[2:6]])
    tot1 = np.array([float(v) for v in fields[6:10]])
    got = np.fromfile(out, dtype=np.float64).reshape(4, 192, 256)

    U0 = _initial_state()
    m = oracle.Mesh(2, (256, 192), 1.4, (0, 0))
    ref, t_ref, k_ref = oracle.advance(m, U0, 0.5, 1.0, max_steps=10)
    assert steps == k_ref == 10
    assert abs(t - t_ref) <= 1e-13 * t_ref
    assert rel_err(got, ref) <= 1e-12
    np.testing.assert_allclose(tot0, oracle.totals(m, U0), rtol=1e-13, atol=1e-15)
    assert abs(tot1[0] - tot0[0]) <= 1e-13 * abs(tot0[0])
    for q in (1, 2, 3):
        assert abs(tot1[q] - tot0[q]) <= 1e-12 * max(1.0, abs(tot0[q]))
