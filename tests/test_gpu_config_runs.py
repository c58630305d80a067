"""The benchmarked workloads' multi-step runs, at reduced meshes, against the oracle.

The KH configuration advances 200 steps (FP64 and FP32), the 3D box 100
steps and the batch of uneven meshes 50 steps (FP32), each on its tuned
kernel.  At reduced sizes the oracle finishes these runs in seconds, so the
whole trajectory is compared: the same step count, the time reached, the
final state cell by cell and the conserved totals.  Inputs are the workloads'
own generators; FP32 runs start from the FP32-rounded state, which the oracle
also starts from.

KH at 192^2 is ragged against both the 56-column strips and the 78-row blocks
of the tuned register march; the 32^3 box is narrower than a 60-column strip
and shallower than a 64-plane chunk.

Tolerances: the per-step bars (1e-12 FP64, 1e-5 FP32, relative to each field's
natural scale) accumulated linearly over the steps.  The HLLC flux and the
minmod limiter are Lipschitz-continuous in their arguments, so rounding
differences made in one step are carried, not amplified, over these short runs
(KH reaches t = 0.12, before the shear layer rolls up).
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import inputs, variants

from gpu_util import TOL, as_input, gpu_solver, gpu_state, oracle_mesh, spec_of, state_err

pytestmark = pytest.mark.gpu


def total_scales(m, U, gamma):
    """Natural scale of each conserved total: sum |rho|, sum |E|, and for each
    momentum component sum rho (|v| + c), the momentum of the fastest signal
    (a flow that starts at rest has no momentum to measure against)."""
    d = U.shape[0] - 2
    rho = U[0]
    m2 = sum(U[1 + a] ** 2 for a in range(d))
    c = np.sqrt(gamma * np.maximum((gamma - 1.0) * (U[d + 1] - 0.5 * m2 / rho), 0.0) / rho)
    W = np.abs(U)
    for a in range(d):
        W[1 + a] = rho * (np.sqrt(m2) / rho + c)
    return np.array(oracle.totals(m, W))

STEPS = 200


@pytest.fixture(scope="module")
def kh_reference():
    pr = inputs.kelvin_helmholtz_2d(192, seed=1204)
    U0 = as_input(pr.U, "f32")
    m = oracle_mesh(pr)
    ref, t_ref, n_ref = oracle.advance(m, U0, 0.5, 1e9, max_steps=STEPS)
    assert n_ref == STEPS
    return pr, U0, m, ref, t_ref


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_kh_200_steps_follow_the_oracle(kh_reference, dtype):
    pr, U0, m, ref, t_ref = kh_reference
    print(f"case kh192 {STEPS} steps {dtype}", flush=True)
    s = gpu_solver(spec_of(pr), dtype, variants.tuned("kh2048", dtype), U0)
    t, n = s.advance(1e9, 0.5, max_steps=STEPS)
    assert n == [STEPS]
    assert abs(t[0] - t_ref) <= STEPS * TOL[dtype] * t_ref
    got = gpu_state(s)
    err = state_err(got, ref, pr.gamma)
    print(f"  kh192 {dtype}: t {t[0]:.12f} (oracle {t_ref:.12f}), state-scaled error {err:.3e}", flush=True)
    assert err <= STEPS * TOL[dtype]
    # periodic: the conserved totals stay those of the initial state
    tot0 = np.array(oracle.totals(m, U0))
    tot = np.array(s.totals()[0])
    scale = total_scales(m, U0, pr.gamma)
    assert np.all(np.abs(tot - tot0) <= STEPS * TOL[dtype] * scale)
    s.close()


def test_box_100_steps_follow_the_oracle():
    steps = 100
    pr = inputs.turbulent_box_3d(32, seed=4779)
    U0 = as_input(pr.U, "f32")
    m = oracle_mesh(pr)
    print(f"case box32 {steps} steps f32", flush=True)
    ref, t_ref, n_ref = oracle.advance(m, U0, 0.5, 1e9, max_steps=steps)
    assert n_ref == steps
    s = gpu_solver(spec_of(pr), "f32", variants.tuned("box512", "f32"), U0)
    t, n = s.advance(1e9, 0.5, max_steps=steps)
    assert n == [steps]
    assert abs(t[0] - t_ref) <= steps * TOL["f32"] * t_ref
    err = state_err(gpu_state(s), ref, pr.gamma)
    print(f"  box32 f32: t {t[0]:.9f} (oracle {t_ref:.9f}), state-scaled error {err:.3e}", flush=True)
    assert err <= steps * TOL["f32"]
    tot0 = np.array(oracle.totals(m, U0))
    scale = total_scales(m, U0, pr.gamma)
    assert np.all(np.abs(np.array(s.totals()[0]) - tot0) <= steps * TOL["f32"] * scale)
    s.close()


def test_batch_50_steps_follow_the_oracle():
    steps = 50
    probs = inputs.blob_batch(8, seed=12044779, nmin=24, nmax=64)
    print(f"case batch of {len(probs)} meshes {[p.n[0] for p in probs]}, {steps} steps f32", flush=True)
    U0s = [as_input(p.U, "f32") for p in probs]
    s = gpu_solver([spec_of(p) for p in probs], "f32", variants.tuned("batch512", "f32"), U0s)
    t, n = s.advance(1e9, 0.5, max_steps=steps)
    assert n == [steps] * len(probs)
    worst = 0.0
    for k, p in enumerate(probs):
        m = oracle_mesh(p)
        ref, t_ref, n_ref = oracle.advance(m, U0s[k], 0.5, 1e9, max_steps=steps)
        assert n_ref == steps
        assert abs(t[k] - t_ref) <= steps * TOL["f32"] * t_ref
        err = state_err(gpu_state(s, k), ref, p.gamma)
        worst = max(worst, err)
        assert err <= steps * TOL["f32"], (k, err)
        tot0 = np.array(oracle.totals(m, U0s[k]))
        scale = total_scales(m, U0s[k], p.gamma)
        assert np.all(np.abs(np.array(s.totals()[k]) - tot0) <= steps * TOL["f32"] * scale)
    print(f"  batch f32: worst state-scaled error {worst:.3e}", flush=True)
    s.close()
