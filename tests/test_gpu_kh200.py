"""The Kelvin-Helmholtz workload's 200-step run, at a reduced mesh, against the oracle.

The benchmarked KH configuration advances 200 steps in FP64 and in FP32.  At
192^2 (ragged against both the 56-column strips and the 78-row blocks of the
tuned register march) the oracle's 200 steps take seconds, so the whole
trajectory is compared: the same step count, the time reached, and the final
state cell by cell.  Both precisions start from the same FP32-representable
state, so one oracle run serves both.

Tolerances: the per-step bars (1e-12 FP64, 1e-5 FP32, relative to each field's
natural scale) accumulated linearly over 200 steps.  The flow is smooth over
this interval (t = 0.12, the shear layer has not rolled up), so errors made in
one step are carried, not amplified.
"""
import numpy as np
import pytest

import oracle
from paper_1204_4779_amd import inputs, variants

from gpu_util import TOL, as_input, gpu_solver, gpu_state, oracle_mesh, spec_of, state_err

pytestmark = pytest.mark.gpu

STEPS = 200


@pytest.fixture(scope="module")
def reference():
    pr = inputs.kelvin_helmholtz_2d(192, seed=1204)
    U0 = as_input(pr.U, "f32")
    m = oracle_mesh(pr)
    ref, t_ref, n_ref = oracle.advance(m, U0, 0.5, 1e9, max_steps=STEPS)
    assert n_ref == STEPS
    return pr, U0, m, ref, t_ref


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_kh_200_steps_follow_the_oracle(reference, dtype):
    pr, U0, m, ref, t_ref = reference
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
    scale = np.array(oracle.totals(m, np.abs(U0)))
    assert np.all(np.abs(tot - tot0) <= STEPS * TOL[dtype] * scale)
    s.close()
