"""GPU: explicit time marching (forward Euler with the global step of
eq. (17)), the baseline solver the paper compares fast sweeping and NMG
against, through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import TOL_CONVERGED, TOL_STEP, context, require_gpu, state_err
from paper_2206_13164_amd import inputs as I
from test_gpu_parity import CASES, small_spec

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", CASES)
def test_euler_steps_match_oracle(orc, case):
    # three steps from a random state: every cell from the same old state,
    # the same global step as the oracle's, normalised records
    require_gpu()
    s = small_spec(*case)
    P = orc.problem(s)
    st = I.random_state(s, seed=31, amp=0.06)
    ctx = context(s)
    d = ctx.to_device(st)
    want = st.copy()
    for k in range(3):
        dt_o = orc.euler_step(P, want)
        dt_g = ctx.euler(d)
        assert abs(dt_g - dt_o) <= 1e-14 * dt_o, (k, dt_g, dt_o)
        got = ctx.to_host(d, st.shape[-1])
        assert state_err(got, want, s["M"]) < TOL_STEP, k


def test_euler_on_a_coarse_level_and_zero_steps(orc):
    require_gpu()
    s = small_spec(5, 1, 2, 0, nx=16, ny=12, levels=2)
    P = orc.problem(s)
    ctx = context(s)
    st = I.random_state(dict(s, nx=8, ny=6), seed=32, amp=0.05)
    d = ctx.to_device(st)
    assert ctx.euler(d, nsteps=0, level=1) == 0.0
    assert bool((ctx.to_host(d, st.shape[-1]) == st).all())
    want = st.copy()
    orc.euler_step(P, want, level=1)
    ctx.euler(d, nsteps=1, level=1)
    assert state_err(ctx.to_host(d, st.shape[-1]), want, s["M"]) < TOL_STEP


def test_euler_marches_to_the_fast_sweeping_state():
    # 8x8, config-1 physics, first order: explicit time marching conserves
    # mass step by step and reaches the state the fast-sweeping solver
    # (single level, with the mass correction) converges to, in far more
    # iterations
    require_gpu()
    s = I.spec("lid32_bgk_m3", nx=8, ny=8, levels=1, s3=1)
    cf = context(s)
    a = cf.empty(0)
    cf.init_maxwellian(a)
    rc, cyc, hist = cf.solve(a, 1e-12, 4000)
    assert rc == 0
    ce = context(s)
    b = ce.empty(0)
    ce.init_maxwellian(b)
    m0 = ce.mass(b)
    r0 = ce.residual(b)
    steps, r = 0, r0
    while r > 1e-12 * r0 and steps < 60000:
        ce.euler(b, nsteps=500)
        steps += 500
        assert abs(ce.mass(b) - m0) < 1e-13 * steps * m0
        r = ce.residual(b)
    print(f"Euler: {steps} steps to {r / r0:.1e}; fast sweeping: {cyc} steps")
    assert r <= 1e-12 * r0
    n = I.nalpha(s["M"]) + 3
    assert state_err(ce.to_host(b, n), cf.to_host(a, n), s["M"]) < 1e-9
    assert cyc < steps / 3
