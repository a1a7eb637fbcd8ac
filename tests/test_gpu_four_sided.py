"""GPU: the four-sided lid-driven cavity with anti-parallel wall motion
(Sec. 4.2): every wall moves, opposite walls the opposite way."""
import numpy as np
import pytest

from gpu_common import TOL_STEP, context, require_gpu, state_err
from paper_2206_13164_amd import inputs as I

pytestmark = pytest.mark.gpu


def rot180(M, st):
    """(x, y) -> (Lx - x, Ly - y): u -> -u, f_alpha -> (-1)^(alpha_1 + alpha_2) f_alpha."""
    al = I.alpha_list(M)
    out = st[::-1, ::-1, :].copy()
    out[..., :2] *= -1
    out[..., 3:] *= (-1.0) ** (al[:, 0] + al[:, 1])
    return out


def test_four_sided_vcycles_match_oracle(orc):
    # the paper's four-sided setup (Shakhov, Kn 0.777, M = 5, 1st order) on
    # 16x16 with two levels: two NMG iterations with the mass correction
    require_gpu()
    s = I.spec("four_sided64_shakhov_m5", nx=16, ny=16, levels=2)
    P = orc.problem(s)
    ctx = context(s)
    st = I.maxwellian_state(s)
    d = ctx.to_device(st)
    for _ in range(2):
        orc.vcycle(P, st)
        orc.mass_fix(P, st)
        gn = ctx.fas_vcycle(d)
        assert state_err(ctx.to_host(d, st.shape[-1]), st, s["M"]) < TOL_STEP
    _, wn = orc.residual(P, 0, st)
    assert abs(gn - wn) < 1e-10 * wn


@pytest.mark.parametrize("order", [1, 2])
def test_four_sided_steady_state_is_rotation_symmetric(order):
    # the configuration is its own 180-degree rotation, so is the steady
    # state (the sweep order is not: only the converged state is symmetric)
    require_gpu()
    s = I.spec("four_sided64_shakhov_m5", nx=32, ny=32, levels=3, order=order, limiter=1)
    ctx = context(s)
    d = ctx.empty(0)
    ctx.init_maxwellian(d)
    rc, cyc, hist = ctx.solve(d, 1e-10, 200)
    assert rc == 0, hist
    n = I.nalpha(s["M"]) + 3
    st = ctx.to_host(d, n)
    err = state_err(rot180(s["M"], st), st, s["M"])
    print(f"order {order}: {cyc} cycles, rotation asymmetry {err:.1e}")
    assert err < 1e-7
    # the flow turns: the velocity field is not trivially zero
    assert np.abs(st[..., :2]).max() > 1e-2
