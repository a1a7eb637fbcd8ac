"""Operator-level pins of the oracle's R_ij (Sec. 2.3, eq. (13)-(15)):
fixed points, conservation, equivariance and flux consistency."""
import math

import numpy as np
import pytest

import hermite_quad as HQ
from paper_2206_13164_amd import inputs as I

CASES = [
    dict(M=3, collision=0, order=1),
    dict(M=5, collision=1, Pr=2.0 / 3.0, order=2, limiter=0),
    dict(M=5, collision=1, Pr=2.0 / 3.0, order=2, limiter=1),
    dict(M=8, collision=1, Pr=2.0 / 3.0, order=2, limiter=0),
]


def small(case, **kw):
    d = dict(nx=8, ny=6, lx=1.0, ly=0.75, Kn=0.2)
    d.update(case)
    d.update(kw)
    return I.spec(None, **d)


@pytest.mark.parametrize("case", CASES)
def test_global_maxwellian_is_fixed_point(orc, case):
    # global Maxwellian, static walls at the gas temperature, moving nowhere:
    # R(f) = 0 (an invariant of the method), also with a bulk velocity parallel to
    # walls that move with it
    s = small(case, wall_theta=[1.3] * 4)
    P = orc.problem(s)
    st = I.maxwellian_state(s, theta=1.3, rho=0.7)
    R, nrm = orc.residual(P, 0, st)
    assert nrm <= 1e-13
    # uniform flow along x with moving S/N walls is not a fixed point of the
    # E/W walls, but a channel (periodic-like) check on the S/N faces: the
    # y-direction fluxes cancel exactly for such a state
    s2 = small(case, wall_theta=[1.0] * 4, wall_u=[0.3, 0.0, 0.3, 0.0])
    P2 = orc.problem(s2)
    st2 = I.maxwellian_state(s2, u=(0.3, 0.0))
    for j in range(s2["ny"]):
        for i in (2, 3):  # interior in x
            r = orc.cell_residual(P2, 0, st2, i, j)
            assert np.max(np.abs(r)) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_mass_is_conserved_by_the_operator(orc, case):
    # sum_ij R_ij,0 ds = 0: interior mass fluxes cancel, walls have zero net
    # mass flux, Q_0 = 0 and the regularisation only touches |alpha| = M
    s = small(case, wall_u=[0.1, -0.2, 0.4, 0.05], wall_theta=[1.5, 1.0, 0.9, 1.2])
    P = orc.problem(s)
    st = I.random_state(s, seed=4, amp=0.08)
    R, _ = orc.residual(P, 0, st)
    tot = R[..., 3].sum()
    assert abs(tot) < 1e-12 * np.abs(R[..., 3]).sum()


def _mirror_x(s, st):
    al = I.alpha_list(s["M"])
    out = st[:, ::-1, :].copy()
    out[..., 0] *= -1
    sign = (-1.0) ** al[:, 0]
    out[..., 3:] *= sign
    return out


@pytest.mark.parametrize("case", CASES)
def test_mirror_equivariance(orc, case):
    # x -> -x: R(mirror f) = mirror R(f) when the walls are mirrored too
    s = small(case, wall_u=[0.2, 0.1, -0.3, 0.25], wall_theta=[1.5, 1.1, 0.9, 1.3])
    sm = dict(s)
    sm["wall_u"] = [-0.2, 0.25, 0.3, 0.1]       # S, N tangential flip; E <-> W
    sm["wall_theta"] = [1.5, 1.3, 0.9, 1.1]
    P, Pm = orc.problem(s), orc.problem(sm)
    st = I.random_state(s, seed=7, amp=0.08)
    R, _ = orc.residual(P, 0, st)
    Rm, _ = orc.residual(Pm, 0, _mirror_x(s, st))
    assert np.max(np.abs(Rm - _mirror_x(s, R))) < 1e-12


def _rot180(s, st):
    al = I.alpha_list(s["M"])
    out = st[::-1, ::-1, :].copy()
    out[..., :2] *= -1
    out[..., 3:] *= (-1.0) ** (al[:, 0] + al[:, 1])
    return out


@pytest.mark.parametrize("case", CASES)
def test_rotation_equivariance_four_sided(orc, case):
    # (x, y) -> (Lx - x, Ly - y) with every wall moving (the four-sided
    # cavity of Sec. 4.2: u_N = -u_S, u_E = -u_W, opposite walls at equal
    # temperature): the configuration is its own rotation, so
    # R(rot f) = rot R(f)
    s = small(case, wall_u=[-0.21, 0.3, 0.21, -0.3], wall_theta=[1.2, 0.9, 1.2, 0.9])
    P = orc.problem(s)
    st = I.random_state(s, seed=9, amp=0.08)
    R, _ = orc.residual(P, 0, st)
    Rr, _ = orc.residual(P, 0, _rot180(s, st))
    assert np.max(np.abs(Rr - _rot180(s, R))) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_transpose_equivariance(orc, case):
    # x <-> y with Lx != Ly: catches any mix-up of the two directions
    s = small(case, nx=8, ny=6, lx=1.0, ly=0.75, wall_u=[0.2, 0.1, -0.3, 0.25],
              wall_theta=[1.5, 1.1, 0.9, 1.3])
    st_ = dict(s)
    st_.update(nx=6, ny=8, lx=0.75, ly=1.0)
    # walls S,E,N,W -> W,N,E,S under the swap
    st_["wall_u"] = [s["wall_u"][3], s["wall_u"][2], s["wall_u"][1], s["wall_u"][0]]
    st_["wall_theta"] = [s["wall_theta"][3], s["wall_theta"][2], s["wall_theta"][1], s["wall_theta"][0]]
    al = I.alpha_list(s["M"])
    perm = [list(map(tuple, al)).index((a2, a1, a3)) for a1, a2, a3 in al]

    def tr(x):
        y = np.transpose(x, (1, 0, 2)).copy()
        y[..., 0], y[..., 1] = x.transpose(1, 0, 2)[..., 1], x.transpose(1, 0, 2)[..., 0]
        y[..., 3:] = y[..., 3:][..., perm]
        return y

    P, Pt = orc.problem(s), orc.problem(st_)
    st = I.random_state(s, seed=8, amp=0.08)
    R, _ = orc.residual(P, 0, st)
    Rt, _ = orc.residual(Pt, 0, tr(st))
    assert np.max(np.abs(Rt - tr(R))) < 1e-12


def test_odd_xi3_coefficients_stay_zero(orc):
    s = small(CASES[3], wall_u=[0.0, 0.0, 0.3, 0.0], wall_theta=[2.0, 1.0, 1.0, 1.0])
    P = orc.problem(s)
    st = I.random_state(s, seed=1)
    al = I.alpha_list(s["M"])
    odd = al[:, 2] % 2 == 1
    R, _ = orc.residual(P, 0, st)
    assert np.all(R[..., 3:][..., odd] == 0)
    orc.sweep(P, 0, st, nsteps=1)
    assert np.all(st[..., 3:][..., odd] == 0)


@pytest.mark.parametrize("M", [3, 5])
def test_face_flux_consistency_and_limits(orc, M):
    # HLL with equal states is the physical flux Pi(xi_d f) (by quadrature);
    # supersonic states give the upwind flux; the mass component is the same
    # in either cell's basis (bitwise)
    s = I.spec(None, M=M)
    P = orc.problem(s)
    al = orc.alpha_list(M)
    st = I.random_state(I.spec(None, M=M, nx=2, ny=1), seed=5, amp=0.08)[0]
    a, b = st[0], st[1]
    for d in (0, 1):
        F, g, wm, wp = orc.face_flux(P, d, a, a, a[:3])
        grid = HQ.Grid(a[:2], a[2])
        fv = HQ.function_values(al, a[3:], a[:2], a[2], grid.xi)
        want = HQ.project(al, fv * grid.xi[:, d], grid, a[:2], a[2])
        assert np.max(np.abs(F - want)) < 1e-12
        assert np.max(np.abs(g)) == 0.0 and abs(wm + wp - 1) < 1e-15
        Fa, _, _, _ = orc.face_flux(P, d, a, b, a[:3])
        Fb, _, _, _ = orc.face_flux(P, d, a, b, b[:3])
        assert Fa[0] == Fb[0]
        # moments of order <= 2 of the flux agree in both bases
        back = orc.basis_change(M, Fb, b[:3], a[:3])
        assert np.max(np.abs(back - Fa)) < 1e-13
    fast = a.copy()
    fast[0] = 10.0  # all signal speeds positive
    fastb = b.copy()
    fastb[0] = 10.0
    F, g, wm, wp = orc.face_flux(P, 0, fast, fastb, fast[:3])
    assert np.max(np.abs(F - orc.xi_mult(M, 0, fast[3:], fast[:3]))) < 1e-12
    assert (wm, wp) == (0.0, 1.0)


def test_hll_density_jump_closed_form(orc):
    # two states at rest with equal temperature and only a density jump: the
    # HLL mass flux is -(C sqrt(th) / 2) (rho_R - rho_L), with C = C_{M+1}
    M = 5
    P = orc.problem(I.spec(None, M=M))
    N = orc.nalpha(M)
    L = np.zeros(N + 3); R = np.zeros(N + 3)
    L[2] = R[2] = 1.44
    L[3], R[3] = 1.0, 1.6
    F, _, wm, wp = orc.face_flux(P, 0, L, R, L[:3])
    C = orc.cmax(M + 1)
    assert abs(F[0] - (-(C * 1.2 / 2) * 0.6)) < 1e-15
    assert abs(wm - 0.5) < 1e-15 and abs(wp - 0.5) < 1e-15


def test_local_dt(orc):
    # eq. (18) with CFL 0.9; the relaxation cap nu*dt <= 1 binds only for
    # small Kn
    s = I.spec(None, M=5, nx=16, ny=16, Kn=0.3)
    P = orc.problem(s)
    rec = np.zeros(orc.nalpha(5) + 3)
    rec[:4] = [0.2, -0.1, 1.21, 1.0]
    C = orc.cmax(6)
    want = 0.9 / ((0.2 + C * 1.1) * 16 + (0.1 + C * 1.1) * 16)
    assert abs(orc.local_dt(P, 0, rec) - want) < 1e-16
    P2 = orc.problem(I.spec(None, M=5, nx=16, ny=16, Kn=0.001))
    nu = math.sqrt(math.pi / 2) * 1.21 ** 0.19 / 0.001
    assert abs(orc.local_dt(P2, 0, rec) - 1.0 / nu) < 1e-16
