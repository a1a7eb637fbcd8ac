"""Pins of the oracle's second-order operator, norm and coarse-grid
correction against definitions that do not go through its own code paths.

* Second-order reconstruction (eq. (15)) with the face and in-cell
  regularisation terms: for a smooth field the discrete operator R_ij of
  eq. (13) must converge at second order to the semi-discrete regularised
  system -Pi(xi_d Pi d_d f) + Q (Sec. 2.2), evaluated here by complex-step
  differentiation of the expansion and Gauss-HermiteE projections.  A slope
  factor 1 instead of 1/2, a swapped face side or a wrong sign or size of the
  in-cell jump leaves an O(1) error and fails.
* Norm of eq. (28): the per-cell weight alpha! theta^-|alpha| is the inner
  product int R^2 / M^[u,theta]_{rho=1} dxi (quadrature).
* Coarse-grid correction of eq. (26): a coarse state that is the same function
  in another basis changes nothing; a known difference delta adds
  T(delta) (quadrature projection) to every child.
"""
import math

import numpy as np
import pytest

import hermite_quad as HQ
from paper_2206_13164_amd import inputs as I


def _linear_field(s, v0, v1, x0=0.5):
    """Records linear in x (constant in y): v(x) = v0 + v1 (x - x0) for every
    record entry; the constraints of eq. (10) are linear, so they hold."""
    nx, ny = s["nx"], s["ny"]
    x = (np.arange(nx) + 0.5) / nx * s["lx"]
    st = np.zeros((ny, nx, len(v0)))
    st[...] = v0[None, None, :] + v1[None, None, :] * (x[None, :, None] - x0)
    return st


def _field_coeffs(M, seed):
    """v0 (a state record at x0) and v1 (its x-derivative), both satisfying
    the linear constraints, with non-zero top-degree coefficients."""
    s = I.spec(None, M=M, nx=1, ny=1)
    v0 = I.random_state(s, seed=seed, amp=0.1)[0, 0]
    v0[:3] = [0.12, -0.07, 1.15]
    g = I.random_state(s, seed=seed + 1, amp=0.1)[0, 0]
    v1 = g.copy()
    v1[:3] = [0.3, 0.2, -0.25]
    v1[3] = 0.2  # d rho / dx
    return v0, v1


def _semi_discrete(al, M, rec0, rec1, xc, x0, d=0, eps=1e-20):
    """-Pi^[c](xi_d Pi^[c] d_x f) at x = xc for f(x) = sum f_alpha(x)
    H_alpha^[u(x), th(x)], with the record v(x) = rec0 + rec1 (x - x0);
    c = v(xc).  Complex step in x, projections by quadrature."""
    c = rec0 + rec1 * (xc - x0)
    vz = rec0.astype(complex) + rec1 * (xc + 1j * eps - x0)
    g = HQ.Grid(c[:2], c[2], nq=28)
    val = HQ.function_values(al, vz[3:], (vz[0], vz[1]), vz[2], g.xi.astype(complex))
    dfx = np.imag(val) / eps
    coef = HQ.project(al, dfx, g, c[:2], c[2])          # Pi^[c] d_x f
    fv = HQ.function_values(al, coef, c[:2], c[2], g.xi)
    return -HQ.project(al, fv * g.xi[:, d], g, c[:2], c[2]), c


@pytest.mark.parametrize("M", [3, 5])
@pytest.mark.parametrize("limiter", [0, 1])
def test_second_order_operator_converges_to_regularised_system(orc, M, limiter):
    al = orc.alpha_list(M)
    v0, v1 = _field_coeffs(M, seed=21 + M)
    errs = []
    for n in (16, 32):
        # square cells; 5 rows between diffuse walls, the checked row j = 2
        # has interior faces on both y sides (the field is constant in y, so
        # the y fluxes cancel and the y regularisation vanishes)
        s = I.spec(None, M=M, nx=n, ny=5, lx=1.0, ly=5.0 / n, order=2, limiter=limiter,
                   collision=0, Kn=1e14, wall_u=[0.0, 0.0, 0.0, 0.0])
        P = orc.problem(s)
        st = _linear_field(s, v0, v1)
        i = n // 2
        xc = (i + 0.5) / n
        R = orc.cell_residual(P, 0, st, i, 2)
        want, c = _semi_discrete(al, M, v0, v1, xc, 0.5)
        assert np.allclose(st[2, i], c, atol=1e-15)
        scale = c[3] * c[2] ** (al.sum(axis=1) / 2.0)
        errs.append(np.max(np.abs(R - want) / scale))
    # second-order convergence to the semi-discrete operator; the terms
    # themselves are O(1)
    assert errs[1] < 2e-3, errs
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_second_order_operator_pin_detects_a_planted_slope_error(orc):
    # the same comparison with the face states moved to x_i +/- dx (slope
    # factor 1 instead of 1/2): emulated by a field of twice the gradient in
    # the reconstruction but not in the target, which must fail the bound
    M = 3
    al = orc.alpha_list(M)
    v0, v1 = _field_coeffs(M, seed=24)
    n = 32
    s = I.spec(None, M=M, nx=n, ny=5, lx=1.0, ly=5.0 / n, order=2, limiter=1, collision=0,
               Kn=1e14)
    P = orc.problem(s)
    i = n // 2
    xc = (i + 0.5) / n
    st = _linear_field(s, v0 + v1 * 0.0, 2.0 * v1, x0=0.5)
    # cell i keeps the value of the one-gradient field at its centre
    st[:, i] = v0 + v1 * (xc - 0.5)
    R = orc.cell_residual(P, 0, st, i, 2)
    want, c = _semi_discrete(al, M, v0, v1, xc, 0.5)
    scale = c[3] * c[2] ** (al.sum(axis=1) / 2.0)
    assert np.max(np.abs(R - want) / scale) > 1e-2


@pytest.mark.parametrize("M", [3, 5, 8])
def test_norm_weight_is_the_maxwellian_weighted_inner_product(orc, M):
    # eq. (28): ||R_ij||^2 = int R(xi)^2 / M^[u,th]_{rho=1}(xi) dxi
    al = orc.alpha_list(M)
    s = I.spec(None, M=M, nx=1, ny=1, lx=1.0, ly=1.0)
    P = orc.problem(s)
    rec = I.random_rhs(s, 0, seed=31, amp=0.3)[0, 0]
    rec[:3] = [0.2, -0.15, 1.7]
    got = orc.norm(P, 0, rec[None, None, :])
    g = HQ.Grid(rec[:2], rec[2])
    Rv = HQ.function_values(al, rec[3:], rec[:2], rec[2], g.xi)
    u = np.array([rec[0], rec[1], 0.0])
    maxw = np.exp(-((g.xi - u) ** 2).sum(axis=1) / (2 * rec[2])) / (2 * math.pi * rec[2]) ** 1.5
    want = math.sqrt(np.sum(g.W * Rv ** 2 / maxw))
    assert abs(got - want) < 1e-12 * want


def _reexpand(al, f, frm, to):
    g = HQ.Grid(frm[:2], frm[2])
    fv = HQ.function_values(al, f, frm[:2], frm[2], g.xi)
    return HQ.project(al, fv, g, to[:2], to[2])


def test_correction_with_a_coarse_state_in_another_basis_is_identity(orc):
    # eq. (26): the coarse difference is formed in one basis, so the same
    # function expressed in another basis is no correction at all
    M = 5
    al = orc.alpha_list(M)
    s = I.spec(None, M=M, nx=8, ny=8)
    P = orc.problem(s)
    st = I.random_state(s, seed=2)
    c, _ = orc.restrict(P, 0, st)
    cn = c.copy()
    for J in range(4):
        for I_ in range(4):
            to = c[J, I_, :3] + np.array([0.07, -0.05, 0.11])
            cn[J, I_, 3:] = _reexpand(al, c[J, I_, 3:], c[J, I_, :3], to)
            cn[J, I_, :3] = to
    out = st.copy()
    kept = orc.correct(P, 0, out, cn, c)
    assert kept == 0
    assert np.max(np.abs(out - st)) < 1e-13


def test_correction_adds_the_projected_difference_to_every_child(orc):
    # a known difference delta of degree >= 3 (it leaves rho, u and theta
    # alone, so the re-normalisation is the identity): each child gets
    # delta projected from the coarse basis into its own basis; the new
    # coarse state is given in a third basis
    M = 5
    al = orc.alpha_list(M)
    deg = al.sum(axis=1)
    s = I.spec(None, M=M, nx=8, ny=8)
    P = orc.problem(s)
    st = I.random_state(s, seed=5)
    c, _ = orc.restrict(P, 0, st)
    rng = np.random.default_rng(77)
    delta = np.where((deg >= 3) & (al[:, 2] % 2 == 0), 0.01 * rng.standard_normal(len(al)), 0.0)
    cn = c.copy()
    for J in range(4):
        for I_ in range(4):
            to = c[J, I_, :3] + np.array([-0.04, 0.06, 0.09])
            cn[J, I_, 3:] = _reexpand(al, c[J, I_, 3:] + delta, c[J, I_, :3], to)
            cn[J, I_, :3] = to
    out = st.copy()
    kept = orc.correct(P, 0, out, cn, c)
    assert kept == 0
    worst = 0.0
    for J in range(8):
        for I_ in range(8):
            par = c[J // 2, I_ // 2]
            want = st[J, I_, 3:] + _reexpand(al, delta, par[:3], st[J, I_, :3])
            assert np.array_equal(out[J, I_, :3], st[J, I_, :3]) or \
                np.max(np.abs(out[J, I_, :3] - st[J, I_, :3])) < 1e-15
            worst = max(worst, np.max(np.abs(out[J, I_, 3:] - want)))
    assert worst < 1e-13
