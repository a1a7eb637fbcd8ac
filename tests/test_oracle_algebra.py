"""Pins of the oracle's Hermite algebra (Sec. 2.2-2.3) against quadrature,
closed forms and library routines that do not share its recurrences."""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He
from scipy import integrate

import hermite_quad as HQ
from paper_2206_13164_amd import inputs as I

MS = [3, 5, 8]


def rec_for(M, seed, u=(0.13, -0.21), th=1.3, amp=0.05):
    s = I.spec(None, M=M, nx=1, ny=1)
    st = I.random_state(s, seed=seed, amp=amp)[0, 0]
    st[0], st[1], st[2] = u[0], u[1], th
    return st


def test_index_order_is_graded(orc):
    for M in [3, 5, 8, 12]:
        al = orc.alpha_list(M)
        assert len(al) == math.comb(M + 3, 3) == orc.nalpha(M)
        assert np.array_equal(al, I.alpha_list(M))
        deg = al.sum(axis=1)
        assert np.all(np.diff(deg) >= 0)
        assert {tuple(a) for a in al} == {(a, b, n - a - b) for n in range(M + 1)
                                         for a in range(n + 1) for b in range(n - a + 1)}


@pytest.mark.parametrize("n", range(2, 27))
def test_cmax_is_largest_hermite_root(orc, n):
    # C_{M+1} of eq. (18): largest root of He_{M+1}; two independent routines
    c = np.zeros(n + 1)
    c[n] = 1
    roots = He.hermeroots(c)
    J = np.diag(np.sqrt(np.arange(1, n)), 1)
    ev = np.linalg.eigvalsh(J + J.T)
    assert abs(orc.cmax(n) - roots.max()) < 1e-12 * roots.max()
    assert abs(orc.cmax(n) - ev.max()) < 1e-12 * ev.max()


@pytest.mark.parametrize("M", MS)
def test_basis_change_matches_quadrature(orc, M):
    al = orc.alpha_list(M)
    f = rec_for(M, seed=M)[3:]
    frm = (0.13, -0.21, 1.3)
    for to in [(0.4, 0.1, 0.9), (-0.3, 0.25, 2.1), (0.13, -0.21, 1.3), (0.0, 0.0, 1.0)]:
        got = orc.basis_change(M, f, frm, to)
        g = HQ.Grid(frm[:2], frm[2])
        fv = HQ.function_values(al, f, frm[:2], frm[2], g.xi)
        want = HQ.project(al, fv, g, to[:2], to[2])
        scale = np.maximum(1.0, np.abs(want))
        assert np.max(np.abs(got - want) / scale) < 1e-12, to


@pytest.mark.parametrize("M", MS)
def test_basis_change_round_trip_and_composition(orc, M):
    f = rec_for(M, seed=11)[3:]
    a, b, c = (0.1, 0.2, 1.1), (-0.35, 0.05, 0.7), (0.2, -0.4, 1.9)
    back = orc.basis_change(M, orc.basis_change(M, f, a, b), b, a)
    assert np.max(np.abs(back - f)) < 1e-13
    two = orc.basis_change(M, orc.basis_change(M, f, a, b), b, c)
    one = orc.basis_change(M, f, a, c)
    assert np.max(np.abs(two - one)) < 1e-13
    # a vector supported on |alpha| = M is invariant (unit lower-triangular map)
    top = np.where(orc.alpha_list(M).sum(axis=1) == M, f, 0.0)
    assert np.array_equal(orc.basis_change(M, top, a, c), top)


@pytest.mark.parametrize("M", MS)
def test_basis_change_closed_form(orc, M):
    # Coefficients of the unit vector e_0: prod_d c_{alpha_d}(du_d, dth) with
    # c_n = dth^{n/2} He_n(-du/sqrt(dth)) / n!  (generating function of He_n)
    al = orc.alpha_list(M)
    e0 = np.zeros(len(al))
    e0[0] = 1.0
    du1, du2, dth = 0.37, -0.52, 0.64
    got = orc.basis_change(M, e0, (0.0, 0.0, 1.0), (du1, du2, 1.0 + dth))
    s = math.sqrt(dth)

    def cn(n, du):
        cc = np.zeros(n + 1)
        cc[n] = 1
        return dth ** (n / 2) * He.hermeval(-du / s, cc) / math.factorial(n)

    want = np.array([cn(a, du1) * cn(b, du2) * cn(c, 0.0) for a, b, c in al])
    assert np.max(np.abs(got - want)) < 1e-14


@pytest.mark.parametrize("M", MS)
@pytest.mark.parametrize("d", [0, 1, 2])
def test_xi_multiplication_matches_quadrature(orc, M, d):
    al = orc.alpha_list(M)
    r = rec_for(M, seed=3)
    u, th = r[:2], r[2]
    got = orc.xi_mult(M, d, r[3:], r[:3])
    g = HQ.Grid(u, th)
    fv = HQ.function_values(al, r[3:], u, th, g.xi)
    want = HQ.project(al, fv * g.xi[:, d], g, u, th)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("M", MS)
def test_normalise_preserves_moments_and_sets_constraints(orc, M):
    al = orc.alpha_list(M)
    r = rec_for(M, seed=5)
    rng = np.random.default_rng(9)
    e = [k for k, a in enumerate(al) if a.sum() == 1]
    e2 = [k for k, a in enumerate(al) if tuple(a) in ((2, 0, 0), (0, 2, 0), (0, 0, 2))]
    r[3 + e[0]], r[3 + e[1]] = 0.07, -0.04  # momentum and energy off the basis
    r[3 + e2[0]] += 0.05
    r[3 + e2[1]] += 0.03
    r[3 + e2[2]] += 0.02
    rho0, mom0, en0 = HQ.moments(al, r[3:], r[:2], r[2])
    rc, out = orc.normalise(M, r)
    assert rc == 0
    assert np.all(out[3 + np.array(e)] == 0.0)
    assert out[3 + e2[0]] + out[3 + e2[1]] + out[3 + e2[2]] == 0.0
    rho1, mom1, en1 = HQ.moments(al, out[3:], out[:2], out[2])
    assert abs(rho1 - rho0) < 1e-14 and np.max(np.abs(mom1 - mom0)) < 1e-13 and abs(en1 - en0) < 1e-13
    assert abs(out[3] - rho0) < 1e-14
    # the new basis is the mean velocity and temperature of the function (eq. (3))
    assert np.allclose(out[:2], mom0[:2] / rho0, atol=1e-14)
    th = (en0 / rho0 - (mom0 ** 2).sum() / rho0 ** 2) / 3.0
    assert abs(out[2] - th) < 1e-13
    # a non-physical input is refused
    bad = r.copy()
    bad[3] = -1.0
    assert orc.normalise(M, bad)[0] != 0


@pytest.mark.parametrize("M", MS)
def test_macroscopic_relations_match_quadrature(orc, M):
    # eq. (10): sigma_ij = (1 + delta_ij) f_{e_i+e_j}, q_i = 2 f_{3e_i} + sum_d f_{2e_d+e_i},
    # against the definitions eq. (3)-(4) evaluated by quadrature
    al = orc.alpha_list(M)
    r = rec_for(M, seed=21, amp=0.1)
    u = np.array([r[0], r[1], 0.0])
    g = HQ.Grid(r[:2], r[2])
    fv = HQ.function_values(al, r[3:], r[:2], r[2], g.xi)
    c = g.xi - u
    rho = np.sum(g.W * fv)
    mac = orc.macro(M, r)
    assert abs(mac[0] - rho) < 1e-14
    assert np.allclose([np.sum(g.W * fv * g.xi[:, d]) / rho for d in range(2)], r[:2], atol=1e-14)
    th = np.sum(g.W * fv * (c ** 2).sum(axis=1)) / (3 * rho)
    assert abs(th - r[2]) < 1e-13
    sig = lambda i, j: np.sum(g.W * fv * c[:, i] * c[:, j]) - rho * th * (i == j)
    assert np.allclose([mac[4], mac[5], mac[6], mac[7]], [sig(0, 0), sig(0, 1), sig(1, 1), sig(2, 2)],
                       atol=1e-13)
    q = [0.5 * np.sum(g.W * fv * (c ** 2).sum(axis=1) * c[:, i]) for i in range(3)]
    assert np.allclose(mac[8:11], q, atol=1e-13)


def _prob(M, collision, Pr=2.0 / 3.0, Kn=0.3, omega=0.81, beta=1.0, **kw):
    import oracle
    return oracle.problem(I.spec(None, M=M, collision=collision, Pr=Pr, Kn=Kn, omega=omega,
                                 beta=beta, **kw))


@pytest.mark.parametrize("M", MS)
def test_shakhov_equilibrium_matches_quadrature(orc, M):
    # f^E of eq. (8) projected by quadrature vs f + Q/nu of the oracle
    al = orc.alpha_list(M)
    r = rec_for(M, seed=8, amp=0.1)
    Pr = 2.0 / 3.0
    nu = -orc.collision(_prob(M, 0), r)[5] / r[3 + 5]  # BGK: Q_alpha = -nu f_alpha
    fE = r[3:] + orc.collision(_prob(M, 1, Pr=Pr), r) / nu
    g = HQ.Grid(r[:2], r[2])
    fv = HQ.function_values(al, r[3:], r[:2], r[2], g.xi)
    u = np.array([r[0], r[1], 0.0])
    c = g.xi - u
    rho = np.sum(g.W * fv)
    th = r[2]
    q = np.array([0.5 * np.sum(g.W * fv * (c ** 2).sum(axis=1) * c[:, i]) for i in range(3)])
    maxw = rho / (2 * math.pi * th) ** 1.5 * np.exp(-(c ** 2).sum(axis=1) / (2 * th))
    shak = (1 + (1 - Pr) * (c @ q) / (5 * rho * th ** 2) * ((c ** 2).sum(axis=1) / th - 5)) * maxw
    want = HQ.project(al, shak, g, r[:2], r[2])
    assert np.max(np.abs(fE - want)) < 1e-13
    # heat flux of f^E is (1 - Pr) q
    mac = orc.macro(M, np.concatenate([r[:3], fE]))
    assert np.allclose(mac[8:11], (1 - Pr) * q, atol=1e-13)
    # Pr = 1 reduces Shakhov to BGK (Sec. 2.1)
    assert np.array_equal(orc.collision(_prob(M, 1, Pr=1.0), r), orc.collision(_prob(M, 0), r))
    # conservation: Q_0 = Q_{e_i} = 0, sum_d Q_{2e_d} = 0
    Q = orc.collision(_prob(M, 1, Pr=Pr), r)
    assert Q[0] == 0 and np.all(Q[1:4] == 0)
    assert abs(Q[4] + Q[7] + Q[9]) < 1e-15


def test_collision_frequency(orc):
    # eq. (29), with rho and theta of the cell
    r = rec_for(5, seed=2)
    P = _prob(5, 0, Kn=0.07, omega=0.81, beta=1.0)
    nu = -orc.collision(P, r)[5] / r[3 + 5]
    assert abs(nu - math.sqrt(math.pi / 2) * r[3] * r[2] ** 0.19 / 0.07) < 1e-12 * nu


@pytest.mark.parametrize("M", [3, 5])
@pytest.mark.parametrize("d", [0, 1])
def test_regularisation_matches_projected_derivative(orc, M, d):
    # G = Pi(xi_d df) - Pi(xi_d Pi df) for df = d/ds f(xi; u + s du, th + s dth)
    # with the coefficients held fixed; derivative by complex step, projections
    # by quadrature (Sec. 2.2, the regularised system eq. (12)).
    al = orc.alpha_list(M)
    r = rec_for(M, seed=13, amp=0.1)
    u, th = r[:2], r[2]
    du1, du2, dth = 0.3, -0.2, 0.25
    h = 1e-20
    g = HQ.Grid(u, th, nq=28)
    uc = (u[0] + 1j * h * du1, u[1] + 1j * h * du2)
    val = HQ.function_values(al, r[3:].astype(complex), uc, th + 1j * h * dth, g.xi.astype(complex))
    df = np.imag(val) / h
    full = HQ.project(al, df * g.xi[:, d], g, u, th)
    dfc = HQ.project(al, df, g, u, th)
    dfM = HQ.function_values(al, dfc, u, th, g.xi)
    trunc = HQ.project(al, dfM * g.xi[:, d], g, u, th)
    want = full - trunc
    got = orc.regularisation(M, d, r[3:], du1, du2, dth)
    assert np.max(np.abs(got - want)) < 1e-11
    assert np.all(got[al.sum(axis=1) < M] == 0)


def _half_range_flux(al, f, u, th, d, sig):
    """Pi[(xi.n) 1_{xi.n>0} f] by quadrature: scipy.quad along the normal,
    Gauss-HermiteE across (exact there)."""
    v, w = He.hermegauss(20)
    w = w / math.sqrt(2 * math.pi)
    t = 1 - d
    out = np.zeros(len(al))
    sq = math.sqrt(th)
    for k, a in enumerate(al):
        fac = math.factorial(a[0]) * math.factorial(a[1]) * math.factorial(a[2])
        acc = 0.0
        for b_idx, b in enumerate(al):
            if f[b_idx] == 0 or b[t] != a[t] or b[2] != a[2]:
                continue
            # transverse integrals: int He_{a_t} He_{b_t} w = a_t! (same index)
            tr = math.factorial(a[t]) * math.factorial(a[2])
            ca = np.zeros(a[d] + 1); ca[a[d]] = 1
            cb = np.zeros(b[d] + 1); cb[b[d]] = 1

            def integrand(vv):
                xi_n = sig * (u[d] + sq * vv)
                return (xi_n * He.hermeval(vv, ca) * He.hermeval(vv, cb)
                        * math.exp(-0.5 * vv * vv) / math.sqrt(2 * math.pi))
            lo, hi = (-u[d] / sq, np.inf) if sig > 0 else (-np.inf, -u[d] / sq)
            val, _ = integrate.quad(integrand, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=200)
            acc += f[b_idx] * th ** (-sum(b) / 2.0) * tr * val
        out[k] = th ** (sum(a) / 2.0) / fac * acc
    return out


@pytest.mark.parametrize("wall", [0, 1, 2, 3])
def test_wall_flux_matches_quadrature(orc, wall):
    M = 3
    al = orc.alpha_list(M)
    r = rec_for(M, seed=17 + wall, u=(0.11, -0.07), th=1.2, amp=0.1)
    P = _prob(M, 0, wall_u=[0.3, -0.2, 0.4, 0.1], wall_theta=[1.5, 0.8, 1.0, 1.3])
    d = 1 if wall in (0, 2) else 0
    sig = 1.0 if wall in (1, 2) else -1.0
    out = _half_range_flux(al, r[3:], r[:2], r[2], d, sig)
    # entering half: rho_w (xi.n) 1_{xi.n<0} M_w, rho_w from zero net mass flux
    thw = P.wall_theta[wall]
    uw = [0.0, 0.0]
    uw[1 - d] = P.wall_u[wall]
    # half-line integral of a Gaussian: exact value of the mass flux of M_w
    in_mass = -math.sqrt(thw / (2 * math.pi))
    rho_w = -out[0] / in_mass
    # project the entering half in the cell basis by 1-D quad along the normal
    vq, wq = He.hermegauss(30)
    want_in = np.zeros(len(al))
    for k, a in enumerate(al):
        fac = math.factorial(a[0]) * math.factorial(a[1]) * math.factorial(a[2])
        ca = [np.eye(a[j] + 1)[a[j]] for j in range(3)]

        def lin(xn):  # integrand along the normal velocity component
            vloc = (xn - r[d]) / math.sqrt(r[2])
            return He.hermeval(vloc, ca[d]) * xn * sig * math.exp(-0.5 * (xn - 0.0) ** 2 / thw) / math.sqrt(2 * math.pi * thw)
        lo, hi = (-np.inf, 0.0) if sig > 0 else (0.0, np.inf)
        val, _ = integrate.quad(lin, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=200)
        # tangential component: Gaussian around uw[t] with variance thw, polynomial He_{a_t}((x-u_t)/sqrt th)
        t = 1 - d
        xt = uw[t] + math.sqrt(thw) * vq
        tv = np.sum(wq / math.sqrt(2 * math.pi) * He.hermeval((xt - r[t]) / math.sqrt(r[2]), ca[t]))
        x3 = math.sqrt(thw) * vq
        tv3 = np.sum(wq / math.sqrt(2 * math.pi) * He.hermeval(x3 / math.sqrt(r[2]), ca[2]))
        want_in[k] = r[2] ** (sum(a) / 2.0) / fac * rho_w * val * tv * tv3
    got = orc.wall_flux(P, wall, r)
    want = out + want_in
    assert abs(want[0]) < 1e-12 and abs(got[0]) < 1e-14  # zero net mass flux
    assert np.max(np.abs(got - want)) < 2e-11


def test_wall_matched_maxwellian_gives_full_flux(orc):
    # a wall-matched Maxwellian: rho_w = rho and the two halves add up to
    # Pi(xi_n M), i.e. exactly the full-range flux of the Maxwellian
    M = 5
    for wall in range(4):
        d = 1 if wall in (0, 2) else 0
        sig = 1.0 if wall in (1, 2) else -1.0
        P = _prob(M, 0, wall_u=[0.2, 0.3, -0.1, 0.15], wall_theta=[1.4, 0.9, 1.1, 1.7])
        rec = np.zeros(orc.nalpha(M) + 3)
        rec[1 - d] = P.wall_u[wall]
        rec[2] = P.wall_theta[wall]
        rec[3] = 0.8
        got = orc.wall_flux(P, wall, rec)
        want = sig * orc.xi_mult(M, d, rec[3:], rec[:3])
        assert np.max(np.abs(got - want)) < 1e-14
