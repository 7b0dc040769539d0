"""The exact Riemann solver (pinned by the jump conditions it must satisfy) and
the oracle's Sod shock tube against it (Sec. V.C-D): grid refinement, and the
1-D result against the 2-D centreline."""
import math

import numpy as np
import pytest

import oracle
from oracle.riemann import RiemannSolution, l1_error
from paper_1602_02675_amd import inputs

G = 1.4


def _energy(rho, u, p):
    return p / (G - 1.0) + 0.5 * rho * u * u


@pytest.mark.parametrize("left,right", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
                                        ((1.0, 0.0, 1.0), (0.3, 0.0, 0.01)),
                                        ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)),
                                        ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),
                                        ((5.99924, 19.5975, 460.894), (5.99242, -6.19633, 46.0950))])
def test_riemann_jump_conditions(left, right):
    rs = RiemannSolution(left, right, G)
    p = rs.p_star
    for (rho_k, u_k, p_k), shock, rho_s, sign in ((left, rs.left_shock, rs.rho_star_l, -1),
                                                  (right, rs.right_shock, rs.rho_star_r, +1)):
        if shock:
            S = rs.s_l if sign < 0 else rs.s_r
            # Rankine-Hugoniot: mass, momentum, energy fluxes in the shock frame
            m1 = rho_k * (u_k - S)
            m2 = rho_s * (rs.u_star - S)
            assert m1 == pytest.approx(m2, rel=1e-10, abs=1e-12)
            big = max(p, p_k) + rho_s * (rs.u_star - S) ** 2  # size of the cancelling terms
            assert rho_k * u_k * (u_k - S) + p_k == pytest.approx(
                rho_s * rs.u_star * (rs.u_star - S) + p, abs=1e-12 * big)
            assert _energy(rho_k, u_k, p_k) * (u_k - S) + p_k * u_k == pytest.approx(
                _energy(rho_s, rs.u_star, p) * (rs.u_star - S) + p * rs.u_star,
                abs=1e-12 * big * (abs(S) + abs(rs.u_star) + 1))
        else:
            # isentrope and Riemann invariant across the rarefaction
            assert p / rho_s ** G == pytest.approx(p_k / rho_k ** G, rel=1e-12)
            c_k = math.sqrt(G * p_k / rho_k)
            c_s = math.sqrt(G * p / rho_s)
            assert u_k - sign * 2 * c_k / (G - 1) == pytest.approx(
                rs.u_star - sign * 2 * c_s / (G - 1), rel=1e-12, abs=1e-12)


def test_riemann_fan_and_symmetry():
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    s = np.linspace(rs.head_l, rs.tail_l, 50)[1:-1]
    rho, u, p = rs.sample(s)
    c = np.sqrt(G * p / rho)
    assert np.allclose(u - c, s, atol=1e-12)  # the fan is made of C- characteristics
    assert np.allclose(u + 2 * c / (G - 1), 2 * math.sqrt(G) / (G - 1), rtol=1e-12)
    # symmetric double rarefaction: u* = 0
    sym = RiemannSolution((1.0, -1.0, 1.0), (1.0, 1.0, 1.0), G)
    assert abs(sym.u_star) < 1e-14
    # equal states: nothing happens
    eq = RiemannSolution((0.7, 0.3, 2.0), (0.7, 0.3, 2.0), G)
    r, uu, pp = eq.sample(np.linspace(-3, 3, 11))
    assert np.allclose(r, 0.7) and np.allclose(uu, 0.3) and np.allclose(pp, 2.0)


def test_riemann_mass_conservation():
    """The exact profile holds the initial mass (ends at rest, no flux)."""
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    n = 400000
    x = (np.arange(n) + 0.5) / n
    rho, u, p = rs.profile(x, 0.5, 0.2)
    assert np.sum(rho) / n == pytest.approx(0.5 * (1.0 + 0.125), rel=1e-5)
    E = p / (G - 1) + 0.5 * rho * u * u
    assert np.sum(E) / n == pytest.approx(0.5 * (2.5 + 0.25), rel=1e-5)


def _sod_1d(nx, lam=None, t_end=0.2):
    P = oracle.Problem(1, nx)
    n, lam_c = inputs.steps_and_lambda(t_end, 1.0 / nx, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    lam = lam_c if lam is None else lam
    n = int(round(t_end * nx / lam))
    x = inputs.node_x(nx)
    Y0 = oracle.to_lattice(P, oracle.riemann_moments(P, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), lam)
    Y, st, reach = oracle.run(P, Y0, n)
    assert st == 0
    return P, x, oracle.from_lattice(P, Y, lam), n * lam / nx


def test_sod_l1_falls_under_refinement():
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    errs = []
    for nx in (250, 500, 1000, 2000):
        P, x, Y, t = _sod_1d(nx)
        assert t == pytest.approx(0.2, rel=1e-12)
        rho_ex, _, _ = rs.profile(x, 0.5, t)
        errs.append(l1_error(Y[0, 0], rho_ex, 1.0 / nx))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    order = math.log(errs[0] / errs[-1], 2) / 3
    assert 0.4 < order < 1.2, (errs, order)


def test_sod_profiles_close_to_exact():
    """Sec. V.D: the solution agrees with the analytical one (first-order scheme)."""
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    P, x, Y, t = _sod_1d(1000)
    pr = oracle.primitives(P, Y)
    rho_ex, u_ex, p_ex = rs.profile(x, 0.5, t)
    dx = 1e-3
    assert l1_error(pr["rho"][0], rho_ex, dx) < 0.01
    assert l1_error(pr["u"][0], u_ex, dx) < 0.02
    assert l1_error(pr["p"][0], p_ex, dx) < 0.01


def test_1d_matches_2d_centreline():
    """Sec. V.D: the 1-D and 2-D solutions are close; here the 1-D result is
    closer to the 2-D centreline than either is to the exact solution."""
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    nx = 400
    _, x, Y1, t = _sod_1d(nx)
    P2 = oracle.Problem(2, nx, 4)
    n, lam = inputs.steps_and_lambda(0.2, 1.0 / nx, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    Y0 = oracle.to_lattice(P2, oracle.riemann_moments(P2, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), lam)
    Y2, st, _ = oracle.run(P2, Y0, n)
    Y2 = oracle.from_lattice(P2, Y2, lam)
    rho_ex, _, _ = rs.profile(x, 0.5, t)
    d12 = l1_error(Y1[0, 0], Y2[0, 2], 1.0 / nx)
    d1x = l1_error(Y1[0, 0], rho_ex, 1.0 / nx)
    d2x = l1_error(Y2[0, 2], rho_ex, 1.0 / nx)
    assert d12 < d1x and d12 < d2x, (d12, d1x, d2x)
