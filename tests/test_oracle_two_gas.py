"""Pins of the oracle with two gases (1-D lattice): a species moment rho chi
(chi = mass fraction of gas 1) carried by the packets, and each node's gas
the mixture of the two by mass fraction (one gas constant R:
gamma - 1 = 1 / (chi / (gamma_1 - 1) + (1 - chi) / (gamma_2 - 1))).

The conclusions name different gases on the two sides of the tube as an
extension; what pins the oracle's reading, independently of its code:

* the exact solution of the two-gas Riemann problem (each wave inside one
  gas, the contact between them), itself pinned by the Rankine-Hugoniot and
  isentropic relations with each side's gamma and by conservation;
* a hand-derived node (chi = 1/2 of gamma 1.4 and 5/3 is the gas with
  gamma = 3/2) and the moment identities with the species field;
* a single gas split in two labels (gamma_1 = gamma_2) is the one-gas scheme
  with a passive scalar; chi stays in [0, 1]; periodic conservation of all
  four moments;
* the two-gas shock tube converges to the exact solution.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.riemann import RiemannSolution, l1_error
from paper_1602_02675_amd import inputs

G1, G2 = 1.4, 5.0 / 3.0


@pytest.mark.parametrize("left,right", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
                                        ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)),
                                        ((1.0, 0.5, 1.0), (0.5, -0.5, 2.0))])
def test_exact_two_gas_jump_conditions(left, right):
    rs = RiemannSolution(left, right, (G1, G2))
    p = rs.p_star
    for (rho_k, u_k, p_k), shock, rho_s, sign, g in ((left, rs.left_shock, rs.rho_star_l, -1, G1),
                                                     (right, rs.right_shock, rs.rho_star_r, +1, G2)):
        if shock:
            S = rs.s_l if sign < 0 else rs.s_r
            assert rho_k * (u_k - S) == pytest.approx(rho_s * (rs.u_star - S), rel=1e-10, abs=1e-12)
            big = max(p, p_k) + rho_s * (rs.u_star - S) ** 2
            assert rho_k * u_k * (u_k - S) + p_k == pytest.approx(
                rho_s * rs.u_star * (rs.u_star - S) + p, abs=1e-12 * big)
            E_k = p_k / (g - 1) + 0.5 * rho_k * u_k ** 2
            E_s = p / (g - 1) + 0.5 * rho_s * rs.u_star ** 2
            assert E_k * (u_k - S) + p_k * u_k == pytest.approx(
                E_s * (rs.u_star - S) + p * rs.u_star, abs=1e-12 * big * (abs(S) + abs(rs.u_star) + 1))
        else:
            assert p / rho_s ** g == pytest.approx(p_k / rho_k ** g, rel=1e-12)
            c_k, c_s = math.sqrt(g * p_k / rho_k), math.sqrt(g * p / rho_s)
            assert u_k - sign * 2 * c_k / (g - 1) == pytest.approx(
                rs.u_star - sign * 2 * c_s / (g - 1), rel=1e-12, abs=1e-12)


def test_exact_two_gas_conservation_and_reduction():
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (G1, G2))
    n, t = 400000, 0.2
    x = (np.arange(n) + 0.5) / n
    rho, u, p = rs.profile(x, 0.5, t)
    gas1 = x < 0.5 + rs.u_star * t  # left of the contact
    g = np.where(gas1, G1, G2)
    assert np.sum(rho) / n == pytest.approx(0.5 * (1.0 + 0.125), rel=1e-5)
    E = p / (g - 1) + 0.5 * rho * u * u
    assert np.sum(E) / n == pytest.approx(0.5 * (1.0 / (G1 - 1) + 0.1 / (G2 - 1)), rel=1e-5)
    assert np.sum(rho[gas1]) / n == pytest.approx(0.5, rel=1e-4)  # gas 1 stays behind the contact
    one = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G1)
    two = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (G1, G1))
    assert two.p_star == one.p_star and two.u_star == one.u_star


def test_mixture_node_by_hand():
    """chi = 1/2 of gamma 7/5 and 5/3: gamma - 1 = 1 / (1/2 * 5/2 + 1/2 * 3/2)
    = 1/2.  rho = 1, u = 0, p = 1, delta0 = 1/2: e = 2, phi = (1 - 1/4) e =
    3/2, A = (1/2)(2)/(1/2) = 2, c' = (1, 2), d = (1/2, 1/6, 1/12)."""
    P = oracle.Problem(1, 4, gamma=G1, gamma2=G2)
    node = [1.0, 0.0, 2.0, 0.5]
    L = oracle.levels(P, node)
    assert L["gm1"] == pytest.approx(0.5, rel=1e-15)
    assert L["e"] == 2.0 and L["phi"] == pytest.approx(1.5, rel=1e-15)
    assert L["A"] == pytest.approx(2.0, rel=1e-15)
    assert (L["c1"], L["c2"]) == (1, 2)
    assert (L["d0"], L["d1"], L["d2"]) == pytest.approx((0.5, 1.0 / 6.0, 1.0 / 12.0), rel=1e-14)
    # pure gases
    assert oracle.levels(P, [1.0, 0.0, 2.0, 1.0])["gm1"] == pytest.approx(G1 - 1.0, rel=1e-15)
    assert oracle.levels(P, [1.0, 0.0, 2.0, 0.0])["gm1"] == pytest.approx(G2 - 1.0, rel=1e-15)


def test_moment_identities_with_species():
    P = oracle.Problem(1, 4, gamma=G1, gamma2=G2)
    rng = np.random.default_rng(41)
    for _ in range(300):
        rho, v, e, chi = rng.uniform(0.01, 5.0), rng.uniform(-2.5, 2.5), rng.uniform(0.0, 6.0), rng.uniform()
        node = [rho, rho * v, rho * (e + 0.5 * v * v), rho * chi]
        L = oracle.levels(P, node)
        off, pay = oracle.packets(P, node)
        assert pay.shape == (10, 4)
        tot = pay.sum(axis=0)
        scale = np.array([rho, rho * (abs(v) + math.sqrt(e) + 1), node[2] + rho, rho])
        assert np.all(np.abs(tot - np.array(node)) <= 3e-14 * scale)
        p = L["gm1"] * rho * L["e"]
        assert 2 * L["d1"] * L["c1"] ** 2 + 2 * L["d2"] * L["c2"] ** 2 == pytest.approx(p, rel=1e-12, abs=1e-14 * rho)
        # every packet carries its source's chi
        m = pay[:, 0]
        assert np.allclose(pay[:, 3], m * chi, rtol=1e-15, atol=1e-300)


def test_equal_gases_are_one_gas_with_a_passive_label():
    nx = 300
    Y0 = inputs.random_state(42, 1, nx, vel=(-1.2, 1.2), e=(0.1, 2.0), smooth=5)
    P1 = oracle.Problem(1, nx, bc_x=oracle.PERIODIC)
    P2 = oracle.Problem(1, nx, bc_x=oracle.PERIODIC, gamma2=P1.gamma)
    chi = np.where(np.arange(nx) < nx // 2, 1.0, 0.0)
    Y2 = np.concatenate([Y0, (Y0[0] * chi)[None]], axis=0)
    A, st, _ = oracle.run(P1, Y0, 50)
    B, st2, _ = oracle.run(P2, Y2, 50)
    assert st == 0 and st2 == 0
    assert np.max(np.abs(A - B[:3]) / np.max(np.abs(A), axis=(1, 2), keepdims=True)) < 1e-13
    chi_new = B[3] / B[0]
    assert np.all(chi_new >= -1e-15) and np.all(chi_new <= 1 + 1e-15)
    assert np.sum(B[3]) == pytest.approx(np.sum(Y2[3]), rel=1e-13)


def test_two_gas_conservation_and_bounds():
    nx = 257
    P = oracle.Problem(1, nx, bc_x=oracle.PERIODIC, gamma2=G2)
    Y0 = inputs.random_state(43, 1, nx, vel=(-1.2, 1.2), e=(0.1, 2.0), smooth=5)
    chi = 0.5 + 0.5 * np.sin(np.linspace(0, 6 * np.pi, nx))
    Y = np.concatenate([Y0, (Y0[0] * chi)[None]], axis=0)
    B, st, reach = oracle.run(P, Y, 40)
    assert st == 0 and reach <= 5
    t0, t1 = oracle.totals(P, Y), oracle.totals(P, B)
    assert np.all(np.abs(t1 - t0) <= 2e-13 * np.array([t0[0], np.sum(np.abs(Y[1])), t0[2], t0[0]]))
    chi_new = B[3] / B[0]
    assert np.all(chi_new >= -1e-15) and np.all(chi_new <= 1 + 1e-15)
    assert np.all(B[0] > 0)


def _two_gas_sod(nx, t_end=0.2):
    P = oracle.Problem(1, nx, gamma=G1, gamma2=G2)
    speeds = [abs(u) + math.sqrt(g * p / r) for (r, u, _, p), g in
              ((inputs.SOD_LEFT, G1), (inputs.SOD_RIGHT, G2))]
    lam = 1.0 / max(speeds)
    n = int(math.ceil(t_end * nx / lam))
    lam = t_end * nx / n
    x = inputs.node_x(nx)
    Y0 = oracle.to_lattice(P, oracle.riemann_moments(P, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), lam)
    Y, st, _ = oracle.run(P, Y0, n)
    assert st == 0
    return P, x, oracle.from_lattice(P, Y, lam)


def test_two_gas_shock_tube_converges_to_exact():
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (G1, G2))
    errs = []
    for nx in (250, 500, 1000, 2000):
        P, x, Y = _two_gas_sod(nx)
        rho_ex, _, _ = rs.profile(x, 0.5, 0.2)
        errs.append(l1_error(Y[0, 0], rho_ex, 1.0 / nx))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    P, x, Y = _two_gas_sod(1000)
    pr = oracle.primitives(P, Y)
    rho_ex, u_ex, p_ex = rs.profile(x, 0.5, 0.2)
    assert l1_error(pr["u"][0], u_ex, 1e-3) < 0.02
    assert l1_error(pr["p"][0], p_ex, 1e-3) < 0.01
    # the gases meet near the exact contact
    xc = 0.5 + rs.u_star * 0.2
    i = int(np.argmax(pr["chi"][0] < 0.5))
    assert abs(x[i] - xc) < 0.01
    # differs from the one-gas tube (the right gas matters)
    one = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G1)
    assert abs(one.p_star - rs.p_star) > 0.01


# ---------------------------------------------------------------- square lattice
# The same mixture rule on the square dual-level set (D = 2: phi = (1 - gm1) e,
# A = 2 gm1 e, b_1 = 4).


def test_mixture_node_by_hand_square():
    """chi = 1/2 of gamma 7/5 and 5/3 (gamma - 1 = 1/2) on the square set:
    rho = 1, v = 0, p = 1: e = 2, phi = (1 - 1/2) e = 1, A = 2 (1/2) 2 = 2,
    c' = (1, 2); d_1 = (4 - 2) / (4 * 3) = 1/6, d_2 = (2 - 1) / 12 = 1/12
    (4 (d_1 + d_2) = rho, 2 (d_1 c_1^2 + d_2 c_2^2) = p)."""
    P = oracle.Problem(2, 4, 4, gamma=G1, gamma2=G2)
    node = [1.0, 0.0, 0.0, 2.0, 0.5]
    L = oracle.levels(P, node)
    assert L["gm1"] == pytest.approx(0.5, rel=1e-15)
    assert L["e"] == 2.0 and L["phi"] == pytest.approx(1.0, rel=1e-15)
    assert L["A"] == pytest.approx(2.0, rel=1e-15)
    assert (L["c1"], L["c2"]) == (1, 2)
    assert (L["d1"], L["d2"]) == pytest.approx((1.0 / 6.0, 1.0 / 12.0), rel=1e-14)
    # pure gases
    assert oracle.levels(P, [1.0, 0.0, 0.0, 2.0, 1.0])["gm1"] == pytest.approx(G1 - 1.0, rel=1e-15)
    assert oracle.levels(P, [1.0, 0.0, 0.0, 2.0, 0.0])["gm1"] == pytest.approx(G2 - 1.0, rel=1e-15)


def test_moment_identities_with_species_square():
    P = oracle.Problem(2, 4, 4, gamma=G1, gamma2=G2)
    rng = np.random.default_rng(44)
    for _ in range(200):
        rho, e, chi = rng.uniform(0.01, 5.0), rng.uniform(0.0, 6.0), rng.uniform()
        v = rng.uniform(-2.5, 2.5, size=2)
        node = [rho, rho * v[0], rho * v[1], rho * (e + 0.5 * v @ v), rho * chi]
        L = oracle.levels(P, node)
        off, pay = oracle.packets(P, node)
        assert pay.shape == (32, 5)
        tot = pay.sum(axis=0)
        vm = np.abs(v).max() + math.sqrt(e) + 1
        scale = np.array([rho, rho * vm, rho * vm, node[3] + rho, rho])
        assert np.all(np.abs(tot - np.array(node)) <= 3e-14 * scale)
        # pressure of the mixture: the x-lane second moment about v (eq. 24-25)
        p = L["gm1"] * rho * L["e"]
        assert 2 * L["d1"] * L["c1"] ** 2 + 2 * L["d2"] * L["c2"] ** 2 == pytest.approx(p, rel=1e-12, abs=1e-14 * rho)
        m = pay[:, 0]
        assert np.allclose(pay[:, 4], m * chi, rtol=1e-15, atol=1e-300)


def test_equal_gases_are_one_gas_with_a_passive_label_square():
    nx, ny = 41, 23
    Y0 = inputs.random_state(45, 2, nx, ny, vel=(-1.1, 1.1), e=(0.1, 1.5), smooth=3)
    P1 = oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    P2 = oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC, gamma2=P1.gamma)
    chi = np.where(np.arange(nx)[None, :] + np.arange(ny)[:, None] < (nx + ny) // 2, 1.0, 0.0)
    Y2 = np.concatenate([Y0, (Y0[0] * chi)[None]], axis=0)
    A, st, _ = oracle.run(P1, Y0, 12)
    B, st2, _ = oracle.run(P2, Y2, 12)
    assert st == 0 and st2 == 0
    assert np.max(np.abs(A - B[:4]) / np.max(np.abs(A), axis=(1, 2), keepdims=True)) < 1e-13
    chi_new = B[4] / B[0]
    assert np.all(chi_new >= -1e-15) and np.all(chi_new <= 1 + 1e-15)


def test_two_gas_conservation_and_transpose_square():
    n = 29
    P = oracle.Problem(2, n, n, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC, gamma2=G2)
    Y0 = inputs.random_state(46, 2, n, n, vel=(-1.1, 1.1), e=(0.1, 1.5), smooth=3)
    chi = np.random.default_rng(47).uniform(0.0, 1.0, size=(n, n))
    Y = np.concatenate([Y0, (Y0[0] * chi)[None]], axis=0)
    B, st, reach = oracle.run(P, Y, 10)
    assert st == 0 and reach <= 5
    t0, t1 = oracle.totals(P, Y), oracle.totals(P, B)
    mom = np.sum(np.abs(Y[1])) + np.sum(np.abs(Y[2]))
    assert np.all(np.abs(t1 - t0) <= 2e-13 * np.array([t0[0], mom, mom, t0[3], t0[0]]))
    chi_new = B[4] / B[0]
    assert np.all(chi_new >= -1e-15) and np.all(chi_new <= 1 + 1e-15)
    # x <-> y: the transposed state evolves into the transposed result
    T = np.stack([Y[0].T, Y[2].T, Y[1].T, Y[3].T, Y[4].T])
    C, _, _ = oracle.run(P, T, 10)
    C = np.stack([C[0].T, C[2].T, C[1].T, C[3].T, C[4].T])
    assert np.max(np.abs(B - C) / np.max(np.abs(B), axis=(1, 2), keepdims=True)) <= 1e-13


def _two_gas_sod_planar(nx, t_end=0.2):
    P = oracle.Problem(2, nx, 4, gamma=G1, gamma2=G2, bc_y=oracle.TRANSMISSIVE)
    speeds = [abs(u) + math.sqrt(g * p / r) for (r, u, _, p), g in
              ((inputs.SOD_LEFT, G1), (inputs.SOD_RIGHT, G2))]
    lam = 1.0 / max(speeds)
    n = int(math.ceil(t_end * nx / lam))
    lam = t_end * nx / n
    x = inputs.node_x(nx)
    Y0 = oracle.to_lattice(P, oracle.riemann_moments(P, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), lam)
    Y, st, _ = oracle.run(P, Y0, n)
    assert st == 0
    return P, x, oracle.from_lattice(P, Y, lam)


def test_two_gas_planar_tube_converges_to_exact():
    rs = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (G1, G2))
    errs = []
    for nx in (200, 400, 800):
        P, x, Y = _two_gas_sod_planar(nx)
        assert np.all(Y == Y[:, :1, :])  # rows stay identical
        rho_ex, _, _ = rs.profile(x, 0.5, 0.2)
        errs.append(l1_error(Y[0, 0], rho_ex, 1.0 / nx))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    pr = oracle.primitives(P, Y)
    rho_ex, u_ex, p_ex = rs.profile(x, 0.5, 0.2)
    assert l1_error(pr["p"][0], p_ex, 1.0 / 800) < 0.015
    xc = 0.5 + rs.u_star * 0.2
    i = int(np.argmax(pr["chi"][0] < 0.5))
    assert abs(x[i] - xc) < 0.015


def test_mixture_node_by_hand_square_rest_level():
    """The square set with a rest level (d_0 = 0.4 rho), chi = 1/2 of gamma
    7/5 and 5/3: rho = 1, v = 0, p = 1: e = 2, phi = 1, A = 2 (1/2) 2 / 0.6 =
    10/3, c' = (1, 2), d_1 = (4 (0.6) - 2) / 12 = 1/30, d_2 = (2 - 0.6) / 12 =
    7/60 (d_0 + 4 (d_1 + d_2) = rho, 2 (d_1 + 4 d_2) = p); the rest packets
    carry chi like the others."""
    P = oracle.Problem(2, 4, 4, gamma=G1, gamma2=G2, delta0=0.4)
    node = [1.0, 0.0, 0.0, 2.0, 0.5]
    L = oracle.levels(P, node)
    assert L["gm1"] == pytest.approx(0.5, rel=1e-15)
    assert L["phi"] == pytest.approx(1.0, rel=1e-15)
    assert L["A"] == pytest.approx(10.0 / 3.0, rel=1e-15)
    assert (L["c1"], L["c2"]) == (1, 2)
    assert (L["d0"], L["d1"], L["d2"]) == pytest.approx((0.4, 1.0 / 30.0, 7.0 / 60.0), rel=1e-14)
    rng = np.random.default_rng(48)
    for _ in range(100):
        rho, e, chi = rng.uniform(0.01, 5.0), rng.uniform(0.0, 6.0), rng.uniform()
        v = rng.uniform(-2.5, 2.5, size=2)
        node = [rho, rho * v[0], rho * v[1], rho * (e + 0.5 * v @ v), rho * chi]
        off, pay = oracle.packets(P, node)
        assert pay.shape == (36, 5)
        vm = np.abs(v).max() + math.sqrt(e) + 1
        scale = np.array([rho, rho * vm, rho * vm, node[3] + rho, rho])
        assert np.all(np.abs(pay.sum(axis=0) - np.array(node)) <= 3e-14 * scale)
        assert np.allclose(pay[:, 4], pay[:, 0] * chi, rtol=1e-15, atol=1e-300)
