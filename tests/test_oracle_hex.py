"""Pins of the oracle's hexagonal lattice (Fig. 1; Sec. III.B with b_v = 6).

Nothing here restates the oracle's formulas: each test checks a property the
paper or the geometry fixes.

* eq. 16-18 with b_v = 6, D = 2 on the directions the packets travel;
* eq. 22 (mass, momentum, energy of a node's packets) and the pressure
  tensor that eq. 17 implies, on random nodes;
* the mean displacement of a node's mass is its velocity (the three
  surrounding nodes of Fig. 1 carry the barycentric weights);
* hand-derived node tables: the three vertices and weights for end points in
  both triangles of a cell, and eq. 24-26 worked by hand for one node;
* a 60-degree rotation of the whole field commutes with the step;
* a periodic field conserves mass, momentum and energy, and a uniform moving
  state stays uniform;
* a Sod tube along the lattice converges to the exact Euler solution.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.riemann import RiemannSolution

H3 = math.sqrt(3.0) / 2.0


def cart(off):
    """Cartesian vector of an axial lattice step (p, q) = p e_1 + q e_2."""
    off = np.asarray(off, dtype=np.float64)
    return np.stack([off[..., 0] + 0.5 * off[..., 1], H3 * off[..., 1]], axis=-1)


def node(rho, vx, vy, e):
    return np.array([rho, rho * vx, rho * vy, rho * (e + 0.5 * (vx * vx + vy * vy))])


def test_directions_eq16_18():
    """A node at rest with A = 1 exactly (gamma = 3/2, e = 1): c'_1 = 1 and
    d_2 = 0, so the packets with mass are the six c'_1 lanes, each on the
    node's own corner.  Their velocities satisfy eq. 16-18 with b_v / D = 3,
    and each lands one lattice step away along its own velocity."""
    P = oracle.Problem(2, 8, 8, hex=True, gamma=1.5, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    lv = oracle.levels(P, node(1.0, 0.0, 0.0, 1.0))
    assert (lv["c1"], lv["c2"], lv["b"]) == (1, 2, (0, 6, 6))
    assert lv["d2"] == 0.0
    off, pay = oracle.packets(P, node(1.0, 0.0, 0.0, 1.0))
    live = pay[:, 0] > 0.0
    assert live.sum() == 6
    xi = pay[live, 1:3] / pay[live, :1]
    np.testing.assert_allclose(np.hypot(xi[:, 0], xi[:, 1]), 1.0, atol=1e-15)
    np.testing.assert_allclose(cart(off[live]), xi, atol=1e-15)
    np.testing.assert_allclose(xi.sum(0), 0.0, atol=1e-15)                                    # eq. 16
    np.testing.assert_allclose(np.einsum("ja,jb->ab", xi, xi), 3.0 * np.eye(2), atol=1e-14)  # eq. 17
    np.testing.assert_allclose(np.einsum("ja,jb,jc->abc", xi, xi, xi), 0.0, atol=1e-14)      # eq. 18
    # the six directions are 60 degrees apart
    ang = np.sort(np.mod(np.degrees(np.arctan2(xi[:, 1], xi[:, 0])), 360.0))
    np.testing.assert_allclose(np.diff(ang), 60.0, atol=1e-12)


@pytest.mark.parametrize("delta0", [0.0, 0.35])
def test_moments_eq22_and_pressure(delta0):
    """Random nodes: sum m = rho, sum m xi = rho v, sum m zeta = rho E (eq. 22);
    sum m xi xi = rho v v + p I with p = (gamma - 1) rho e (eq. 17, 27); the
    mass-weighted mean displacement is v (barycentric split, eq. 13, 23)."""
    P = oracle.Problem(2, 8, 8, hex=True, delta0=delta0, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    rng = np.random.default_rng(11)
    for _ in range(200):
        rho = rng.uniform(0.2, 3.0)
        vx, vy = rng.uniform(-1.6, 1.6, 2)
        e = rng.uniform(0.0, 4.0)
        y = node(rho, vx, vy, e)
        off, pay = oracle.packets(P, y)
        assert len(off) == (39 if delta0 > 0 else 36)
        assert (pay[:, 0] >= 0.0).all()
        np.testing.assert_allclose(pay[:, 0].sum(), rho, rtol=1e-14)
        np.testing.assert_allclose(pay[:, 1:3].sum(0), rho * np.array([vx, vy]), atol=1e-13 * rho)
        np.testing.assert_allclose(pay[:, 3].sum(), y[3], rtol=1e-13)
        m = pay[:, 0]
        xi = pay[:, 1:3] / np.where(m > 0, m, 1.0)[:, None]
        flux = np.einsum("j,ja,jb->ab", m, xi, xi)
        p = 0.4 * rho * e
        np.testing.assert_allclose(flux, rho * np.outer([vx, vy], [vx, vy]) + p * np.eye(2), atol=1e-12 * (1 + rho))
        # where the mass goes: the mean displacement is v (eq. 13 with the weights of eq. 23)
        np.testing.assert_allclose((m[:, None] * cart(off)).sum(0), rho * np.array([vx, vy]), atol=1e-13 * rho)


@pytest.mark.parametrize("v,corners", [
    # end point (a, b) = (1/4, 1/2): lower triangle of cell (0, 0)
    ((0.5, H3 / 2), {(0, 0): 0.25, (1, 0): 0.25, (0, 1): 0.5}),
    # (a, b) = (3/4, 1/2): upper triangle, vertex (1, 1)
    ((1.0, H3 / 2), {(1, 1): 0.25, (1, 0): 0.5, (0, 1): 0.25}),
    # (a, b) = (-1/4, -1/2): cell (-1, -1), upper triangle
    ((-0.5, -H3 / 2), {(0, 0): 0.25, (0, -1): 0.5, (-1, 0): 0.25}),
    # on a lattice direction, (a, b) = (0, 1/2): the edge (0,0)-(0,1)
    ((0.25, H3 / 2), {(0, 0): 0.5, (0, 1): 0.5}),
])
def test_node_table_rest_group(v, corners):
    """The rest group (delta0 > 0) does not move: its packets land on the
    three nodes around the end point of v with masses alpha_k d_0 (eq. 23).
    The vertices and weights are worked out by hand from v = a e_1 + b e_2."""
    P = oracle.Problem(2, 8, 8, hex=True, delta0=0.5, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    y = node(1.0, v[0], v[1], 1.0)
    off, pay = oracle.packets(P, y)
    rest = pay[:3]  # the rest lane comes first
    d0 = 0.5
    got = {}
    for o, q in zip(off[:3], rest):
        if q[0] > 1e-15:
            got[tuple(int(t) for t in o)] = q[0] / d0
    assert set(got) == set(corners), got
    for k, a in corners.items():
        assert got[k] == pytest.approx(a, abs=1e-14)


def test_levels_by_hand():
    """eq. 24-26 with b_0 = 1, b_1 = b_2 = 6 by hand: rho = 1 at rest,
    gamma = 3/2, e = 9/4, delta0 = 1/2: A = e rho / (rho - d_0) = 4.5,
    c'_1 = 2, c'_2 = 3, d_1 = (9 * 1/2 - 9/4) / (6 * 5) = 0.075,
    d_2 = (9/4 - 4 * 1/2) / 30 = 1/120."""
    P = oracle.Problem(2, 8, 8, hex=True, gamma=1.5, delta0=0.5, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    lv = oracle.levels(P, node(1.0, 0.0, 0.0, 2.25))
    assert (lv["c1"], lv["c2"]) == (2, 3)
    assert lv["A"] == pytest.approx(4.5, rel=1e-15)
    assert lv["d0"] == pytest.approx(0.5, rel=1e-15)
    assert lv["d1"] == pytest.approx(0.075, rel=1e-14)
    assert lv["d2"] == pytest.approx(1.0 / 120.0, rel=1e-13)


def _smooth_field(n, seed, vmax=0.8):
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n), np.arange(n))
    Y = np.zeros((4, n, n))
    rho = np.ones((n, n))
    vx = np.zeros((n, n))
    vy = np.zeros((n, n))
    e = np.full((n, n), 1.6)
    for k in range(3):  # a few periodic Fourier modes in the axial indices
        ka, kb = rng.integers(-2, 3, 2)
        ph = rng.uniform(0, 2 * np.pi, 4)
        arg = 2 * np.pi * (ka * i + kb * j) / n
        rho += 0.2 * np.cos(arg + ph[0])
        vx += vmax / 3 * np.cos(arg + ph[1])
        vy += vmax / 3 * np.cos(arg + ph[2])
        e += 0.4 * np.cos(arg + ph[3])
    Y[0], Y[1], Y[2] = rho, rho * vx, rho * vy
    Y[3] = rho * (e + 0.5 * (vx * vx + vy * vy))
    return Y


def _rotate60(Y):
    """The field rotated by 60 degrees about node (0, 0) of the periodic n x n
    lattice: node (i, j) moves to (-j, i + j) (e_1 -> e_2, e_2 -> e_2 - e_1)
    and vectors turn by 60 degrees."""
    n = Y.shape[-1]
    out = np.empty_like(Y)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ti, tj = (-j) % n, (i + j) % n
    c, s = 0.5, H3
    mx, my = Y[1], Y[2]
    out[0][tj, ti] = Y[0]
    out[1][tj, ti] = c * mx - s * my
    out[2][tj, ti] = s * mx + c * my
    out[3][tj, ti] = Y[3]
    return out


@pytest.mark.parametrize("steps", [1, 3])
def test_rotation_commutes(steps):
    """Rotating the field by 60 degrees, then stepping, equals stepping, then
    rotating (the hexagonal lattice, its triangles and its velocity set are
    invariant under the rotation).  A wrong direction, vertex or weight
    breaks it."""
    n = 12
    P = oracle.Problem(2, n, n, hex=True, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y = _smooth_field(n, 3)
    a, st, _ = oracle.run(P, Y, steps)
    assert st == 0
    b, st, _ = oracle.run(P, _rotate60(Y), steps)
    assert st == 0
    ra = _rotate60(a)
    for f in range(4):
        assert np.max(np.abs(ra[f] - b[f])) <= 1e-12 * np.max(np.abs(b[f])), f


def test_periodic_conservation_and_uniform_state():
    n = 10
    P = oracle.Problem(2, n, n, hex=True, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y = _smooth_field(n, 5)
    t0 = oracle.totals(P, Y)
    Yn, st, _ = oracle.run(P, Y, 5)
    assert st == 0
    np.testing.assert_allclose(oracle.totals(P, Yn), t0, rtol=1e-13, atol=1e-12)
    assert (Yn[0] > 0).all()
    # a uniform moving state stays uniform
    U = np.broadcast_to(node(0.8, 0.37, -0.21, 1.7)[:, None, None], (4, n, n)).copy()
    Un, st, _ = oracle.run(P, U, 4)
    assert st == 0
    np.testing.assert_allclose(Un, U, rtol=1e-14, atol=1e-15)


def _sod_l1(nx, ny=4):
    """Sod tube along e_1 on the hexagonal lattice: the state depends on the
    axial index i only (the diaphragm runs along e_2), rows wrap.  In lattice
    units with lambda = 1 / sqrt(gamma) (left sound speed 1) after 0.2 nx
    steps; node (i, j) lies at distance i sqrt(3)/2 along the normal of the
    e_2 lines.  Returns the mean |rho - rho_exact| and the spread across rows."""
    g = 1.4
    lam2 = 1.0 / g
    P = oracle.Problem(2, nx, ny, hex=True, bc_x=oracle.TRANSMISSIVE, bc_y=oracle.PERIODIC)
    left = np.arange(nx) < nx // 2
    Y = np.zeros((4, ny, nx))
    Y[0] = np.where(left, 1.0, 0.125)
    Y[3] = np.where(left, 1.0, 0.1) * lam2 / (g - 1.0)
    N = int(round(0.2 * nx))
    Yn, st, reach = oracle.run(P, Y, N)
    assert st == 0 and reach <= 5
    s = (np.arange(nx) - (nx // 2 - 0.5)) * H3
    rho_x, _, _ = RiemannSolution((1.0, 0.0, lam2), (0.125, 0.0, 0.1 * lam2), g).sample(s / N)
    return np.mean(np.abs(Yn[0, 0] - rho_x)), np.max(np.abs(Yn[0] - Yn[0, :1]))


def test_sod_converges_to_euler():
    """Consistency with the Euler equations (the macroscopic limit the paper
    compares against, Sec. V.C-D): the L1 density error against the exact
    Riemann solution is small and shrinks under refinement, and the rows stay
    equal (planar data stays planar)."""
    e1, s1 = _sod_l1(200)
    e2, s2 = _sod_l1(400)
    assert e1 < 0.015 and e2 < 0.01
    assert e2 < 0.75 * e1
    assert max(s1, s2) < 1e-10
