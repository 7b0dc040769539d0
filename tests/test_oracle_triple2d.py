"""Pins of the oracle's square lattice with a rest level (2-D triple-level set).

The paper's eq. 24-26 carry the rest weight through b_0 and d_0 for any
lattice; its square lattice (Sec. IV.B) takes d_0 = 0.  With delta0 > 0 the
oracle adds one rest particle group (b_0 = 1, d_0 = delta0 rho) to the four
directions at c'_1, c'_2.  What fixes it, independently of the code:

* the hand-derived tables in golden/equilibrium_tables.json (two cases);
* eq. 22 and eq. 17 with eq. 24-25: the 36 packets reproduce rho, rho v, rho E,
  their velocity spread is p I, d >= 0, sum b d = rho, sum b d c'^2 = D p;
* the rest group obeys eq. 16-18 (a single particle at c' = 0);
* continuity: delta0 -> 0 approaches the dual-level set;
* whole-step invariants: periodic conservation, uniform states stay uniform,
  mirror and transpose symmetry, positivity.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs


def _node(rho, v, E):
    return [rho, rho * v[0], rho * v[1], rho * E]


def _rand_nodes(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = rng.uniform(0.01, 5.0)
        v = rng.uniform(-2.5, 2.5, size=2)
        e = rng.choice([rng.uniform(0, 0.05), rng.uniform(0, 3), rng.uniform(3, 15)])
        yield rho, v, e


@pytest.mark.parametrize("delta0", [0.1, 0.4, 0.55])
def test_moments_pressure_and_weights(delta0):
    g = 1.4
    P = oracle.Problem(2, 4, 4, gamma=g, delta0=delta0)
    for rho, v, e in _rand_nodes(300, 21):
        node = _node(rho, v, e + 0.5 * float(v @ v))
        L = oracle.levels(P, node)
        assert L["b"] == (1, 4, 4)
        assert L["d0"] == pytest.approx(delta0 * rho, rel=1e-15)
        p = (g - 1.0) * rho * L["e"]
        for d in (L["d0"], L["d1"], L["d2"]):
            assert d >= -1e-15 * rho
        assert L["d0"] + 4 * L["d1"] + 4 * L["d2"] == pytest.approx(rho, rel=1e-14)
        assert 4 * L["d1"] * L["c1"] ** 2 + 4 * L["d2"] * L["c2"] ** 2 == pytest.approx(
            2 * p, rel=1e-12, abs=1e-14 * rho)
        # eq. 26 with b_0 d_0: A = D (gamma - 1) e rho / (rho - d_0)
        assert L["A"] == pytest.approx(2 * (g - 1.0) * L["e"] / (1.0 - delta0), rel=1e-13)
        assert L["c1"] ** 2 <= L["A"] < L["c2"] ** 2
        off, pay = oracle.packets(P, node)
        assert len(off) == 36
        tot = pay.sum(axis=0)
        scale = np.array([rho] + [rho * (abs(c) + np.sqrt(e) + 1) for c in v] + [node[-1] + rho])
        assert np.all(np.abs(tot - np.array(node)) <= 4e-15 * scale * 8)
        m = pay[:, 0]
        xi = pay[:, 1:3] / np.where(m > 0, m, 1)[:, None]
        dv = xi - np.asarray(v)[None, :]
        T = np.einsum("p,pa,pb->ab", m, dv, dv)
        assert np.allclose(T, p * np.eye(2), rtol=1e-11, atol=1e-12 * rho)


def test_rest_group_symmetry():
    """eq. 16-18 per level at rest: the rest group is one particle at c' = 0."""
    P = oracle.Problem(2, 4, 4, delta0=0.5)
    node = _node(1.0, [0.0, 0.0], 4.0)
    L = oracle.levels(P, node)
    off, pay = oracle.packets(P, node)
    rest = [(o, p) for o, p in zip(off, pay) if p[0] > 0 and o[0] == 0 and o[1] == 0]
    assert len(rest) == 1 and rest[0][1][0] == pytest.approx(L["d0"], rel=1e-15)
    # its momentum is m v = 0 and its energy m phi
    assert rest[0][1][1] == 0.0 and rest[0][1][2] == 0.0
    assert rest[0][1][3] == pytest.approx(L["d0"] * L["phi"], rel=1e-15)


def test_continuity_at_delta0_zero():
    nx, ny = 24, 18
    Y0 = inputs.random_state(22, 2, nx, ny, vel=(-1.1, 1.1), e=(0.1, 1.5), smooth=3)
    A, st, _ = oracle.run(oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC), Y0, 2)
    B, st2, _ = oracle.run(oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC,
                                          delta0=1e-9), Y0, 2)
    assert st == 0 and st2 == 0
    d = np.max(np.abs(A - B)) / np.max(np.abs(A))
    assert 0.0 < d < 1e-7  # moves, and only by O(delta0)


def test_periodic_conservation_and_positivity():
    nx, ny = 37, 29
    P = oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC, delta0=0.5)
    Y0 = inputs.random_state(23, 2, nx, ny, rho=(0.05, 2.0), vel=(-1.5, 1.5), e=(0.0, 2.0), smooth=5)
    Y, st, reach = oracle.run(P, Y0, 25)
    assert st == 0 and reach <= 5
    t0, t1 = oracle.totals(P, Y0), oracle.totals(P, Y)
    assert abs(t1[0] - t0[0]) < 2e-13 * t0[0]
    assert abs(t1[3] - t0[3]) < 2e-13 * t0[3]
    mom = np.sum(np.abs(Y0[1:3]))
    assert np.all(np.abs(t1[1:3] - t0[1:3]) < 2e-13 * mom)
    assert np.all(Y[0] > 0)
    e = Y[3] / Y[0] - 0.5 * ((Y[1] / Y[0]) ** 2 + (Y[2] / Y[0]) ** 2)
    assert np.all(e >= -1e-12 * Y[3] / Y[0])


def test_uniform_state_stays_uniform():
    rng = np.random.default_rng(24)
    P = oracle.Problem(2, 23, 9, bc_x=oracle.TRANSMISSIVE, bc_y=oracle.TRANSMISSIVE, delta0=0.5)
    for _ in range(6):
        rho, v, e = rng.uniform(0.1, 3.0), rng.uniform(-1.7, 1.7, size=2), rng.uniform(0.0, 2.5)
        node = np.array(_node(rho, v, e + 0.5 * float(v @ v)))
        Y0 = np.broadcast_to(node[:, None, None], P.shape).copy()
        Y, st, _ = oracle.run(P, Y0, 4)
        assert st == 0
        assert np.allclose(Y, Y0, rtol=1e-14, atol=1e-14 * (rho + node[-1]))
        assert np.all(Y == Y[:, :1, :1])


def test_mirror_and_transpose_symmetry():
    nx, ny = 31, 17
    P = oracle.Problem(2, nx, ny, bc_y=oracle.TRANSMISSIVE, delta0=0.45)
    Y0 = inputs.random_state(25, 2, nx, ny, vel=(-1.2, 1.2), smooth=3)
    M = Y0[:, :, ::-1].copy()
    M[1] *= -1
    A, _, _ = oracle.run(P, Y0, 3)
    B, _, _ = oracle.run(P, M, 3)
    B = B[:, :, ::-1].copy()
    B[1] *= -1
    assert np.max(np.abs(A - B)) <= 1e-13 * np.max(np.abs(A))
    P2 = oracle.Problem(2, 19, 19, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC, delta0=0.45)
    Y1 = inputs.random_state(26, 2, 19, 19, vel=(-1.2, 1.2), smooth=3)
    T = np.stack([Y1[0].T, Y1[2].T, Y1[1].T, Y1[3].T])
    A, _, _ = oracle.run(P2, Y1, 3)
    B, _, _ = oracle.run(P2, T, 3)
    B = np.stack([B[0].T, B[2].T, B[1].T, B[3].T])
    assert np.max(np.abs(A - B)) <= 1e-13 * np.max(np.abs(A))
