"""Pins of the oracle's whole step (scatter over all sources, Sec. V.A-B).

Invariants that hold for the method in exact arithmetic, checked to rounding:
conservation on periodic domains (eq. 22 plus migration), uniform states stay
uniform, mirror symmetry, positivity, the transmissive-end momentum balance
(the discrete pressure of eq. 17 / 24-25 acting on the tube ends), planar 2-D
runs keep identical rows, and the 1-D / 2-D identity of rho and rho u after one
step (equal level weights when d_0 = rho / 2).
"""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs


def _rel_totals_drift(P, Y0, Y1):
    t0, t1 = oracle.totals(P, Y0), oracle.totals(P, Y1)
    scale = np.array([abs(t0[0])] + [np.sum(np.abs(Y0[1:-1]))] * P.dim + [abs(t0[-1])])
    return np.abs(t1 - t0) / scale


@pytest.mark.parametrize("dim,nx,ny", [(1, 257, 1), (2, 37, 29)])
def test_periodic_conservation(dim, nx, ny):
    P = oracle.Problem(dim, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y0 = inputs.random_state(3, dim, nx, ny, vel=(-1.5, 1.5), e=(0.0, 2.0), smooth=5)
    Y, st, reach = oracle.run(P, Y0, 25)
    assert st == 0 and reach <= 5
    assert np.all(_rel_totals_drift(P, Y0, Y) < 2e-13)


@pytest.mark.parametrize("dim,bcx", [(1, oracle.PERIODIC), (1, oracle.TRANSMISSIVE),
                                     (2, oracle.PERIODIC), (2, oracle.TRANSMISSIVE)])
def test_uniform_state_stays_uniform(dim, bcx):
    rng = np.random.default_rng(5)
    nx, ny = 23, (9 if dim == 2 else 1)
    for _ in range(6):
        rho = rng.uniform(0.1, 3.0)
        v = rng.uniform(-1.7, 1.7, size=dim)
        e = rng.uniform(0.0, 2.5)
        P = oracle.Problem(dim, nx, ny, bc_x=bcx, bc_y=bcx)
        node = np.array([rho] + list(rho * v) + [rho * (e + 0.5 * float(v @ v))])
        Y0 = np.broadcast_to(node[:, None, None], P.shape).copy()
        Y, st, _ = oracle.run(P, Y0, 4)
        assert st == 0
        assert np.allclose(Y, Y0, rtol=1e-14, atol=1e-14 * (rho + node[-1]))
        if bcx == oracle.TRANSMISSIVE:
            # every node sees its packets in the same order: bit-identical nodes
            assert np.all(Y == Y[:, :1, :1])


def test_mirror_symmetry_1d():
    nx = 301
    P = oracle.Problem(1, nx)
    Y0 = inputs.random_state(8, 1, nx, vel=(-1.4, 1.4), smooth=7)
    M = Y0[:, :, ::-1].copy()
    M[1] *= -1
    A, _, _ = oracle.run(P, Y0, 6)
    B, _, _ = oracle.run(P, M, 6)
    B = B[:, :, ::-1].copy()
    B[1] *= -1
    scale = np.max(np.abs(A), axis=(1, 2), keepdims=True)
    assert np.all(np.abs(A - B) <= 1e-13 * scale)


def test_mirror_symmetry_2d():
    nx, ny = 31, 17
    P = oracle.Problem(2, nx, ny, bc_y=oracle.TRANSMISSIVE)
    Y0 = inputs.random_state(9, 2, nx, ny, vel=(-1.2, 1.2), smooth=3)
    # x -> -x
    M = Y0[:, :, ::-1].copy()
    M[1] *= -1
    A, _, _ = oracle.run(P, Y0, 3)
    B, _, _ = oracle.run(P, M, 3)
    B = B[:, :, ::-1].copy()
    B[1] *= -1
    scale = np.max(np.abs(A[[0, 3]]))
    mscale = np.max(np.abs(A[1:3]))
    assert np.max(np.abs(A[[0, 3]] - B[[0, 3]])) <= 1e-13 * scale
    assert np.max(np.abs(A[1:3] - B[1:3])) <= 1e-13 * mscale
    # x <-> y transpose on a square grid with equal boundaries
    P2 = oracle.Problem(2, 19, 19, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y1 = inputs.random_state(10, 2, 19, 19, vel=(-1.2, 1.2), smooth=3)
    T = np.stack([Y1[0].T, Y1[2].T, Y1[1].T, Y1[3].T])
    A, _, _ = oracle.run(P2, Y1, 3)
    B, _, _ = oracle.run(P2, T, 3)
    B = np.stack([B[0].T, B[2].T, B[1].T, B[3].T])
    assert np.max(np.abs(A - B)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("dim", [1, 2])
def test_positivity(dim):
    nx, ny = (400, 1) if dim == 1 else (48, 40)
    P = oracle.Problem(dim, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y0 = inputs.random_state(12, dim, nx, ny, rho=(0.01, 3.0), vel=(-1.5, 1.5), e=(0.0, 1.5))
    Y, st, reach = oracle.run(P, Y0, 15)
    assert st == 0
    rho = Y[0]
    assert np.all(rho > 0)
    v2 = sum((Y[1 + a] / rho) ** 2 for a in range(dim))
    e = Y[-1] / rho - 0.5 * v2
    assert np.all(e >= -1e-12 * (Y[-1] / rho))


def test_transmissive_sod_balances():
    """While the ends see undisturbed states at rest, mass and energy stay in the
    tube and the momentum grows by exactly p_L - p_R (lattice units) per step."""
    nx = 400
    P = oracle.Problem(1, nx)
    x = inputs.node_x(nx)
    for lam in (1.0, 0.8):
        Y0 = oracle.to_lattice(P, oracle.riemann_moments(P, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), lam)
        n = 55  # numerical signals move at most reach = 3 nodes per step: 165 < 200
        Y, st, reach = oracle.run(P, Y0, n)
        assert st == 0 and reach == 3
        t0, t1 = oracle.totals(P, Y0), oracle.totals(P, Y)
        assert abs(t1[0] - t0[0]) <= 1e-13 * t0[0]
        assert abs(t1[2] - t0[2]) <= 1e-13 * t0[2]
        dp = lam * lam * (inputs.SOD_LEFT[3] - inputs.SOD_RIGHT[3])
        assert t1[1] - t0[1] == pytest.approx(n * dp, rel=1e-12)


def test_planar_2d_rows_identical():
    nx, ny = 60, 12
    P = oracle.Problem(2, nx, ny, bc_y=oracle.TRANSMISSIVE)
    x = inputs.node_x(nx)
    Y0 = oracle.to_lattice(P, oracle.riemann_moments(P, x, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5), 0.8)
    Y, st, _ = oracle.run(P, Y0, 10)
    assert st == 0
    assert np.all(Y == Y[:, :1, :])
    assert np.all(Y[2] == 0.0) or np.max(np.abs(Y[2])) < 1e-15


def test_one_step_1d_equals_2d_planar():
    """delta0 = 1/2 gives the 1-D and the square lattice the same c'_1, d_1, d_2;
    the 2-D y-lanes then carry what the 1-D rest lane carries, so rho and
    rho u agree after one step (rho E does not: phi differs, eq. 15)."""
    nx = 120
    P1 = oracle.Problem(1, nx, bc_x=oracle.PERIODIC)
    P2 = oracle.Problem(2, nx, 6, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    Y1 = inputs.random_state(21, 1, nx, vel=(-1.4, 1.4), e=(0.0, 2.0), smooth=4)
    Y2 = np.zeros(P2.shape)
    Y2[0] = Y1[0]
    Y2[1] = Y1[1]
    Y2[3] = Y1[2]
    A, _, _ = oracle.step(P1, Y1)
    B, _, _ = oracle.step(P2, Y2)
    assert np.allclose(B[0], A[0][None, :], rtol=1e-13, atol=0)
    assert np.allclose(B[1], A[1][None, :], rtol=1e-13, atol=1e-13 * np.max(np.abs(A[1])))
    assert not np.allclose(B[3], A[2][None, :], rtol=1e-6)


def test_reach_reported():
    nx = 64
    P = oracle.Problem(1, nx, bc_x=oracle.PERIODIC)
    Y0 = np.zeros(P.shape)
    Y0[0] = 1.0
    Y0[1] = 2.5  # v = 2.5: f = 2
    Y0[2] = 0.5 * 2.5 ** 2 + 1.0  # e = 1: A = 0.8 -> c'_1 = 0, c'_2 = 1
    _, st, reach = oracle.step(P, Y0)
    assert st == 0 and reach == 2 + 1 + 1
    Y0[0, 0, 5] = -1.0
    _, st, _ = oracle.step(P, Y0)
    assert st == -4


def test_square_lattice_transverse_growth():
    """Characterisation (not a pin): on the square dual-level lattice (d_0 = 0)
    a gas at rest with c'_1 = 1 amplifies small perturbations, while the 1-D
    triple-level set and c'_1 = 0 damp them.  Planar runs therefore have to
    keep their rows identical bit for bit to stay planar."""
    rng = np.random.default_rng(0)
    lam2 = 0.8439 ** 2

    def growth(dim, e):
        nx, ny = (48, 48) if dim == 2 else (256, 1)
        P = oracle.Problem(dim, nx, ny, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
        Y = np.zeros(P.shape)
        Y[0] = 1.0 + 1e-8 * rng.standard_normal((ny, nx))
        Y[-1] = Y[0] * e * lam2
        s0 = np.std(Y[0])
        Y, st, _ = oracle.run(P, Y, 40)
        return np.std(Y[0]) / s0

    assert growth(2, 2.5) > 100.0          # A = 1.42: c'_1 = 1, unstable
    assert growth(2, 0.25 * 2.5 / 0.8) < 1.0  # A = 0.45: c'_1 = 0, damped
    assert growth(1, 2.5) < 1.0            # 1-D, rest particle d_0 = rho/2: damped
