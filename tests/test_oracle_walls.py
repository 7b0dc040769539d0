"""Pins of the oracle's reflecting walls.

The paper's conclusions name the reflection of shocks on walls as an extension
and give no rule.  The reading: a wall stands on the outer face of each edge
node and reflects every packet that crosses it specularly (landing as far
inside as it would have landed outside, normal momentum negated).  What that
reading fixes, independently of the oracle's code for it:

* mirror doubling: a problem between walls equals one half of the periodic
  problem on the domain doubled by mirroring about the wall (coordinate
  reflected, normal velocity negated).  The step is mirror-symmetric, so the
  packets the mirror half sends across the wall face are the mirror images of
  the packets that cross it from inside; equal up to rounding;
* a closed box conserves mass and total energy (a reflection changes neither);
* a uniform stream against a wall is stopped by a reflected shock whose state
  is the exact solution of the symmetric Riemann problem (u, -u): two shocks,
  u* = 0.
"""
import numpy as np
import pytest

import oracle
from oracle.riemann import RiemannSolution
from paper_1602_02675_amd import inputs

W, P_, T = oracle.REFLECTING, oracle.PERIODIC, oracle.TRANSMISSIVE


def _mirror(Y, axis):
    """Reflect a moment field [nf, ny, nx] about its low face along axis
    (0: x, 1: y): reversed order, normal momentum negated."""
    M = np.flip(Y, axis=2 - axis).copy()
    M[1 + axis] *= -1.0
    return M


def _double(Y, axis):
    return np.concatenate([_mirror(Y, axis), Y], axis=2 - axis)


def _normwise(a, b):
    scale = np.max(np.abs(b), axis=(1, 2), keepdims=True)
    return float(np.max(np.abs(a - b) / scale))


def test_reflect_1d_equals_mirror_doubled_periodic():
    nx = 90
    Y0 = inputs.random_state(11, 1, nx, vel=(-1.2, 1.2), e=(0.2, 2.5), smooth=5)
    A, st, reach = oracle.run(oracle.Problem(1, nx, bc_x=W), Y0, 40)
    assert st == 0 and 1 <= reach <= 5
    B, st, _ = oracle.run(oracle.Problem(1, 2 * nx, bc_x=P_), _double(Y0, 0), 40)
    assert st == 0
    assert _normwise(A, B[:, :, nx:]) < 1e-12
    # the walls matter: the transmissive run is far from it
    C, _, _ = oracle.run(oracle.Problem(1, nx, bc_x=T), Y0, 40)
    assert _normwise(C, A) > 1e-2


@pytest.mark.parametrize("bcx,bcy", [(W, P_), (T, W), (W, W), (W, T)])
def test_reflect_2d_equals_mirror_doubled(bcx, bcy):
    nx, ny, n = 26, 22, 10
    Y0 = inputs.random_state(12, 2, nx, ny, vel=(-1.1, 1.1), e=(0.2, 2.0), smooth=3)
    A, st, reach = oracle.run(oracle.Problem(2, nx, ny, bc_x=bcx, bc_y=bcy), Y0, n)
    assert st == 0 and 1 <= reach <= 5
    D, dbx, dby = Y0, bcx, bcy
    if bcx == W:
        D, dbx = _double(D, 0), P_
    if bcy == W:
        D, dby = _double(D, 1), P_
    B, st, _ = oracle.run(oracle.Problem(2, D.shape[2], D.shape[1], bc_x=dbx, bc_y=dby), D, n)
    assert st == 0
    B = B[:, (ny if bcy == W else 0):, (nx if bcx == W else 0):]
    assert _normwise(A, B) < 1e-12


@pytest.mark.parametrize("dim", [1, 2])
def test_closed_box_conserves_mass_and_energy(dim):
    nx, ny = (120, 1) if dim == 1 else (30, 24)
    P = oracle.Problem(dim, nx, ny, bc_x=W, bc_y=W)
    Y0 = inputs.random_state(13, dim, nx, ny, vel=(-1.5, 1.5), e=(0.0, 2.5), smooth=4)
    Y, st, _ = oracle.run(P, Y0, 30)
    assert st == 0
    t0, t1 = oracle.totals(P, Y0), oracle.totals(P, Y)
    assert abs(t1[0] - t0[0]) < 1e-13 * t0[0]
    assert abs(t1[-1] - t0[-1]) < 1e-13 * t0[-1]
    assert np.all(Y[0] > 0)


def test_reflected_shock_state():
    """Uniform stream (rho, u, p) = (1, 0.5, 1) against the wall at x = 1:
    behind the reflected shock the gas rests at the star state of the
    symmetric Riemann problem."""
    g, nx = 1.4, 400
    u0 = 0.5
    lam = 1.0 / (u0 + np.sqrt(g))  # CFL 1 on the initial state
    P = oracle.Problem(1, nx, bc_x=W)
    x = (np.arange(nx) + 0.5) / nx
    Y = np.zeros((3, 1, nx))
    Y[0] = 1.0
    Y[1] = u0
    Y[2] = 1.0 / (g - 1.0) + 0.5 * u0 * u0
    steps = 150
    t = steps * lam / nx
    Yl, st, _ = oracle.run(P, oracle.to_lattice(P, Y, lam), steps)
    assert st == 0
    pr = oracle.primitives(P, oracle.from_lattice(P, Yl, lam))
    ex = RiemannSolution((1.0, u0, 1.0), (1.0, -u0, 1.0), g)
    assert ex.left_shock and ex.right_shock and abs(ex.u_star) < 1e-12
    rho_ex, _, p_ex = ex.profile(x, 1.0, t)
    xs = 1.0 + ex.s_l * t  # reflected shock position
    plateau = (x > xs + 8.0 / nx) & (x < 1.0 - 8.0 / nx)
    assert plateau.sum() > 20
    rho = pr["rho"][0]
    assert abs(np.mean(rho[plateau]) / ex.rho_star_l - 1.0) < 0.01
    assert abs(np.mean(pr["p"][0][plateau]) / ex.p_star - 1.0) < 0.01
    assert np.max(np.abs(pr["u"][0][plateau])) < 0.02 * u0
    # the shock sits where the exact one is: half the jump is crossed within 3 nodes
    mid = 0.5 * (1.0 + ex.rho_star_l)
    i_half = int(np.argmax(rho > mid))
    assert abs(x[i_half] - xs) < 3.0 / nx
