"""Hexagonal lattice (Fig. 1; Sec. III.B with b_v = 6): HIP path against the
oracle on the same seeded inputs.

Grids span several 64 x 16 tiles with ragged tails in both axial directions;
fields range from pure noise (every window mixes floors, speeds and
triangles) to smooth and planar data; boundaries transmissive and periodic
along either axis; the dual-level set and the one with a rest group.  FP64
fields within the 1e-12 normwise bar; FP32 within 2e-5 after a few steps
(each step rounds the stored state to FP32, relative 6e-8, and the weights
and velocities of each packet are rounded as well); floors and c'_1 bit-exact
(the same device function as the step); the planar tube keeps its rows bit
for bit equal.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs

from parity_helpers import TOL64, normwise_err

pytestmark = pytest.mark.gpu

BC = {"transmissive": oracle.TRANSMISSIVE, "periodic": oracle.PERIODIC}
TOL32 = 2e-5


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def _pair(lbsd, Y, nx, ny, bcx, bcy, d0, n, prec="fp64"):
    P = oracle.Problem(2, nx, ny, hex=True, bc_x=BC[bcx], bc_y=BC[bcy], delta0=d0)
    ref, st, reach = oracle.run(P, Y, n)
    assert st == 0 and reach <= 5
    s = lbsd.Solver(2, nx, ny, lattice="hex", bc_x=bcx, bc_y=bcy, d0_frac=d0, precision=prec)
    s.init_moments(Y, 1.0)  # lambda = 1: physical units are lattice units
    s.step(n)
    got = s.moments()
    return P, ref, got, s


CASES = [  # nx, ny, bc_x, bc_y, d0_frac, seed, smoothing, steps
    (150, 22, "periodic", "periodic", 0.0, 1, 0, 4),
    (150, 22, "transmissive", "periodic", 0.0, 2, 5, 4),
    (97, 13, "transmissive", "transmissive", 0.0, 3, 3, 3),
    (130, 9, "periodic", "transmissive", 0.4, 4, 0, 3),
    (64, 16, "periodic", "periodic", 0.5, 5, 2, 5),  # exactly one tile
    (7, 3, "periodic", "periodic", 0.0, 6, 0, 2),    # smaller than the halo: wrapped many times
]


@pytest.mark.parametrize("nx,ny,bcx,bcy,d0,seed,sm,n", CASES)
def test_random_fields_fp64(lbsd, nx, ny, bcx, bcy, d0, seed, sm, n):
    Y = inputs.random_state(seed, 2, nx, ny, smooth=sm)
    P, ref, got, s = _pair(lbsd, Y, nx, ny, bcx, bcy, d0, n)
    assert normwise_err(got, ref, 2) <= TOL64
    if bcx == "periodic" and bcy == "periodic":  # conservation: the totals of the step
        np.testing.assert_allclose(s.totals(), oracle.totals(P, Y), rtol=1e-12, atol=1e-10)
    s.close()


@pytest.mark.parametrize("nx,ny,bcx,bcy,d0,seed,sm,n", CASES[:4])
def test_random_fields_fp32(lbsd, nx, ny, bcx, bcy, d0, seed, sm, n):
    Y = inputs.random_state(seed, 2, nx, ny, smooth=sm)
    _, ref, got, s = _pair(lbsd, Y, nx, ny, bcx, bcy, d0, n, prec="fp32")
    assert normwise_err(got, ref, 2) <= TOL32
    s.close()


def test_lanes_bit_exact(lbsd):
    """floor of the axial velocity and c'_1 of every node: the step's device
    function against the oracle, on states that straddle many floors and
    speeds."""
    nx, ny = 300, 40
    Y = inputs.random_state(7, 2, nx, ny, vel=(-2.2, 2.2), e=(0.0, 5.0))
    P = oracle.Problem(2, nx, ny, hex=True, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    fa, fb, c1 = oracle.lanes(P, Y)
    s = lbsd.Solver(2, nx, ny, lattice="hex", bc_x="periodic", bc_y="periodic")
    s.init_moments(Y, 1.0)
    ga, gb, gc = s.lanes()
    s.close()
    assert len(np.unique(fa)) >= 4 and len(np.unique(fb)) >= 4 and len(np.unique(c1)) >= 2
    assert np.array_equal(ga, fa) and np.array_equal(gb, fb) and np.array_equal(gc, c1)


def test_planar_tube_rows_identical(lbsd):
    """Sod along e_1 (state depends on the axial index i only, rows wrap):
    oracle parity after 60 steps, and every row of the HIP result is the same
    bit for bit."""
    nx, ny = 300, 8
    lam2 = 1.0 / 1.4
    Y = np.zeros((4, ny, nx))
    left = np.arange(nx) < nx // 2
    Y[0] = np.where(left, 1.0, 0.125)
    Y[3] = np.where(left, 1.0, 0.1) * lam2 / 0.4
    _, ref, got, s = _pair(lbsd, Y, nx, ny, "transmissive", "periodic", 0.0, 60)
    assert normwise_err(got, ref, 2) <= TOL64
    assert np.all(got == got[:, :1, :])
    s.close()


def test_uniform_state_stays_uniform(lbsd):
    """A uniform moving state (periodic) stays uniform: every node equal bit
    for bit, and equal to the start to rounding."""
    nx, ny = 130, 10
    rho, vx, vy, e = 0.8, 0.37, -0.21, 1.7
    Y = np.broadcast_to(np.array([rho, rho * vx, rho * vy, rho * (e + 0.5 * (vx * vx + vy * vy))])[:, None, None],
                        (4, ny, nx)).copy()
    s = lbsd.Solver(2, nx, ny, lattice="hex", bc_x="periodic", bc_y="periodic")
    s.init_moments(Y, 1.0)
    s.step(5)
    got = s.moments()
    s.close()
    assert np.all(got == got[:, :1, :1])
    np.testing.assert_allclose(got, Y, rtol=1e-14, atol=1e-15)


def test_large_grid_one_step(lbsd):
    """2048 x 2048, periodic, a smooth seeded field: the full field after one
    step (the oracle's 4 M nodes take a few seconds)."""
    n = 2048
    Y = inputs.random_state(8, 2, n, n, vel=(-1.2, 1.2), e=(0.5, 2.5), smooth=9)
    _, ref, got, s = _pair(lbsd, Y, n, n, "periodic", "periodic", 0.0, 1)
    assert normwise_err(got, ref, 2) <= TOL64
    s.close()


def test_reach_error(lbsd):
    """A node whose packets would move further than LB_HALO: LB_EREACH."""
    nx, ny = 70, 8
    Y = inputs.random_state(9, 2, nx, ny, vel=(-0.5, 0.5), e=(0.5, 1.0))
    Y[1, 3, 20] = Y[0, 3, 20] * 4.2  # v = (4.2, 0): floor(a) = 4, reach 4 + 1 + c'_2 >= 6
    Y[2, 3, 20] = 0.0
    Y[3, 3, 20] = Y[0, 3, 20] * (0.6 + 0.5 * 4.2 ** 2)
    P = oracle.Problem(2, nx, ny, hex=True, bc_x=oracle.PERIODIC, bc_y=oracle.PERIODIC)
    _, st, reach = oracle.step(P, Y)
    assert reach > 5
    s = lbsd.Solver(2, nx, ny, lattice="hex", bc_x="periodic", bc_y="periodic")
    s.init_moments(Y, 1.0)
    s.step(1)
    with pytest.raises(lbsd.LBError) as ei:
        s.sync()
    assert ei.value.code == lbsd.LB_EREACH
    s.close()


def test_rejected_configurations(lbsd):
    with pytest.raises(lbsd.LBError):
        lbsd.Solver(2, 64, 8, lattice="hex", bc_x="reflecting")
    with pytest.raises(lbsd.LBError):
        lbsd.Solver(2, 64, 8, lattice="hex", gamma2=5.0 / 3.0)
