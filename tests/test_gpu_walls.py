"""GPU parity of reflecting walls against the oracle, through the C ABI.

The oracle reflects each packet that crosses a wall face (specular: landing
-1 - i / 2n - 1 - i, normal momentum negated); the HIP path instead reads the
halo sources beyond a wall as mirror images of the nodes inside (normal
momentum negated) and drops packets that leave.  The two agree because the
step is mirror-symmetric; only rounding differs, so the parity bar is the
usual one (FP64 1e-12 normwise; FP32 relative L1 density 1e-5).
"""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs

from parity_helpers import TOL64, normwise_err, run_pair, self_divergence

pytestmark = pytest.mark.gpu

W = oracle.REFLECTING


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def _rel_l1(got, ref):
    return float(np.sum(np.abs(got[0] - ref[0])) / np.sum(np.abs(ref[0])))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sod_closed_tube_1d(lbsd, prec):
    """Sod between two walls, 1000 nodes, 600 steps (t = 0.51): the shock
    reflects off the right wall and the rarefaction off the left one."""
    nx = 1000
    n0, lam = inputs.steps_and_lambda(0.2, 1.0 / nx, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    n = 600
    P = oracle.Problem(1, nx, bc_x=W)
    Y0 = oracle.riemann_moments(P, inputs.node_x(nx), inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5)
    ref, st, _ = oracle.run(P, oracle.to_lattice(P, Y0, lam), n)
    assert st == 0
    ref = oracle.from_lattice(P, ref, lam)
    s = lbsd.Solver(1, nx, precision=prec, bc_x="reflecting")
    s.init_riemann(0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, lam=lam)
    s.step(n)
    got = s.moments()
    if prec == "fp64":
        assert normwise_err(got, ref, 1) <= TOL64
    else:
        assert _rel_l1(got, ref) <= 1e-5
    # closed tube: mass and energy stay what they were
    t0 = oracle.totals(P, Y0)
    tot = s.totals()
    rt = 1e-13 if prec == "fp64" else 1e-6
    assert tot[0] == pytest.approx(t0[0], rel=rt)
    assert tot[3] == pytest.approx(t0[2], rel=rt)
    # the reflected shock has come back: the walls changed the solution
    Pt = oracle.Problem(1, nx)
    open_end, _, _ = oracle.run(Pt, oracle.to_lattice(Pt, Y0, lam), n)
    assert normwise_err(oracle.from_lattice(Pt, open_end, lam), ref, 1) > 1e-2
    s.close()


@pytest.mark.parametrize("nx", [5, 6, 777, 2049])
def test_random_1d_walls(lbsd, nx):
    """Random states (both velocity signs at the walls); nx = 5 is the
    smallest grid whose mirror images cover the halo."""
    for smooth, seed in ((9, 21), (0, 22)):
        Y = inputs.random_state(seed, 1, nx, vel=(-1.3, 1.3), e=(0.0, 1.5), smooth=smooth if nx > 9 else 0)
        P, ref, got, s = run_pair(lbsd, 1, Y, 1.0, 12, nx=nx, bcx=W)
        assert normwise_err(got, ref, 1) <= TOL64, (nx, smooth)
        s.close()


@pytest.mark.parametrize("shape", [(5, 5), (70, 37), (300, 9)])
@pytest.mark.parametrize("bcs", [(W, 1), (0, W), (W, W), (W, 0), (1, W)])
def test_random_2d_walls(lbsd, shape, bcs):
    nx, ny = shape
    for smooth, seed in ((5, 23), (0, 24)):
        Y = inputs.random_state(seed, 2, nx, ny, vel=(-1.1, 1.1), e=(0.0, 1.2), smooth=smooth if nx > 5 else 0)
        P, ref, got, s = run_pair(lbsd, 2, Y, 1.0, 4, nx=nx, ny=ny, bcx=bcs[0], bcy=bcs[1])
        assert normwise_err(got, ref, 2) <= TOL64, (shape, bcs, smooth)
        s.close()


def test_random_2d_hot_walls(lbsd):
    """c'_1 up to 2 next to the walls: tiles recomputed with the full y-FIFO
    read mirrored rows too."""
    nx, ny = 150, 77
    Y = inputs.random_state(25, 2, nx, ny, vel=(-0.9, 0.9), e=(0.0, 7.0), smooth=3)
    P, ref, got, s = run_pair(lbsd, 2, Y, 1.0, 3, nx=nx, ny=ny, bcx=W, bcy=W)
    assert normwise_err(got, ref, 2) <= TOL64
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_planar_sod_2d_walls(lbsd, prec):
    """Planar Sod on 300 x 64 with walls at both x ends and periodic y, 200
    steps (the shock has reflected): rows stay bit-identical and match the
    oracle on a 300 x 4 strip (transmissive y keeps its rows identical)."""
    nx, ny = 300, 64
    n0, lam = inputs.steps_and_lambda(0.2, 1.0 / nx, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    n = 200
    P = oracle.Problem(2, nx, 4, bc_x=W, bc_y=oracle.TRANSMISSIVE)
    Y0 = oracle.riemann_moments(P, inputs.node_x(nx), inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5)
    ref, st, _ = oracle.run(P, oracle.to_lattice(P, Y0, lam), n)
    assert st == 0
    ref = oracle.from_lattice(P, ref, lam)
    s = lbsd.Solver(2, nx, ny, precision=prec, bc_x="reflecting", bc_y="periodic")
    s.init_riemann(0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, lam=lam)
    s.step(n)
    got = s.moments()
    assert np.all(got == got[:, :1, :])
    if prec == "fp64":
        assert normwise_err(got[:, :4, :], ref, 2) <= TOL64
    else:
        assert _rel_l1(got[:, :4, :], ref) <= 1e-5
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32", 2e-4)])
def test_quadrant_closed_box(lbsd, prec, tol):
    """A four-state 2-D Riemann problem in a box with four walls: 10 steps at
    the parity bar; 30 steps (waves at the walls) within 4x the oracle's own
    sensitivity to rounding-level input changes; mass and energy conserved."""
    nx, ny = 97, 83
    states, center = inputs.quadrant_riemann(3)
    lam = inputs.quadrant_lambda(states)
    Y = inputs.quadrant_moments(states, center, nx, ny)
    P, ref, got, s = run_pair(lbsd, 2, Y, lam, 10, nx=nx, ny=ny, bcx=W, bcy=W, prec=prec)
    assert normwise_err(got, ref, 2) <= tol
    if prec == "fp32":
        assert _rel_l1(got, ref) <= 1e-5
    s.close()
    if prec == "fp64":
        P, ref, got, s = run_pair(lbsd, 2, Y, lam, 30, nx=nx, ny=ny, bcx=W, bcy=W, prec=prec)
        sens = self_divergence(P, oracle.to_lattice(P, Y, lam), 30)
        assert normwise_err(got, ref, 2) <= max(TOL64, 4.0 * sens)
        t0 = oracle.totals(P, Y)
        tot = s.totals()
        assert tot[0] == pytest.approx(t0[0], rel=1e-13)
        assert tot[3] == pytest.approx(t0[3], rel=1e-13)
        s.close()
