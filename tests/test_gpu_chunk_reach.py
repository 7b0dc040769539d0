"""Packets that cross a row-chunk boundary from beyond the short FIFO.

The square-lattice march computes every tile first with a short y-FIFO that
stages only 3 halo rows on each side of the tile's destination rows.  A
source 4 or 5 rows outside the tile can still reach its edge rows (c'_1 = 2
with a fractional v_y, eq. 29 corners): then the neighbouring row chunk,
which holds that source, has to send the tile to the full pass.  These cases
build tubes along y with hot bands (c'_1 = 2) that end 4 rows from a chunk
boundary, in both directions, while the chunks across the boundary are cold
(c'_1 = 1) and complete in the short pass.  Parity with the oracle at the
FP64 bar (rows are uniform along x; 16-row chunks on these sizes).
"""
import numpy as np
import pytest

import oracle

from parity_helpers import TOL64, normwise_err

GAMMA = 1.4
E_COLD, E_HOT = 2.5, 6.25  # A = 2 (gamma - 1) e = 2 (c'_1 = 1) and 5 (c'_1 = 2), lattice units
SY = 16                    # destination rows per tile on grids this small (the strip height's floor)


def band_state(nx, ny, bands, v_cold=0.3, seed=None):
    """Physical moments with lambda = 1: rho = 1, v_x = 0, rows cold with
    v_y = v_cold except the hot bands [(y0, y1, v_y), ...].  seed: small
    smooth perturbations along x (rows then differ from each other)."""
    rho = np.ones((ny, nx))
    vy = np.full((ny, nx), v_cold)
    e = np.full((ny, nx), E_COLD)
    for y0, y1, v in bands:
        for y in range(y0, y1):
            vy[y % ny] = v
            e[y % ny] = E_HOT
    vx = np.zeros((ny, nx))
    if seed is not None:
        rng = np.random.default_rng(seed)
        k = np.ones(7) / 7.0
        for a in (rho, vx, vy, e):
            n = rng.uniform(-1.0, 1.0, size=(ny, nx))
            n = np.apply_along_axis(lambda r: np.convolve(np.concatenate([r[-3:], r, r[:3]]), k, "valid"), 1, n)
            a += (0.02 if a is rho else 0.04) * n
    Y = np.empty((4, ny, nx))
    Y[0] = rho
    Y[1] = rho * vx
    Y[2] = rho * vy
    Y[3] = rho * (e + 0.5 * (vx * vx + vy * vy))
    return Y


# (ny, bands, bc_y): hot rows [35, 40) move down (floor v_y = -1: row 35
# reaches row 31 of chunk [16, 32), which stages rows up to 34) and [40, 45)
# up (row 44 reaches row 48 of chunk [48, 64), which stages rows from 45);
# on 49 rows, periodic, the hot rows [3, 8) move down across the wrap into
# the one-row last chunk [48, 49), which stages rows 45 .. 2 (mod 49).
CASES = [
    (64, [(35, 40, -0.3), (40, 45, 0.3)], "periodic"),
    (64, [(35, 40, -0.3), (40, 45, 0.3)], "transmissive"),
    (64, [(35, 40, -0.3), (40, 45, 0.3)], "reflecting"),
    (49, [(3, 8, -0.3)], "periodic"),
]
BC = {"transmissive": oracle.TRANSMISSIVE, "periodic": oracle.PERIODIC, "reflecting": oracle.REFLECTING}


def test_band_layout_reaches_past_short_fifo():
    """The premise of the GPU cases (CPU): each band edge's source has
    c'_1 = 2 and the floor(v_y) that carries a packet 4 rows across the chunk
    boundary with non-zero mass, and every row the neighbouring chunk stages
    is cold (y-reach <= 3, so that chunk completes in the short pass)."""
    for ny, bands, bc in CASES:
        P = oracle.Problem(2, 64, ny, bc_y=BC[bc])
        Y = oracle.to_lattice(P, band_state(64, ny, bands), 1.0)
        fx, fy, c1 = oracle.lanes(P, Y)
        reach = np.maximum(fy + 2 + c1, c1 + 1 - fy)  # largest |y displacement| of a node's packets
        if ny == 64:
            assert c1[35, 0] == 2 and fy[35, 0] == -1  # reaches 35 - 1 - 3 = 31
            assert c1[44, 0] == 2 and fy[44, 0] == 0   # reaches 44 + 1 + 3 = 48 (k_y = 1, r_y = 0.3)
            assert np.all(reach[13:35] <= 3) and np.all(reach[45:64] <= 3)
        else:
            assert c1[3, 0] == 2 and fy[3, 0] == -1    # reaches 3 - 4 = -1, i.e. row 48
            assert np.all(reach[45:49] <= 3) and np.all(reach[0:3] <= 3)


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


@pytest.mark.gpu
@pytest.mark.parametrize("ny,bands,bc", CASES)
@pytest.mark.parametrize("perturb", [None, 11])
def test_hot_band_across_chunk_boundary(lbsd, ny, bands, bc, perturb):
    nx = 64
    Y = band_state(nx, ny, bands, seed=perturb)
    P = oracle.Problem(2, nx, ny, bc_x=oracle.PERIODIC, bc_y=BC[bc])
    s = lbsd.Solver(2, nx, ny, bc_x="periodic", bc_y=bc)
    s.init_moments(Y, 1.0)
    Yl = oracle.to_lattice(P, Y, 1.0)
    done = 0
    for n in (1, 2, 5):
        ref, st, reach = oracle.run(P, Yl, n)
        assert st == 0 and reach <= 5
        s.step(n - done)
        done = n
        got = s.moments()
        err = normwise_err(got, oracle.from_lattice(P, ref, 1.0), 2)
        assert err <= TOL64, (ny, bc, perturb, n, err)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hot_band_across_chunk_boundary_pool(lbsd, prec):
    """The same layouts as pool slots, next to each other in one pool: each
    slot equals its solver run bit for bit, and the FP64 slots the oracle."""
    steps = 5
    pool = lbsd.Pool(2, 8, 64 << 20, precision=prec)
    slots, refs = [], []
    for i, (ny, bands, bc) in enumerate(CASES):
        Y = band_state(64, ny, bands, seed=None if i % 2 == 0 else 11)
        s = lbsd.Solver(2, 64, ny, bc_x="periodic", bc_y=bc, precision=prec)
        s.init_moments(Y, 1.0)
        s.step(steps)
        refs.append(s.moments())
        s.close()
        slots.append(pool.admit_moments(Y, 1.0, steps, bc_x="periodic", bc_y=bc))
        if prec == "fp64":
            P = oracle.Problem(2, 64, ny, bc_x=oracle.PERIODIC, bc_y=BC[bc])
            ref, st, _ = oracle.run(P, oracle.to_lattice(P, Y, 1.0), steps)
            assert normwise_err(refs[-1], oracle.from_lattice(P, ref, 1.0), 2) <= TOL64
    pool.advance(steps + 2)
    for sl, ref in zip(slots, refs):
        assert pool.poll(sl) == (steps, 1)
        assert np.array_equal(pool.moments(sl), ref)
    pool.close()
