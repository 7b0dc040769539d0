"""Row chunks of the square lattice's short and full passes.

A tile whose windows take the slow paths is cut into chunks of rows that
different blocks march, each with its own halo rows; the tile's last chunk
adds the chunks' partial sums in chunk order.  Node values must not depend on
the cut: lb_step (which cuts tiles by the work measured in the previous step,
and the full pass's tiles by their count) is compared bit for bit with
lb_step_static, which never cuts, over many steps of smooth random fields
whose windows mix floor(v_x), floor(v_y) and c'_1 nearly everywhere (so most
tiles are cut from the second step on).  The totals of the cut run equal the
sums of its own moments to rounding, and two runs give the same totals bit
for bit.
"""
import numpy as np
import pytest

from paper_1602_02675_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def _state(nx, ny, seed):
    return inputs.random_state(seed, 2, nx, ny, vel=(-0.9, 0.9), e=(0.0, 1.5), smooth=3)


def _cut_run(lbsd, Y, n, prec, **kw):
    ny, nx = Y.shape[-2], Y.shape[-1]
    s = lbsd.Solver(2, nx, ny, precision=prec, **kw)
    s.init_moments(Y, 1.0)  # lambda = 1: lattice units are physical units
    s.step(n)
    out, tot = s.moments(), s.totals()
    s.close()
    return out, tot


def _uncut_run(lbsd, Y, n, prec, **kw):
    import torch

    ny, nx = Y.shape[-2], Y.shape[-1]
    dt = torch.float64 if prec == "fp64" else torch.float32
    s = lbsd.Solver(2, nx, ny, precision=prec, **kw)
    a = torch.tensor(Y.reshape(s.nf, ny, nx), dtype=dt, device="cuda")
    b = torch.empty_like(a)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    for i in range(n):
        s.step_static(a, b, status[i:i + 1])
        a, b = b, a
    torch.cuda.synchronize()
    out = a.double().cpu().numpy()
    st = status.cpu().numpy()
    s.close()
    return out, st


CASES = [  # nx, ny, seed, steps, precision, boundaries
    (700, 500, 1, 40, "fp64", {"bc_x": "transmissive", "bc_y": "periodic"}),
    (520, 333, 2, 30, "fp64", {"bc_x": "periodic", "bc_y": "transmissive"}),
    (700, 500, 3, 30, "fp32", {"bc_x": "periodic", "bc_y": "periodic"}),
]


@pytest.mark.parametrize("nx,ny,seed,n,prec,bcs", CASES)
def test_cut_tiles_equal_uncut(lbsd, nx, ny, seed, n, prec, bcs):
    Y = _state(nx, ny, seed)
    got, tot = _cut_run(lbsd, Y, n, prec, **bcs)
    want, st = _uncut_run(lbsd, Y, n, prec, **bcs)
    assert np.all(st == lbsd.LB_OK), st
    assert np.array_equal(got, want.reshape(got.shape)), (nx, ny, seed, prec)
    # the totals the chunks' slots add up to: the sums of the step's moments
    rtol = 1e-12 if prec == "fp64" else 1e-5
    np.testing.assert_allclose(tot, got.reshape(got.shape[0], -1).sum(axis=1)[:4], rtol=rtol, atol=1e-9 * nx * ny)
    tot2 = _cut_run(lbsd, Y, n, prec, **bcs)[1]
    assert np.array_equal(tot, tot2)
