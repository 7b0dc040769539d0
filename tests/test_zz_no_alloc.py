"""lb_step_static, the allocation-free step, against lb_step.

lb_step_static takes the step's scratch from a static device array instead
of the solver's bound buffer; the kernels are the same.  Each case compares
its output with lb_step's for the same state and step count, bit for bit
(the parity bar for the same kernels on the same inputs), in two calls in a
row where the second has a smaller input, so that it runs on the scratch
the first left behind.
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


def _state(dim, nx, ny, seed, hot=False):
    e = (0.0, 6.0) if hot else (0.0, 1.5)
    return inputs.random_state(seed, dim, nx, ny, vel=(-0.9, 0.9), e=e, smooth=3 if nx > 3 else 0)


def _lb_step(lbsd, dim, Y, n, prec, **kw):
    """n steps of lb_step from Y (lambda = 1: lattice units = physical)."""
    ny, nx = Y.shape[-2], Y.shape[-1]
    s = lbsd.Solver(dim, nx, ny, precision=prec, **kw)
    s.init_moments(Y, 1.0)
    s.step(n)
    out = s.moments()
    s.close()
    return out


def _static_steps(lbsd, dim, Y, n, prec, **kw):
    """n steps of lb_step_static, alternating two device buffers; also the
    status code each step wrote."""
    import torch

    ny, nx = Y.shape[-2], Y.shape[-1]
    dt = torch.float64 if prec == "fp64" else torch.float32
    s = lbsd.Solver(dim, nx, ny, precision=prec, **kw)
    a = torch.tensor(Y.reshape(s.nf, ny, nx), dtype=dt, device="cuda")
    b = torch.empty_like(a)
    status = torch.full((max(n, 1),), 99, dtype=torch.int32, device="cuda")
    for i in range(n):
        s.step_static(a, b, status[i:i + 1])
        a, b = b, a
    torch.cuda.synchronize()
    out = a.double().cpu().numpy()
    s.close()
    return out, status.cpu().numpy()[:n]


CASES = [  # (dim, first (nx, ny, seed, hot), second, smaller (nx, ny, seed, hot), boundaries)
    (2, (300, 200, 3, True), (70, 37, 4, False), {"bc_x": "transmissive", "bc_y": "periodic"}),
    (2, (257, 129, 5, False), (33, 17, 6, True), {"bc_x": "reflecting", "bc_y": "reflecting"}),
    (1, (100_000, 1, 7, True), (1025, 1, 8, False), {"bc_x": "transmissive"}),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,first,second,bcs", CASES)
def test_static_step_equals_lb_step(lbsd, prec, dim, first, second, bcs):
    for nx, ny, seed, hot in (first, second):
        Y = _state(dim, nx, ny, seed, hot)
        for n in (1, 3):
            want = _lb_step(lbsd, dim, Y, n, prec, **bcs)
            got, st = _static_steps(lbsd, dim, Y, n, prec, **bcs)
            assert np.all(st == lbsd.LB_OK), st
            assert np.array_equal(got, want.reshape(got.shape)), (prec, dim, nx, ny, n)


def test_static_step_two_gases(lbsd):
    """The two-gas instances (species field) through the same entry point."""
    Y = _state(2, 120, 40, 9)
    rng = np.random.default_rng(9)
    chi = np.clip(rng.random((40, 120)), 0.0, 1.0)
    Y5 = np.concatenate([Y, (Y[0] * chi)[None]], axis=0)
    want = _lb_step(lbsd, 2, Y5, 3, "fp64", gamma2=5.0 / 3.0)
    got, st = _static_steps(lbsd, 2, Y5, 3, "fp64", gamma2=5.0 / 3.0)
    assert np.all(st == 0)
    assert np.array_equal(got, want)


def test_static_step_reports_reach(lbsd):
    """A state whose packets move past the halo: the status says LB_EREACH,
    as lb_step reports it, and the input is untouched."""
    import torch

    nx = 2000
    Y = _state(1, nx, 1, 10)
    Y[1] = Y[0] * 6.5  # v = 6.5: a packet moves 6 + 1 + c'_2 > 5 nodes
    Y[2] = Y[0] * (1.0 + 0.5 * 6.5 ** 2)
    s = lbsd.Solver(1, nx)
    a = torch.tensor(Y.reshape(3, 1, nx), dtype=torch.float64, device="cuda")
    keep = a.clone()
    b = torch.empty_like(a)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    s.step_static(a, b, status)
    torch.cuda.synchronize()
    assert int(status.item()) == lbsd.LB_EREACH
    assert torch.equal(a, keep)
    s.close()


def test_static_step_rejects(lbsd):
    """Sizes beyond the static scratch, overlapping or host buffers."""
    import torch

    import ctypes

    nx = 40_000_000  # 39 K partial rows of 64 bytes: more than 2 MiB (a handle that is never bound)

    g = lbsd.lb_grid(1, nx, 1, 0.0, 1.0, 0, 1)
    vs = lbsd.lb_velset(lbsd.LB_LATTICE_D1_TRIPLE, 0.5)
    h = ctypes.c_void_p()
    assert lbsd._lib.lb_create(ctypes.byref(g), 1.4, ctypes.byref(vs), lbsd.LB_FP32, ctypes.byref(h)) == 0
    a = torch.zeros((3, nx), dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    rc = lbsd._lib.lb_step_static(h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), None, None)
    assert rc == lbsd.LB_EINVAL and b"scratch" in lbsd._lib.lb_last_error()
    rc = lbsd._lib.lb_step_static(h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr() + 256), None, None)
    assert rc == lbsd.LB_EINVAL
    host = np.zeros((3, nx), dtype=np.float32)
    rc = lbsd._lib.lb_step_static(h, ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(b.data_ptr()), None, None)
    assert rc == lbsd.LB_EINVAL
    lbsd._lib.lb_destroy(h)
