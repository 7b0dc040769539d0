"""Seeded workload generators: determinism, ranges and the time-step rule."""
import math

import numpy as np
import pytest

from paper_1602_02675_amd import inputs


def test_steps_and_lambda_sod():
    # 1000 nodes to t = 0.2 with CFL 1 on the Sod states: max |u| + c = sqrt(1.4)
    n, lam = inputs.steps_and_lambda(0.2, 1e-3, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    assert n == 237 and lam == pytest.approx(0.2 / (237 * 1e-3))
    assert lam <= 1.0 / math.sqrt(1.4)
    n2, lam2 = inputs.steps_and_lambda(0.2, 1.0 / 800, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    assert n2 == 190


def test_riemann_instance_ranges_and_determinism():
    for seed in range(50):
        left, right, xd = inputs.riemann_instance(seed)
        assert left == (1.0, 0.0, 0.0, 1.0)
        rp = left[3] / right[3]
        rr = left[0] / right[0]
        assert 2.0 <= rp <= 100.0 and 1.0 <= rr <= 10.0 and 0.3 <= xd <= 0.7
        assert inputs.riemann_instance(seed) == (left, right, xd)


def test_tube_lengths_and_requests():
    L = inputs.tube_lengths(0)
    assert L.shape == (512,) and L.min() >= 256 and L.max() <= 65536
    assert np.array_equal(L, inputs.tube_lengths(0))
    reqs = inputs.serve_requests(1, 50, rate_per_s=10.0)
    t = [r["arrival"] for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert all(64 <= r["side"] <= 2048 and 100 <= r["steps"] <= 5000 for r in reqs)


def test_node_positions_cell_centred():
    x = inputs.node_x(4)
    assert np.allclose(x, [0.125, 0.375, 0.625, 0.875])


def test_random_state_physical():
    Y = inputs.random_state(0, 2, 33, 7, smooth=3)
    assert Y.shape == (4, 7, 33)
    rho = Y[0]
    assert np.all(rho > 0)
    e = Y[3] / rho - 0.5 * ((Y[1] / rho) ** 2 + (Y[2] / rho) ** 2)
    assert np.all(e >= -1e-12)


def test_quadrant_riemann_layout():
    states, (xc, yc) = inputs.quadrant_riemann(4)
    assert len(states) == 4 and 0.3 <= xc <= 0.7 and 0.3 <= yc <= 0.7
    for rho, u, v, p in states:
        assert 0.1 <= rho <= 1.0 and 0.05 <= p <= 1.0 and math.hypot(u, v) <= 0.3
    nx, ny = 50, 40
    Y = inputs.quadrant_moments(states, (xc, yc), nx, ny)
    x = inputs.node_x(nx)
    y = (np.arange(ny) + 0.5) / nx
    for j in (0, ny - 1):
        for i in (0, nx - 1):
            k = int(x[i] >= xc) + 2 * int(y[j] >= yc)
            rho, u, v, p = states[k]
            assert Y[0, j, i] == rho and Y[1, j, i] == rho * u and Y[2, j, i] == rho * v
            assert Y[3, j, i] == pytest.approx(p / 0.4 + 0.5 * rho * (u * u + v * v), rel=1e-15)
    lam = inputs.quadrant_lambda(states)
    assert lam == pytest.approx(1.0 / max(math.hypot(u, v) + math.sqrt(1.4 * p / r) for r, u, v, p in states))
