"""Seeded synthetic inputs (workload shapes and states), shared by tests and bench.

This module holds none of the method's arithmetic: it draws states, sizes and
arrival times, and applies the time-step rule.  Every generator uses numpy's
PCG64 (``np.random.default_rng(seed)``) with a fixed draw order.

Workloads (the paper measures no dataset; its only input is Sod's shock tube,
Sec. V.C, with u = 0 on both sides):

* ``sod``: rho_L = 1, p_L = 1, rho_R = 0.125, p_R = 0.1, u = v = 0.
* ``riemann_instance(seed)``: rho_L = 1, p_L = 1, u = 0;
  p_R = p_L / r_p with log10 r_p ~ U[log10 2, 2]; rho_R = rho_L / r_rho with
  r_rho ~ U[1, 10]; diaphragm x_d ~ U[0.3, 0.7].
* ``tube_lengths(seed, n)``: round(exp(U[ln 256, ln 65536])).
* ``serve_requests(seed, n)``: square sides round(exp(U[ln 64, ln 2048])),
  steps ~ U{100..5000}, states as ``riemann_instance``, exponential
  inter-arrival gaps.
* ``quadrant_riemann(seed)``: a 2-D Riemann problem of four seeded
  constant states (non-planar data for the square lattice).
* ``random_state(seed, ...)``: random positive-density moment fields in
  lattice units, for index and field parity.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4

SOD_LEFT = (1.0, 0.0, 0.0, 1.0)      # (rho, u, v, p)
SOD_RIGHT = (0.125, 0.0, 0.0, 0.1)


def node_x(nx: int, x_lo: float = 0.0, x_hi: float = 1.0) -> np.ndarray:
    """Cell-centred node positions x_i = x_lo + (i + 1/2) dx."""
    dx = (x_hi - x_lo) / nx
    return x_lo + (np.arange(nx, dtype=np.float64) + 0.5) * dx


def max_signal_speed(states, gamma: float = GAMMA) -> float:
    """max over the given primitive states of |u| + sqrt(gamma p / rho)."""
    return max(abs(u) + math.sqrt(gamma * p / rho) for (rho, u, _v, p) in states)


def steps_and_lambda(t_end: float, dx: float, states, cfl: float = 1.0, gamma: float = GAMMA):
    """Time-step rule: lambda = dt/dx from the CFL bound of the initial states,
    n = ceil(t_end / (lambda dx)), then lambda := t_end / (n dx) so that n
    steps end exactly at t_end."""
    lam = cfl / max_signal_speed(states, gamma)
    n = int(math.ceil(t_end / (lam * dx) - 1e-12))
    return n, t_end / (n * dx)


def cfl_lambda(states, cfl: float = 1.0, gamma: float = GAMMA) -> float:
    return cfl / max_signal_speed(states, gamma)


def riemann_instance(seed: int):
    """(left, right, x_d) of one seeded planar shock tube."""
    rng = np.random.default_rng(seed)
    log_rp = rng.uniform(math.log10(2.0), 2.0)
    r_rho = rng.uniform(1.0, 10.0)
    x_d = rng.uniform(0.3, 0.7)
    left = (1.0, 0.0, 0.0, 1.0)
    right = (1.0 / r_rho, 0.0, 0.0, 1.0 / (10.0 ** log_rp))
    return left, right, float(x_d)


def tube_lengths(seed: int, n: int = 512, lo: int = 256, hi: int = 65536) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))).astype(np.int64)


def serve_requests(seed: int, n: int, rate_per_s: float, side_lo: int = 64, side_hi: int = 2048,
                   steps_lo: int = 100, steps_hi: int = 5000):
    """List of dicts: arrival time, side, steps, Riemann states."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    sides = np.rint(np.exp(rng.uniform(math.log(side_lo), math.log(side_hi), size=n))).astype(np.int64)
    steps = rng.integers(steps_lo, steps_hi + 1, size=n)
    state_seeds = rng.integers(0, 2**31 - 1, size=n)
    out = []
    t = 0.0
    for i in range(n):
        t += float(gaps[i])
        left, right, x_d = riemann_instance(int(state_seeds[i]))
        out.append(dict(arrival=t, side=int(sides[i]), steps=int(steps[i]),
                        left=left, right=right, x_d=x_d))
    return out


def quadrant_riemann(seed: int):
    """A seeded 2-D Riemann problem: four constant states meeting at (x_c, y_c)
    in the unit square.  Each state has rho log-uniform in [0.1, 1], p
    log-uniform in [0.05, 1] and a velocity of modulus up to 0.3 in a random
    direction; x_c, y_c ~ U[0.3, 0.7].  Returns (states, (x_c, y_c)) with
    states ordered lower-left, lower-right, upper-left, upper-right."""
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        rho = float(np.exp(rng.uniform(math.log(0.1), 0.0)))
        p = float(np.exp(rng.uniform(math.log(0.05), 0.0)))
        sp, ang = rng.uniform(0.0, 0.3), rng.uniform(0.0, 2.0 * math.pi)
        states.append((rho, float(sp * math.cos(ang)), float(sp * math.sin(ang)), p))
    xc, yc = rng.uniform(0.3, 0.7, size=2)
    return states, (float(xc), float(yc))


def quadrant_moments(states, center, nx: int, ny: int, gamma: float = GAMMA) -> np.ndarray:
    """Conserved moments [4, ny, nx] (physical units) of a quadrant problem on
    cell-centred nodes of [0, 1] x [0, ny/nx] (dy = dx)."""
    x = node_x(nx)
    y = (np.arange(ny, dtype=np.float64) + 0.5) / nx
    X, Yy = np.meshgrid(x, y)
    Y = np.zeros((4, ny, nx))
    for k, (rho, u, v, p) in enumerate(states):
        right, upper = k & 1, k >> 1
        m = ((X >= center[0]) == bool(right)) & ((Yy >= center[1]) == bool(upper))
        Y[0][m] = rho
        Y[1][m] = rho * u
        Y[2][m] = rho * v
        Y[3][m] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return Y


def quadrant_lambda(states, cfl: float = 1.0, gamma: float = GAMMA) -> float:
    """lambda = cfl / max(|v| + sqrt(gamma p / rho)) over the four states."""
    return cfl / max(math.hypot(u, v) + math.sqrt(gamma * p / rho) for (rho, u, v, p) in states)


def random_state(seed: int, dim: int, nx: int, ny: int = 1, *, rho=(0.2, 2.0), vel=(-1.8, 1.8),
                 e=(0.0, 3.0), smooth: int = 0) -> np.ndarray:
    """Random moment field [nf, ny, nx] in lattice units.

    rho, each velocity component and e are drawn uniformly in the given
    ranges (optionally box-smoothed over ``smooth`` neighbours along x to
    give piecewise-smooth fields); the moments are rho, rho*v, rho*(e + |v|^2/2).
    """
    rng = np.random.default_rng(seed)
    ny = ny if dim == 2 else 1
    shp = (ny, nx)
    r = rng.uniform(*rho, size=shp)
    vs = [rng.uniform(*vel, size=shp) for _ in range(dim)]
    ee = rng.uniform(*e, size=shp)
    if smooth > 0:
        k = np.ones(smooth) / smooth
        def sm(a):
            return np.stack([np.convolve(np.pad(row, (smooth, smooth), mode="wrap"), k, "same")[smooth:-smooth]
                             for row in a])
        r, ee = sm(r), sm(ee)
        vs = [sm(v) for v in vs]
    Y = np.zeros((dim + 2, ny, nx))
    Y[0] = r
    v2 = np.zeros(shp)
    for a, v in enumerate(vs):
        Y[1 + a] = r * v
        v2 = v2 + v * v
    Y[-1] = r * (ee + 0.5 * v2)
    return Y
