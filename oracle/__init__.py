"""Plain FP64 CPU oracle of the semi-discrete lattice Boltzmann step (tau = 1).

TEST INFRASTRUCTURE ONLY.  The product path never imports this package: only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP library.

* ``lb_oracle.c`` -- one step as a literal scatter (Sec. III.B, IV, V.A-B of
  the paper), compiled by :func:`build` with gcc into ``liboracle.so``.
* :mod:`oracle.riemann` -- the exact Riemann solution of the Euler equations
  (the analytical Sod solution the paper compares against, Sec. V.C-D).

Everything here works in lattice units (dx = dt = 1); :func:`to_lattice` and
:func:`from_lattice` convert with lambda = dt_phys / dx_phys (velocity scales
by lambda, energy per unit mass by lambda**2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TRANSMISSIVE = 0
PERIODIC = 1
REFLECTING = 2


def build() -> str:
    """Compile the C oracle (always recompiles)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_long), ("ny", ctypes.c_long),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("gamma", ctypes.c_double), ("delta0", ctypes.c_double),
                ("species", ctypes.c_int), ("gamma2", ctypes.c_double), ("hex", ctypes.c_int)]


class _Levels(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int), ("rho", ctypes.c_double),
                ("v", ctypes.c_double * 2), ("E", ctypes.c_double), ("e", ctypes.c_double),
                ("phi", ctypes.c_double), ("A", ctypes.c_double),
                ("c1", ctypes.c_int), ("c2", ctypes.c_int),
                ("d0", ctypes.c_double), ("d1", ctypes.c_double), ("d2", ctypes.c_double),
                ("b0", ctypes.c_int), ("b1", ctypes.c_int), ("b2", ctypes.c_int),
                ("f", ctypes.c_int * 2), ("vp0", ctypes.c_double * 2),
                ("vp1", ctypes.c_double * 2), ("chi", ctypes.c_double), ("gm1", ctypes.c_double),
                ("r", ctypes.c_double * 2), ("tri", ctypes.c_int)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P, D, I = ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.oc_levels_of.argtypes = [P, D, ctypes.POINTER(_Levels)]
    lib.oc_levels_of.restype = ctypes.c_int
    lib.oc_packets.argtypes = [P, D, I, D]
    lib.oc_packets.restype = ctypes.c_int
    lib.oc_step.argtypes = [P, D, D, I]
    lib.oc_step.restype = ctypes.c_int
    lib.oc_run.argtypes = [P, D, ctypes.c_long, I]
    lib.oc_run.restype = ctypes.c_int
    lib.oc_totals.argtypes = [P, D, D]
    lib.oc_totals.restype = None
    lib.oc_lanes.argtypes = [P, D, I, I, I]
    lib.oc_lanes.restype = None
    _lib = lib
    return lib


class Problem:
    """Lattice, grid, boundaries and gas of one oracle problem."""

    def __init__(self, dim: int, nx: int, ny: int = 1, *, gamma: float = 1.4,
                 delta0: float | None = None, bc_x: int = TRANSMISSIVE, bc_y: int = PERIODIC,
                 gamma2: float | None = None, hex: bool = False):
        """gamma2: a second gas (gamma of gas 2, gamma of gas 1); the state
        then has a species field rho chi (mass of gas 1) after rho E.
        hex (dim 2): the hexagonal lattice of Fig. 1, nodes at i e_1 + j e_2
        with e_1 = (1, 0), e_2 = (1/2, sqrt(3)/2), stored [.][j][i]; bc_x and
        bc_y then apply to the axial indices i and j."""
        if delta0 is None:
            delta0 = 0.5 if dim == 1 else 0.0
        self.dim, self.nx, self.ny = dim, int(nx), int(ny if dim == 2 else 1)
        self.gamma, self.delta0, self.bc_x, self.bc_y = float(gamma), float(delta0), bc_x, bc_y
        self.species = gamma2 is not None
        self.gamma2 = float(gamma2) if self.species else self.gamma
        self.hex = bool(hex) and dim == 2
        self._c = _Problem(dim, self.nx, self.ny, bc_x, bc_y, self.gamma, self.delta0,
                           1 if self.species else 0, self.gamma2, 1 if self.hex else 0)

    @property
    def ie(self) -> int:
        """Index of the energy field rho E."""
        return self.dim + 1

    @property
    def nf(self) -> int:
        return self.dim + 2 + (1 if self.species else 0)

    @property
    def shape(self):
        return (self.nf, self.ny, self.nx)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def levels(P: Problem, node) -> dict:
    """Equilibrium of one node: v, e, phi, A, c'_1, c'_2, d_0, d_1, d_2, floor(v)."""
    lib = _load()
    y = np.ascontiguousarray(node, dtype=np.float64)
    L = _Levels()
    lib.oc_levels_of(ctypes.byref(P._c), _dptr(y), ctypes.byref(L))
    return dict(valid=L.valid, rho=L.rho, v=tuple(L.v[: P.dim]), E=L.E, e=L.e, phi=L.phi,
                A=L.A, c1=L.c1, c2=L.c2, d0=L.d0, d1=L.d1, d2=L.d2, b=(L.b0, L.b1, L.b2),
                f=tuple(L.f[: P.dim]), vp0=tuple(L.vp0[: P.dim]), vp1=tuple(L.vp1[: P.dim]),
                chi=L.chi, gm1=L.gm1, r=tuple(L.r[: P.dim]), tri=L.tri)


def packets(P: Problem, node):
    """All packets of one node: (offsets [n, 2] int, payload [n, nf] = m, m*xi, m*zeta)."""
    lib = _load()
    y = np.ascontiguousarray(node, dtype=np.float64)
    off = np.zeros((40, 2), dtype=np.int32)  # at most 39 packets (hexagonal lattice with a rest level)
    pay = np.zeros(40 * 5, dtype=np.float64)
    n = lib.oc_packets(ctypes.byref(P._c), _dptr(y), _iptr(off), _dptr(pay))
    return off[:n].copy(), pay[: n * P.nf].reshape(n, P.nf).copy()


def _as_state(P: Problem, Y) -> np.ndarray:
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(P.shape)
    return Y.copy()


def step(P: Problem, Y):
    """One step; returns (Y_new, status, max_reach)."""
    lib = _load()
    Y = _as_state(P, Y)
    out = np.empty_like(Y)
    reach = ctypes.c_int(0)
    st = lib.oc_step(ctypes.byref(P._c), _dptr(Y), _dptr(out), ctypes.byref(reach))
    return out, st, reach.value


def run(P: Problem, Y, nsteps: int):
    """nsteps steps; returns (Y, status, max_reach)."""
    lib = _load()
    Y = _as_state(P, Y)
    reach = ctypes.c_int(0)
    st = lib.oc_run(ctypes.byref(P._c), _dptr(Y), int(nsteps), ctypes.byref(reach))
    return Y, st, reach.value


def totals(P: Problem, Y) -> np.ndarray:
    lib = _load()
    Y = _as_state(P, Y)
    out = np.zeros(P.nf, dtype=np.float64)
    lib.oc_totals(ctypes.byref(P._c), _dptr(Y), _dptr(out))
    return out


def lanes(P: Problem, Y):
    """Per-node (floor v_x, floor v_y, c'_1) of a whole field."""
    lib = _load()
    Y = _as_state(P, Y)
    n = P.nx * P.ny
    fx, fy, c1 = (np.zeros(n, dtype=np.int32) for _ in range(3))
    lib.oc_lanes(ctypes.byref(P._c), _dptr(Y), _iptr(fx), _iptr(fy), _iptr(c1))
    shp = (P.ny, P.nx)
    return fx.reshape(shp), fy.reshape(shp), c1.reshape(shp)


def riemann_moments(P: Problem, x, prim_left, prim_right, x_d: float) -> np.ndarray:
    """Conserved moments (physical units) of a Riemann initial state.

    prim_* = (rho, u, v, p); node i is on the left iff x_i < x_d.  The total
    energy follows from the equation of state p = (gamma - 1) rho e (eq. 27).
    """
    left = np.asarray(x) < x_d
    Y = np.zeros(P.shape)
    # with two gases, gas 1 (gamma) fills the left side and gas 2 (gamma2) the right
    for side, (rho, u, v, p), g, chi in ((left, prim_left, P.gamma, 1.0), (~left, prim_right, P.gamma2, 0.0)):
        rE = p / (g - 1.0) + 0.5 * rho * (u * u + v * v)
        cols = np.nonzero(side)[0]
        Y[0][:, cols] = rho
        Y[1][:, cols] = rho * u
        if P.dim == 2:
            Y[2][:, cols] = rho * v
        Y[P.ie][:, cols] = rE
        if P.species:
            Y[P.ie + 1][:, cols] = rho * chi
    return Y


def to_lattice(P: Problem, Y, lam: float) -> np.ndarray:
    """Physical -> lattice units: rho*v scales by lambda, rho*E by lambda**2."""
    Y = np.array(Y, dtype=np.float64).reshape(P.shape)
    lam2 = lam * lam
    Y[1:1 + P.dim] *= lam
    Y[P.ie] *= lam2
    return Y


def from_lattice(P: Problem, Y, lam: float) -> np.ndarray:
    Y = np.array(Y, dtype=np.float64).reshape(P.shape)
    lam2 = lam * lam
    Y[1:1 + P.dim] /= lam
    Y[P.ie] /= lam2
    return Y


def primitives(P: Problem, Y_phys) -> dict:
    """rho, u, (v), e, p (and chi with two gases) from physical-unit moments
    (Sec. V.D outputs); p uses the node's gas."""
    Y = np.asarray(Y_phys).reshape(P.shape)
    rho = Y[0]
    u = Y[1] / rho
    v = Y[2] / rho if P.dim == 2 else np.zeros_like(u)
    e = Y[P.ie] / rho - 0.5 * (u * u + v * v)
    out = dict(rho=rho, u=u, v=v, e=e)
    gm1 = P.gamma - 1.0
    if P.species:
        chi = np.clip(Y[P.ie + 1] / rho, 0.0, 1.0)
        gm1 = 1.0 / (chi / (P.gamma - 1.0) + (1.0 - chi) / (P.gamma2 - 1.0))
        out["chi"] = chi
    out["p"] = gm1 * rho * e
    return out
