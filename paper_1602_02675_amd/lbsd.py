"""Python binding of the lbsd C ABI (include/lbsd.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``liblbsd.so``; PyTorch
provides the device memory (one uint8 tensor per solver) and the stream.  If
the library has not been built, importing this module raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its bundled HIP runtime must be the one liblbsd.so binds to
# (the library's libamdhip64.so.7 dependency then resolves to that copy), so
# that torch's device pointers and streams are valid in the library.
import torch  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBSD_LIBRARY") or os.path.join(_PKG, "liblbsd.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE, LB_EREACH = 0, -1, -2, -3, -4, -5
LB_BC_TRANSMISSIVE, LB_BC_PERIODIC, LB_BC_REFLECTING = 0, 1, 2
LB_LATTICE_D1_TRIPLE, LB_LATTICE_D2_SQUARE_DUAL, LB_LATTICE_D2_SQUARE_TRIPLE = 1, 2, 3
LB_LATTICE_D2_HEX_DUAL, LB_LATTICE_D2_HEX_TRIPLE = 4, 5
LB_FP64, LB_FP32 = 0, 1
LB_HALO = 5
LB_POOL_FREE = -100

_ERR_NAMES = {LB_EINVAL: "LB_EINVAL", LB_ENOMEM: "LB_ENOMEM", LB_EDEVICE: "LB_EDEVICE",
              LB_ESTATE: "LB_ESTATE", LB_EREACH: "LB_EREACH"}

EXPORTED = ["lb_create", "lb_create_two_gas", "lb_species_total", "lb_state_bytes", "lb_bind", "lb_set_lambda",
            "lb_set_cfl",
            "lb_init_riemann", "lb_init_moments", "lb_step", "lb_step_timed", "lb_step_profiled", "lb_sync",
            "lb_moments", "lb_totals", "lb_lambda", "lb_dt", "lb_steps_done", "lb_max_reach",
            "lb_debug_lanes", "lb_destroy", "lb_last_error", "lb_step_static",
            "lb_pool_create", "lb_pool_create_two_gas", "lb_pool_bytes", "lb_pool_footprint", "lb_pool_bind", "lb_pool_admit_riemann",
            "lb_pool_admit_moments", "lb_pool_release", "lb_pool_advance", "lb_pool_advance_timed",
            "lb_pool_poll", "lb_pool_status", "lb_pool_snapshot", "lb_pool_snapshot_read", "lb_pool_moments", "lb_pool_totals", "lb_pool_lambda", "lb_pool_live",
            "lb_pool_shapes", "lb_pool_shape", "lb_pool_set_shape", "lb_pool_autotune", "lb_pool_use_graph",
            "lb_pool_destroy"]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class lb_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class lb_velset(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("d0_frac", ctypes.c_double)]


class lb_prim(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("u", ctypes.c_double), ("v", ctypes.c_double),
                ("p", ctypes.c_double)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1602_02675_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    D, I32P = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    sig = {
        "lb_create": (ctypes.c_int, [ctypes.POINTER(lb_grid), dbl, ctypes.POINTER(lb_velset), i32,
                                     ctypes.POINTER(vp)]),
        "lb_create_two_gas": (ctypes.c_int, [ctypes.POINTER(lb_grid), dbl, dbl, ctypes.POINTER(lb_velset),
                                             i32, ctypes.POINTER(vp)]),
        "lb_state_bytes": (ctypes.c_size_t, [vp]),
        "lb_bind": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "lb_set_lambda": (ctypes.c_int, [vp, dbl]),
        "lb_set_cfl": (ctypes.c_int, [vp, dbl]),
        "lb_init_riemann": (ctypes.c_int, [vp, dbl, ctypes.POINTER(lb_prim), ctypes.POINTER(lb_prim)]),
        "lb_init_moments": (ctypes.c_int, [vp, D, dbl]),
        "lb_step": (ctypes.c_int, [vp, i64]),
        "lb_step_timed": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_float)]),
        "lb_step_profiled": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_float)]),
        "lb_sync": (ctypes.c_int, [vp]),
        "lb_moments": (ctypes.c_int, [vp, vp, i32]),
        "lb_totals": (ctypes.c_int, [vp, D]),
        "lb_species_total": (ctypes.c_int, [vp, D]),
        "lb_lambda": (dbl, [vp]),
        "lb_dt": (dbl, [vp]),
        "lb_steps_done": (i64, [vp]),
        "lb_max_reach": (i32, [vp]),
        "lb_debug_lanes": (ctypes.c_int, [vp, I32P, I32P, I32P]),
        "lb_destroy": (None, [vp]),
        "lb_last_error": (ctypes.c_char_p, []),
        "lb_step_static": (ctypes.c_int, [vp, vp, vp, vp, I32P]),
        "lb_pool_create": (ctypes.c_int, [i32, dbl, ctypes.POINTER(lb_velset), i32, i32, ctypes.c_size_t,
                                          ctypes.POINTER(vp)]),
        "lb_pool_create_two_gas": (ctypes.c_int, [i32, dbl, dbl, ctypes.POINTER(lb_velset), i32, i32,
                                                  ctypes.c_size_t, ctypes.POINTER(vp)]),
        "lb_pool_bytes": (ctypes.c_size_t, [vp]),
        "lb_pool_footprint": (ctypes.c_size_t, [vp, i64, i64]),
        "lb_pool_bind": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "lb_pool_admit_riemann": (ctypes.c_int, [vp, ctypes.POINTER(lb_grid), dbl, dbl, ctypes.POINTER(lb_prim),
                                                 ctypes.POINTER(lb_prim), i64, I32P]),
        "lb_pool_admit_moments": (ctypes.c_int, [vp, ctypes.POINTER(lb_grid), D, dbl, i64, I32P]),
        "lb_pool_release": (ctypes.c_int, [vp, i32]),
        "lb_pool_advance": (ctypes.c_int, [vp, i64]),
        "lb_pool_advance_timed": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_float)]),
        "lb_pool_poll": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_int64), I32P]),
        "lb_pool_status": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64), I32P]),
        "lb_pool_snapshot": (ctypes.c_int, [vp, i32]),
        "lb_pool_snapshot_read": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_int64), I32P,
                                                 ctypes.POINTER(ctypes.c_double)]),
        "lb_pool_moments": (ctypes.c_int, [vp, i32, vp, i32]),
        "lb_pool_totals": (ctypes.c_int, [vp, i32, D]),
        "lb_pool_lambda": (dbl, [vp, i32]),
        "lb_pool_live": (i32, [vp]),
        "lb_pool_shapes": (i32, [vp]),
        "lb_pool_shape": (i32, [vp]),
        "lb_pool_set_shape": (ctypes.c_int, [vp, i32]),
        "lb_pool_autotune": (ctypes.c_int, [vp, i32, I32P, ctypes.POINTER(ctypes.c_float)]),
        "lb_pool_use_graph": (ctypes.c_int, [vp, i32]),
        "lb_pool_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def _check(rc: int):
    if rc != LB_OK:
        raise LBError(rc, _lib.lb_last_error().decode())


def _lattice(dim: int, d0_frac: float, lattice: str = "square") -> int:
    """The 1-D triple-level set, or on the square (or hexagonal) lattice the
    dual-level set (d0_frac = 0) or the set with a rest level (d0_frac > 0)."""
    if dim == 1:
        return LB_LATTICE_D1_TRIPLE
    if lattice == "hex":
        return LB_LATTICE_D2_HEX_TRIPLE if d0_frac > 0.0 else LB_LATTICE_D2_HEX_DUAL
    if lattice != "square":
        raise ValueError(f"lattice must be 'square' or 'hex', not {lattice!r}")
    return LB_LATTICE_D2_SQUARE_TRIPLE if d0_frac > 0.0 else LB_LATTICE_D2_SQUARE_DUAL


def _bc(v) -> int:
    if isinstance(v, str):
        return {"transmissive": LB_BC_TRANSMISSIVE, "periodic": LB_BC_PERIODIC,
                "reflecting": LB_BC_REFLECTING}[v]
    return int(v)


class Solver:
    """One grid on one GPU.  State = SoA moments (rho, rho u, (rho v), rho E)."""

    def __init__(self, dim: int, nx: int, ny: int = 1, *, gamma: float = 1.4, d0_frac=None,
                 precision: str = "fp64", bc_x="transmissive", bc_y="periodic", x_lo: float = 0.0,
                 x_hi: float = 1.0, device=None, stream=None, gamma2=None, lattice: str = "square"):
        """gamma2: a second gas (lb_create_two_gas): gamma is gas 1's, and
        the state gains the species field rho chi.  lattice (dim 2): "square"
        or "hex" (the hexagonal lattice, nodes at i e_1 + j e_2, stored
        [f][j][i], Cartesian momenta)."""
        import torch

        if d0_frac is None:
            d0_frac = 0.5 if dim == 1 else 0.0
        self.dim, self.nx, self.ny = dim, int(nx), int(ny if dim == 2 else 1)
        self.species = gamma2 is not None
        self.nf = dim + 2 + (1 if self.species else 0)
        self.precision = precision
        g = lb_grid(dim, self.nx, self.ny, x_lo, x_hi, _bc(bc_x), _bc(bc_y))
        self.lattice = lattice if dim == 2 else "line"
        vs = lb_velset(_lattice(dim, d0_frac, lattice), d0_frac)
        prec = {"fp64": LB_FP64, "fp32": LB_FP32}[precision]
        h = ctypes.c_void_p()
        if self.species:
            _check(_lib.lb_create_two_gas(ctypes.byref(g), gamma, float(gamma2), ctypes.byref(vs), prec,
                                          ctypes.byref(h)))
        else:
            _check(_lib.lb_create(ctypes.byref(g), gamma, ctypes.byref(vs), prec, ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = int(_lib.lb_state_bytes(h))
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        _check(_lib.lb_bind(h, ctypes.c_void_p(self._buf.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream)))

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def state_bytes(self) -> int:
        return int(_lib.lb_state_bytes(self._h))

    # -- initial states --------------------------------------------------------
    def set_lambda(self, lam: float):
        _check(_lib.lb_set_lambda(self._h, float(lam)))

    def set_cfl(self, cfl: float):
        _check(_lib.lb_set_cfl(self._h, float(cfl)))

    def init_riemann(self, x_d: float, left, right, lam: float | None = None):
        """left/right = (rho, u, v, p) in physical units."""
        if lam is not None:
            self.set_lambda(lam)
        L, R = lb_prim(*map(float, left)), lb_prim(*map(float, right))
        _check(_lib.lb_init_riemann(self._h, float(x_d), ctypes.byref(L), ctypes.byref(R)))

    def init_moments(self, Y, lam: float):
        """Y: FP64 [nf, ny, nx] conserved moments, physical units."""
        Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(self.nf, self.ny, self.nx)
        _check(_lib.lb_init_moments(self._h, Y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    float(lam)))

    # -- stepping --------------------------------------------------------------
    def step(self, n: int = 1):
        _check(_lib.lb_step(self._h, int(n)))

    def step_timed(self, n: int) -> float:
        ms = ctypes.c_float(0.0)
        _check(_lib.lb_step_timed(self._h, int(n), ctypes.byref(ms)))
        return float(ms.value)

    def step_profiled(self, n: int):
        """(summed step-kernel ms, total ms) of n steps, from HIP events."""
        k, t = ctypes.c_float(0.0), ctypes.c_float(0.0)
        _check(_lib.lb_step_profiled(self._h, int(n), ctypes.byref(k), ctypes.byref(t)))
        return float(k.value), float(t.value)

    def sync(self):
        _check(_lib.lb_sync(self._h))

    def step_static(self, y_in, y_out, status=None, stream=None):
        """One step from the device moment fields y_in to y_out (torch tensors
        of the storage dtype, [nf, ny, nx], lattice units) with the library's
        static scratch (lb_step_static); status: optional int32 device tensor
        that receives the step's status code.  Queued on `stream` (default:
        the solver's)."""
        st = self.stream if stream is None else stream
        sp = ctypes.cast(ctypes.c_void_p(status.data_ptr()), ctypes.POINTER(ctypes.c_int32)) if status is not None \
            else None
        _check(_lib.lb_step_static(self._h, ctypes.c_void_p(y_in.data_ptr()), ctypes.c_void_p(y_out.data_ptr()),
                                   ctypes.c_void_p(st.cuda_stream), sp))

    # -- outputs ---------------------------------------------------------------
    def moments(self) -> np.ndarray:
        out = np.empty((self.nf, self.ny, self.nx), dtype=np.float64)
        _check(_lib.lb_moments(self._h, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def moments_device(self):
        import torch

        out = torch.empty((self.nf, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(_lib.lb_moments(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def totals(self) -> np.ndarray:
        out = np.zeros(4, dtype=np.float64)
        _check(_lib.lb_totals(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def species_total(self) -> float:
        """Two gases: interior sum of rho chi (lb_species_total)."""
        out = ctypes.c_double(0.0)
        _check(_lib.lb_species_total(self._h, ctypes.byref(out)))
        return float(out.value)

    def lanes(self):
        n = self.nx * self.ny
        fx, fy, c1 = (np.zeros(n, dtype=np.int32) for _ in range(3))
        p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        _check(_lib.lb_debug_lanes(self._h, p(fx), p(fy), p(c1)))
        shp = (self.ny, self.nx)
        return fx.reshape(shp), fy.reshape(shp), c1.reshape(shp)

    @property
    def lam(self) -> float:
        return float(_lib.lb_lambda(self._h))

    @property
    def dt(self) -> float:
        return float(_lib.lb_dt(self._h))

    @property
    def steps_done(self) -> int:
        return int(_lib.lb_steps_done(self._h))

    def max_reach(self) -> int:
        return int(_lib.lb_max_reach(self._h))


class Pool:
    """Many independent problems of one lattice and precision, advanced by one
    persistent launch per step (include/lbsd.h, lb_pool_*).  Memory: one
    uint8 torch tensor; stream: a dedicated torch stream (graph capture needs
    a non-default stream)."""

    def __init__(self, dim: int, max_slots: int, arena_bytes: int, *, gamma: float = 1.4, d0_frac=None,
                 precision: str = "fp32", device=None, stream=None, gamma2=None):
        """gamma2: a pool of two-gas problems (lb_pool_create_two_gas); every
        slot's state then has the species field rho chi last."""
        import torch

        if d0_frac is None:
            d0_frac = 0.5 if dim == 1 else 0.0
        self.species = gamma2 is not None
        self.dim, self.nf, self.precision = dim, dim + 2 + (1 if self.species else 0), precision
        self.max_slots = int(max_slots)
        self.arena_bytes = int(arena_bytes)
        vs = lb_velset(_lattice(dim, d0_frac), d0_frac)  # pools run the 1-D and square lattices
        prec = {"fp64": LB_FP64, "fp32": LB_FP32}[precision]
        h = ctypes.c_void_p()
        if self.species:
            _check(_lib.lb_pool_create_two_gas(dim, gamma, float(gamma2), ctypes.byref(vs), prec, int(max_slots),
                                               int(arena_bytes), ctypes.byref(h)))
        else:
            _check(_lib.lb_pool_create(dim, gamma, ctypes.byref(vs), prec, int(max_slots), int(arena_bytes),
                                       ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = int(_lib.lb_pool_bytes(h))
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device) if stream is None else stream
        torch.cuda.synchronize(self.device)  # the buffer exists before the pool's stream uses it
        _check(_lib.lb_pool_bind(h, ctypes.c_void_p(self._buf.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)))
        self._shape = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lb_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, nx: int, ny: int = 1) -> int:
        return int(_lib.lb_pool_footprint(self._h, int(nx), int(ny)))

    def _grid(self, nx, ny, bc_x, bc_y, x_lo, x_hi):
        ny = int(ny) if self.dim == 2 else 1
        return lb_grid(self.dim, int(nx), ny, float(x_lo), float(x_hi), _bc(bc_x), _bc(bc_y))

    def admit_riemann(self, nx: int, x_d: float, left, right, steps: int, *, ny: int = 1, lam: float = 0.0,
                      bc_x="transmissive", bc_y="periodic", x_lo: float = 0.0, x_hi: float = 1.0):
        """Slot index, or None when the pool has no room now (LB_ENOMEM)."""
        g = self._grid(nx, ny, bc_x, bc_y, x_lo, x_hi)
        L, R = lb_prim(*map(float, left)), lb_prim(*map(float, right))
        slot = ctypes.c_int32(-1)
        rc = _lib.lb_pool_admit_riemann(self._h, ctypes.byref(g), float(lam), float(x_d), ctypes.byref(L),
                                        ctypes.byref(R), int(steps), ctypes.byref(slot))
        if rc == LB_ENOMEM:
            return None
        _check(rc)
        self._shape[slot.value] = (self.nf, g.ny, g.nx)
        return slot.value

    def admit_moments(self, Y, lam: float, steps: int, *, bc_x="transmissive", bc_y="periodic",
                      x_lo: float = 0.0, x_hi: float = 1.0):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        ny, nx = (Y.shape[1], Y.shape[2]) if Y.ndim == 3 else (1, Y.shape[-1])
        g = self._grid(nx, ny, bc_x, bc_y, x_lo, x_hi)
        slot = ctypes.c_int32(-1)
        rc = _lib.lb_pool_admit_moments(self._h, ctypes.byref(g), Y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        float(lam), int(steps), ctypes.byref(slot))
        if rc == LB_ENOMEM:
            return None
        _check(rc)
        self._shape[slot.value] = (self.nf, g.ny, g.nx)
        return slot.value

    def release(self, slot: int):
        _check(_lib.lb_pool_release(self._h, int(slot)))
        self._shape.pop(int(slot), None)

    def advance(self, n: int = 1):
        _check(_lib.lb_pool_advance(self._h, int(n)))

    def advance_timed(self, n: int) -> float:
        ms = ctypes.c_float(0.0)
        _check(_lib.lb_pool_advance_timed(self._h, int(n), ctypes.byref(ms)))
        return float(ms.value)

    def poll(self, slot: int):
        """(steps done, status): status 0 running, 1 finished, LB_EREACH / LB_ESTATE failed."""
        done, st = ctypes.c_int64(0), ctypes.c_int32(0)
        _check(_lib.lb_pool_poll(self._h, int(slot), ctypes.byref(done), ctypes.byref(st)))
        return int(done.value), int(st.value)

    def status(self):
        """(steps done, status) arrays over all slots; free slots have status LB_POOL_FREE."""
        done = np.zeros(self.max_slots, dtype=np.int64)
        st = np.zeros(self.max_slots, dtype=np.int32)
        _check(_lib.lb_pool_status(self._h, done.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return done, st

    def snapshot(self, buf: int):
        """Queue a copy of every slot's progress into host buffer buf (0 or 1)
        behind the queued work; returns at once (lb_pool_snapshot)."""
        _check(_lib.lb_pool_snapshot(self._h, int(buf)))

    def snapshot_read(self, buf: int):
        """Wait for snapshot buf: (steps done, status, totals [max_slots, 4]
        physical units, NaN before a slot's first step)."""
        done = np.zeros(self.max_slots, dtype=np.int64)
        st = np.zeros(self.max_slots, dtype=np.int32)
        tot = np.zeros((self.max_slots, 4), dtype=np.float64)
        _check(_lib.lb_pool_snapshot_read(self._h, int(buf), done.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          tot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return done, st, tot

    def moments(self, slot: int) -> np.ndarray:
        out = np.empty(self._shape[int(slot)], dtype=np.float64)
        _check(_lib.lb_pool_moments(self._h, int(slot), ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def moments_device(self, slot: int):
        import torch

        out = torch.empty(self._shape[int(slot)], dtype=torch.float64, device=self.device)
        _check(_lib.lb_pool_moments(self._h, int(slot), ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def totals(self, slot: int) -> np.ndarray:
        out = np.zeros(4, dtype=np.float64)
        _check(_lib.lb_pool_totals(self._h, int(slot), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def lam(self, slot: int) -> float:
        return float(_lib.lb_pool_lambda(self._h, int(slot)))

    @property
    def live(self) -> int:
        return int(_lib.lb_pool_live(self._h))

    @property
    def shapes(self) -> int:
        return int(_lib.lb_pool_shapes(self._h))

    @property
    def shape(self) -> int:
        return int(_lib.lb_pool_shape(self._h))

    def set_shape(self, shape: int):
        _check(_lib.lb_pool_set_shape(self._h, int(shape)))

    def autotune(self, trials: int = 5):
        """(best shape, its median ms per step)."""
        best, ms = ctypes.c_int32(-1), ctypes.c_float(0.0)
        _check(_lib.lb_pool_autotune(self._h, int(trials), ctypes.byref(best), ctypes.byref(ms)))
        return int(best.value), float(ms.value)

    def use_graph(self, steps_per_graph: int):
        _check(_lib.lb_pool_use_graph(self._h, int(steps_per_graph)))
