"""The C ABI library: it loads, exports every symbol include/lbsd.h declares,
and rejects bad arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbsd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    from paper_1602_02675_amd import lbsd

    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(lbsd.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lbsd.h but not exported"
    assert set(lbsd.EXPORTED) <= set(names)


def _create(lbsd, **kw):
    g = lbsd.lb_grid(kw.get("dim", 1), kw.get("nx", 100), kw.get("ny", 1), kw.get("x_lo", 0.0),
                     kw.get("x_hi", 1.0), kw.get("bc_x", 0), kw.get("bc_y", 1))
    vs = lbsd.lb_velset(kw.get("lattice", 1), kw.get("d0", 0.5))
    h = ctypes.c_void_p()
    rc = lbsd._lib.lb_create(ctypes.byref(g), kw.get("gamma", 1.4), ctypes.byref(vs),
                             kw.get("prec", 0), ctypes.byref(h))
    return rc, h


def test_create_validation():
    from paper_1602_02675_amd import lbsd

    rc, h = _create(lbsd)
    assert rc == lbsd.LB_OK
    assert lbsd._lib.lb_state_bytes(h) >= 2 * 3 * 100 * 8
    lbsd._lib.lb_destroy(h)
    bad = [dict(gamma=1.0), dict(gamma=3.5), dict(dim=2, lattice=2, d0=0.0, gamma=2.5),
           dict(d0=1.0), dict(d0=-0.1), dict(dim=3), dict(nx=0), dict(ny=2),
           dict(dim=2, lattice=1, d0=0.0), dict(dim=2, lattice=2, d0=0.5),
           dict(bc_x=7), dict(x_hi=0.0), dict(prec=5),
           # reflecting walls need the mirror images of the halo inside the grid
           dict(bc_x=2, nx=4), dict(dim=2, lattice=2, d0=0.0, nx=64, ny=4, bc_y=2),
           dict(dim=2, lattice=2, d0=0.0, nx=4, ny=64, bc_x=2),
           # the square set with a rest level needs 0 < d0_frac < 1, and 2-D
           dict(dim=2, lattice=3, d0=0.0), dict(dim=2, lattice=3, d0=1.0), dict(dim=1, lattice=3, d0=0.5)]
    for kw in bad:
        rc, h = _create(lbsd, **kw)
        assert rc == lbsd.LB_EINVAL, kw
        assert lbsd._lib.lb_last_error()
    for kw in (dict(bc_x=2, nx=5), dict(bc_x=2, bc_y=2), dict(dim=2, lattice=3, d0=0.5, nx=8, ny=8),
               dict(dim=2, lattice=2, d0=0.0, nx=5, ny=5, bc_x=2, bc_y=2)):
        rc, h = _create(lbsd, **kw)
        assert rc == lbsd.LB_OK, kw
        lbsd._lib.lb_destroy(h)
    rc, h = _create(lbsd, dim=2, lattice=2, d0=0.0, nx=64, ny=32, prec=1)
    assert rc == lbsd.LB_OK
    # 2 FP32 buffers of 4 fields + FP64 staging
    assert lbsd._lib.lb_state_bytes(h) >= 2 * 4 * 64 * 32 * 4 + 4 * 64 * 32 * 8
    lbsd._lib.lb_destroy(h)


def test_two_gas_create_validation():
    from paper_1602_02675_amd import lbsd

    def make(dim, g1, g2, nx=100, ny=1, lattice=1, d0=0.5):
        g = lbsd.lb_grid(dim, nx, ny, 0.0, 1.0, 0, 1)
        vs = lbsd.lb_velset(lattice, d0)
        h = ctypes.c_void_p()
        return lbsd._lib.lb_create_two_gas(ctypes.byref(g), g1, g2, ctypes.byref(vs), 0, ctypes.byref(h)), h

    rc, h = make(1, 1.4, 5.0 / 3.0)
    assert rc == lbsd.LB_OK
    # four fields (rho, rho u, rho E, rho chi) in two sets
    assert lbsd._lib.lb_state_bytes(h) >= 2 * 4 * 100 * 8
    out = ctypes.c_double()
    lbsd._lib.lb_destroy(h)
    # the square dual-level set: five fields; the gases' gamma in (1, 2]
    rc, h = make(2, 1.4, 5.0 / 3.0, 8, 8, 2, 0.0)
    assert rc == lbsd.LB_OK
    assert lbsd._lib.lb_state_bytes(h) >= 2 * 5 * 64 * 8
    lbsd._lib.lb_destroy(h)
    rc, h = make(2, 1.4, 5.0 / 3.0, 8, 8, 3, 0.5)  # and the square set with a rest level
    assert rc == lbsd.LB_OK
    lbsd._lib.lb_destroy(h)
    for args in ((2, 1.4, 1.4, 8, 8, 3, 0.0), (2, 1.4, 2.5, 8, 8, 2, 0.0), (1, 1.4, 1.0), (1, 1.4, 3.5),
                 (1, 0.9, 1.4)):
        rc, h = make(*args)
        assert rc == lbsd.LB_EINVAL, args
    # pools of two gases: both gammas checked
    g = lbsd.lb_velset(1, 0.5)
    for g2, want in ((5.0 / 3.0, lbsd.LB_OK), (3.5, lbsd.LB_EINVAL), (1.0, lbsd.LB_EINVAL)):
        hp = ctypes.c_void_p()
        assert lbsd._lib.lb_pool_create_two_gas(1, 1.4, g2, ctypes.byref(g), 0, 4, 1 << 20, ctypes.byref(hp)) == want
        if want == lbsd.LB_OK:
            lbsd._lib.lb_pool_destroy(hp)
    # one gas: no species total
    rc, h = _create(lbsd)
    assert rc == lbsd.LB_OK
    assert lbsd._lib.lb_species_total(h, ctypes.byref(out)) == lbsd.LB_EINVAL
    lbsd._lib.lb_destroy(h)


def test_calls_on_unbound_solver_fail_cleanly():
    from paper_1602_02675_amd import lbsd

    rc, h = _create(lbsd)
    assert lbsd._lib.lb_step(h, 1) == lbsd.LB_EINVAL
    out = (ctypes.c_double * 4)()
    assert lbsd._lib.lb_totals(h, out) == lbsd.LB_EINVAL
    assert lbsd._lib.lb_set_lambda(h, -1.0) == lbsd.LB_EINVAL
    assert lbsd._lib.lb_set_cfl(h, 0.0) == lbsd.LB_EINVAL
    assert lbsd._lib.lb_bind(h, None, 0, None) == lbsd.LB_EINVAL
    lbsd._lib.lb_destroy(h)


def _pool(lbsd, dim=1, gamma=1.4, d0=None, prec=0, slots=8, arena=1 << 20):
    vs = lbsd.lb_velset(1 if dim == 1 else 2, (0.5 if dim == 1 else 0.0) if d0 is None else d0)
    h = ctypes.c_void_p()
    rc = lbsd._lib.lb_pool_create(dim, gamma, ctypes.byref(vs), prec, slots, arena, ctypes.byref(h))
    return rc, h


def test_pool_create_validation_and_sizes():
    from paper_1602_02675_amd import lbsd

    rc, h = _pool(lbsd)
    assert rc == lbsd.LB_OK
    assert lbsd._lib.lb_pool_bytes(h) >= 1 << 20
    # footprint: two FP64 sets of 3 fields, each rounded up to 256 bytes
    assert lbsd._lib.lb_pool_footprint(h, 1000, 1) == 2 * ((3 * 1000 * 8 + 255) // 256 * 256)
    assert lbsd._lib.lb_pool_shapes(h) == 5
    # unbound pool: no admission, no stepping
    g = lbsd.lb_grid(1, 100, 1, 0.0, 1.0, 0, 1)
    L = lbsd.lb_prim(1.0, 0.0, 0.0, 1.0)
    slot = ctypes.c_int32(-1)
    assert lbsd._lib.lb_pool_admit_riemann(h, ctypes.byref(g), 0.0, 0.5, ctypes.byref(L), ctypes.byref(L), 10,
                                           ctypes.byref(slot)) == lbsd.LB_EINVAL
    assert lbsd._lib.lb_pool_advance(h, 1) == lbsd.LB_EINVAL
    assert lbsd._lib.lb_pool_bind(h, None, 0, None) == lbsd.LB_EINVAL
    lbsd._lib.lb_pool_destroy(h)
    for kw in (dict(gamma=1.0), dict(dim=3), dict(dim=2, d0=0.3), dict(prec=9), dict(slots=0),
               dict(arena=16), dict(d0=1.0)):
        rc, h = _pool(lbsd, **kw)
        assert rc == lbsd.LB_EINVAL, kw
    rc, h = _pool(lbsd, dim=2, prec=1)
    assert rc == lbsd.LB_OK
    assert lbsd._lib.lb_pool_footprint(h, 64, 64) == 2 * 4 * 64 * 64 * 4
    lbsd._lib.lb_pool_destroy(h)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: with the HIP library missing, importing the binding
    raises instead of running anything else."""
    import subprocess
    import sys

    env = dict(os.environ, LBSD_LIBRARY=str(tmp_path / "absent" / "liblbsd.so"))
    code = "import paper_1602_02675_amd.lbsd"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is missing" in r.stderr
