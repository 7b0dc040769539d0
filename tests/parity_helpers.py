"""Helpers of the GPU parity tests: the normwise error of the parity bar and
a paired run of the HIP path and the oracle on the same input."""
import numpy as np

import oracle

TOL64 = 1e-12  # FP64 parity bar, normwise per field


def normwise_err(got, ref, dim):
    got = np.asarray(got).reshape(ref.shape)
    errs = []
    mom = max(np.max(np.abs(ref[1:1 + dim])), 1e-300)
    for f in range(ref.shape[0]):
        scale = mom if 1 <= f <= dim else max(np.max(np.abs(ref[f])), 1e-300)
        errs.append(np.max(np.abs(got[f] - ref[f])) / scale)
    return max(errs)


def run_pair(lbsd, dim, Y_phys, lam, n, *, nx, ny=1, bcx=0, bcy=1, delta0=None, prec="fp64", gamma2=None):
    """gamma2: two gases (gamma 1.4 for gas 1); Y_phys then holds rho chi last."""
    P = oracle.Problem(dim, nx, ny, bc_x=bcx, bc_y=bcy, delta0=delta0, gamma2=gamma2)
    ref, st, reach = oracle.run(P, oracle.to_lattice(P, Y_phys, lam), n)
    assert st == 0 and reach <= 5
    s = lbsd.Solver(dim, nx, ny, bc_x=bcx, bc_y=bcy, d0_frac=delta0, precision=prec, gamma2=gamma2)
    s.init_moments(Y_phys, lam)
    s.step(n)
    got = s.moments()
    return P, oracle.from_lattice(P, ref, lam), got, s


def self_divergence(P, Yl, n, seed=0):
    """How far the oracle itself moves after n steps when its input is
    perturbed at the level of FP64 rounding (relative 1e-16): the square
    dual-level lattice amplifies rounding differences on non-planar data."""
    rng = np.random.default_rng(seed)
    a, _, _ = oracle.run(P, Yl, n)
    b, _, _ = oracle.run(P, Yl * (1.0 + 1e-16 * rng.standard_normal(Yl.shape)), n)
    return normwise_err(b, a, 2)
