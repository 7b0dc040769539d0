"""Parity at the benchmark's full sizes and launch configurations, on sampled
outputs the oracle can compute: the batch of 512 1-D tubes of uneven lengths
(256 to 65536 nodes, seeded Riemann states) in one pool, autotuned after the
flows have developed and run through HIP graphs as the benchmark runs it;
sampled tubes (the longest, the shortest and two others) are run by the
oracle for the same steps.  FP64 at the parity bar (1e-12 normwise per
field), FP32 at 1e-5 relative L1 density."""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs

from parity_helpers import TOL64, normwise_err

pytestmark = pytest.mark.gpu

N_TUBES, SEED = 512, 0


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def _oracle_tube(nx, left, right, xd, lam, steps):
    P = oracle.Problem(1, nx)
    Y0 = oracle.riemann_moments(P, inputs.node_x(nx), left, right, xd)
    ref, st, reach = oracle.run(P, oracle.to_lattice(P, Y0, lam), steps)
    assert st == 0 and reach <= 5
    return oracle.from_lattice(P, ref, lam)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_512_tubes_sampled_against_oracle(lbsd, prec):
    lens = inputs.tube_lengths(SEED, N_TUBES)
    elem = 8 if prec == "fp64" else 4
    arena = int(sum(2 * (((3 * int(L) * elem) + 255) // 256 * 256) for L in lens)) + (1 << 20)
    pool = lbsd.Pool(1, N_TUBES, arena, precision=prec)
    probs, slots = [], []
    for i, L in enumerate(lens):
        left, right, xd = inputs.riemann_instance(SEED * 100000 + i)
        lam = inputs.cfl_lambda([left, right])
        probs.append((int(L), left, right, xd, lam))
        slots.append(pool.admit_riemann(int(L), xd, left, right, 10 ** 6, lam=lam))
        assert slots[-1] is not None
    pool.advance(50)
    pool.autotune(trials=2)  # trial steps leave every state as it is
    pool.use_graph(50)
    pool.advance(100)
    steps = 150
    rng = np.random.default_rng(1)
    sample = sorted({int(np.argmax(lens)), int(np.argmin(lens)), *rng.choice(N_TUBES, size=2, replace=False).tolist()})
    for i in sample:
        assert pool.poll(slots[i]) == (steps, 0)  # still running (target far away), no error
        nx, left, right, xd, lam = probs[i]
        ref = _oracle_tube(nx, left, right, xd, lam, steps)
        got = pool.moments(slots[i])
        if prec == "fp64":
            assert normwise_err(got, ref, 1) <= TOL64, (i, nx)
        else:
            assert np.sum(np.abs(got[0] - ref[0])) / np.sum(np.abs(ref[0])) <= 1e-5, (i, nx)
    pool.close()


def test_served_requests_sampled_against_oracle(lbsd):
    """The served form's requests (square grids, seeded planar Riemann
    states, FP32 pool, default periodic y) at their full sizes, the largest
    side 2048, admitted while others run and finishing at different steps:
    every row of a request equals its first (the states are planar) and
    matches the oracle on a 4-row strip of the same tube (relative L1 density
    within 1e-5)."""
    reqs = inputs.serve_requests(3, 6, rate_per_s=1.0)
    reqs[0].update(side=2048, steps=150)
    reqs[1].update(side=64, steps=100)
    for r in reqs[2:]:
        r["steps"] = min(r["steps"], 160)
    pool = lbsd.Pool(2, 8, 4 << 30, precision="fp32")
    pool.use_graph(25)
    slots = {}
    for i, r in enumerate(reqs):
        if i == 3:
            pool.advance(40)  # later arrivals join a running pool
        slots[i] = pool.admit_riemann(r["side"], r["x_d"], r["left"], r["right"], r["steps"], ny=r["side"],
                                      lam=inputs.cfl_lambda([r["left"], r["right"]]))
        assert slots[i] is not None
    pool.advance(max(r["steps"] for r in reqs) + 50)
    for i, r in enumerate(reqs):
        assert pool.poll(slots[i]) == (r["steps"], 1)
        got = pool.moments(slots[i])
        assert np.all(got == got[:, :1, :])
        n = r["side"]
        lam = inputs.cfl_lambda([r["left"], r["right"]])
        P = oracle.Problem(2, n, 4, bc_y=oracle.TRANSMISSIVE)
        Y0 = oracle.riemann_moments(P, inputs.node_x(n), r["left"], r["right"], r["x_d"])
        ref, st, _ = oracle.run(P, oracle.to_lattice(P, Y0, lam), r["steps"])
        assert st == 0
        ref = oracle.from_lattice(P, ref, lam)
        err = np.sum(np.abs(got[0, :4] - ref[0])) / np.sum(np.abs(ref[0]))
        assert err <= 1e-5, (i, n, r["steps"], err)
    pool.close()
