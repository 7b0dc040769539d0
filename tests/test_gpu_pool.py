"""GPU tests of the pool (batched and served) form, through the C ABI.

A slot's result must not depend on what else is in the pool: every slot is
compared bit for bit with an lb_solver run of the same problem (whose parity
with the oracle is tested in test_gpu_parity), across tile shapes, graph
capture, admissions and releases while others run, and failures of other
slots.  One slot per lattice is also checked against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02675_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def alone(lbsd, dim, nx, ny, x_d, left, right, lam, steps, prec, bc_x="transmissive", bc_y="periodic"):
    s = lbsd.Solver(dim, nx, ny, precision=prec, bc_x=bc_x, bc_y=bc_y)
    s.init_riemann(x_d, left, right, lam=lam)
    s.step(steps)
    out = s.moments()
    s.close()
    return out


def tube_set(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    lens = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))).astype(int)
    probs = []
    for i, L in enumerate(lens):
        left, right, xd = inputs.riemann_instance(seed * 1000 + i)
        probs.append((int(L), xd, left, right, inputs.cfl_lambda([left, right])))
    return probs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pool_1d_equals_solver_every_shape_and_graph(lbsd, prec):
    probs = tube_set(1, 9, 1, 6000) + [(1, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.8),
                                        (1025, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.8)]
    steps = [40] * len(probs)
    steps[2] = 17  # one slot stops early
    ref = [alone(lbsd, 1, nx, 1, xd, L, R, lam, st, prec) for (nx, xd, L, R, lam), st in zip(probs, steps)]
    pool = lbsd.Pool(1, 16, 8 << 20, precision=prec)
    for shape in range(pool.shapes):
        for graph in (0, 8):
            slots = [pool.admit_riemann(nx, xd, L, R, st, lam=lam) for (nx, xd, L, R, lam), st in zip(probs, steps)]
            pool.set_shape(shape)
            pool.use_graph(graph)
            pool.advance(13)
            pool.advance(30)  # past every target: finished slots stay put
            for i, sl in enumerate(slots):
                done, status = pool.poll(sl)
                assert (done, status) == (steps[i], 1)
                got = pool.moments(sl)
                assert np.array_equal(got, ref[i]), (shape, graph, i)
            for sl in slots:
                pool.release(sl)
            assert pool.live == 0
    pool.close()


def test_pool_1d_slot_against_oracle(lbsd):
    nx = 1000
    n, lam = inputs.steps_and_lambda(0.2, 1.0 / nx, [inputs.SOD_LEFT, inputs.SOD_RIGHT])
    P = oracle.Problem(1, nx)
    Y0 = oracle.riemann_moments(P, inputs.node_x(nx), inputs.SOD_LEFT, inputs.SOD_RIGHT, 0.5)
    ref, st, _ = oracle.run(P, oracle.to_lattice(P, Y0, lam), n)
    ref = oracle.from_lattice(P, ref, lam)
    pool = lbsd.Pool(1, 4, 1 << 20, precision="fp64")
    other = pool.admit_riemann(333, 0.4, inputs.SOD_LEFT, inputs.SOD_RIGHT, 10 * n, lam=0.7)
    sl = pool.admit_riemann(nx, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, n, lam=lam)
    pool.advance(n + 5)
    got = pool.moments(sl)
    err = max(np.max(np.abs(got[f] - ref[f])) / np.max(np.abs(ref[f] if f != 1 else ref[1:2])) for f in range(3))
    assert err <= 1e-12
    tot = pool.totals(sl)
    assert tot[0] == pytest.approx(oracle.totals(P, ref)[0], rel=1e-13)
    assert pool.poll(other)[0] == n + 5
    pool.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pool_2d_equals_solver(lbsd, prec):
    """Square-lattice slots of several sizes and boundary conditions, one hot
    enough to need the full FIFO, and a non-planar random one."""
    cases = [(64, 64, 0), (300, 20, 1), (257, 129, 2), (1000, 7, 3)]
    probs = []
    for nx, ny, seed in cases:
        left, right, xd = inputs.riemann_instance(seed)
        probs.append((nx, ny, xd, left, right, inputs.cfl_lambda([left, right]), "transmissive", "periodic"))
    probs.append((150, 40, 0.5, (1.0, 0.0, 0.0, 1.0), (0.3, 0.0, 0.0, 0.1), 1.7 / np.sqrt(1.4),
                  "transmissive", "transmissive"))
    steps = 12
    ref = [alone(lbsd, 2, nx, ny, xd, L, R, lam, steps, prec, bx, by) for (nx, ny, xd, L, R, lam, bx, by) in probs]
    Yr = inputs.random_state(7, 2, 90, 61, vel=(-0.9, 0.9), e=(0.0, 3.0), smooth=3)
    s = lbsd.Solver(2, 90, 61, precision=prec, bc_x="periodic", bc_y="periodic")
    s.init_moments(Yr, 1.0)
    s.step(steps)
    ref_r = s.moments()
    s.close()
    pool = lbsd.Pool(2, 8, 64 << 20, precision=prec)
    for shape in (0, 3):
        slots = [pool.admit_riemann(nx, xd, L, R, steps, ny=ny, lam=lam, bc_x=bx, bc_y=by)
                 for (nx, ny, xd, L, R, lam, bx, by) in probs]
        sr = pool.admit_moments(Yr, 1.0, steps, bc_x="periodic", bc_y="periodic")
        pool.set_shape(shape)
        pool.use_graph(4)
        pool.advance(steps + 3)
        for i, sl in enumerate(slots):
            assert pool.poll(sl) == (steps, 1)
            assert np.array_equal(pool.moments(sl), ref[i]), (shape, i)
        assert np.array_equal(pool.moments(sr), ref_r)
        for sl in slots + [sr]:
            pool.release(sl)
    pool.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pool_walls_equal_solver(lbsd, prec):
    """Slots with reflecting walls beside open and periodic ones, on both
    lattices, long enough for waves to reflect: each equals its lb_solver
    run bit for bit, for two tile shapes."""
    SL, SR = inputs.SOD_LEFT, inputs.SOD_RIGHT
    lam = inputs.cfl_lambda([SL, SR])
    t1 = [(1000, 0.5, "reflecting"), (5, 0.5, "reflecting"), (333, 0.3, "transmissive"),
          (2049, 0.6, "periodic"), (700, 0.8, "reflecting")]
    t2 = [(64, 64, "reflecting", "reflecting"), (300, 20, "reflecting", "periodic"),
          (90, 45, "transmissive", "reflecting")]
    steps = 400
    ref1 = [alone(lbsd, 1, nx, 1, xd, SL, SR, lam, steps, prec, bx) for nx, xd, bx in t1]
    ref2 = [alone(lbsd, 2, nx, ny, 0.4, SL, SR, lam, 120, prec, bx, by) for nx, ny, bx, by in t2]
    states, center = inputs.quadrant_riemann(4)
    lq = inputs.quadrant_lambda(states)
    Yq = inputs.quadrant_moments(states, center, 61, 53)
    s = lbsd.Solver(2, 61, 53, precision=prec, bc_x="reflecting", bc_y="reflecting")
    s.init_moments(Yq, lq)
    s.step(40)
    ref_q = s.moments()
    s.close()
    p1 = lbsd.Pool(1, 8, 8 << 20, precision=prec)
    p2 = lbsd.Pool(2, 8, 64 << 20, precision=prec)
    for shape in (0, 2):
        s1 = [p1.admit_riemann(nx, xd, SL, SR, steps, lam=lam, bc_x=bx) for nx, xd, bx in t1]
        s2 = [p2.admit_riemann(nx, 0.4, SL, SR, 120, ny=ny, lam=lam, bc_x=bx, bc_y=by)
              for nx, ny, bx, by in t2]
        sq = p2.admit_moments(Yq, lq, 40, bc_x="reflecting", bc_y="reflecting")
        p1.set_shape(shape)
        p2.set_shape(shape)
        p1.advance(steps)
        p2.advance(120)
        for i, sl in enumerate(s1):
            assert np.array_equal(p1.moments(sl), ref1[i]), (shape, i)
            p1.release(sl)
        for i, sl in enumerate(s2):
            assert np.array_equal(p2.moments(sl), ref2[i]), (shape, i)
            p2.release(sl)
        assert np.array_equal(p2.moments(sq), ref_q)
        p2.release(sq)
    p1.close()
    p2.close()


def test_pool_continuous_admission_same_as_alone(lbsd):
    """Requests admitted while others are mid-run, released when done, their
    memory reused by later ones: each result equals its run alone."""
    reqs = inputs.serve_requests(3, 7, rate_per_s=1.0, side_lo=32, side_hi=200, steps_lo=5, steps_hi=60)
    refs = [alone(lbsd, 2, r["side"], r["side"], r["x_d"], r["left"], r["right"],
                  inputs.cfl_lambda([r["left"], r["right"]]), r["steps"], "fp32") for r in reqs]
    fp = [2 * 4 * r["side"] ** 2 * 4 for r in reqs]
    pool = lbsd.Pool(2, 3, max(fp) * 2 + (1 << 16), precision="fp32")
    pool.use_graph(4)
    pending, live, results = list(range(len(reqs))), {}, {}
    ticks = 0
    while pending or live:
        while pending:
            r = reqs[pending[0]]
            sl = pool.admit_riemann(r["side"], r["x_d"], r["left"], r["right"], r["steps"], ny=r["side"],
                                    lam=inputs.cfl_lambda([r["left"], r["right"]]))
            if sl is None:
                break
            live[sl] = pending.pop(0)
        pool.advance(5)
        ticks += 1
        for sl in list(live):
            done, status = pool.poll(sl)
            assert status in (0, 1)
            if status == 1:
                results[live.pop(sl)] = pool.moments(sl)
                pool.release(sl)
        assert ticks < 500
    for i in range(len(reqs)):
        assert np.array_equal(results[i], refs[i]), i
    pool.close()


def test_pool_full_and_failure_isolation(lbsd):
    pool = lbsd.Pool(1, 2, 2 * 3 * 4096 * 8 + 512, precision="fp64")
    a = pool.admit_riemann(4096, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, 100, lam=0.8)
    assert a is not None
    assert pool.admit_riemann(64, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, 10) is None  # arena full
    pool.release(a)
    # a slot whose packets outrun the halo fails at step k; the other finishes
    nx = 400
    left, right = inputs.SOD_LEFT, (1e-4, 0.0, 0.0, 1e-8)
    lam = 0.8 / np.sqrt(1.4)
    P = oracle.Problem(1, nx)
    Y = oracle.to_lattice(P, oracle.riemann_moments(P, inputs.node_x(nx), left, right, 0.5), lam)
    k = 0
    while k < 200:
        Y, st, r = oracle.step(P, Y)
        k += 1
        if r > 5:
            break
    assert 1 < k < 40
    bad = pool.admit_riemann(nx, 0.5, left, right, 50, lam=lam)
    good = pool.admit_riemann(400, 0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT, 50, lam=0.8)
    assert pool.admit_riemann(10, 0.5, left, right, 5) is None  # no free slot
    pool.advance(60)
    done, status = pool.poll(bad)
    assert status == lbsd.LB_EREACH and done == k - 1
    assert pool.poll(good) == (50, 1)
    ref = alone(lbsd, 1, nx, 1, 0.5, left, right, lam, k - 1, "fp64")
    assert np.array_equal(pool.moments(bad), ref)  # the last good step
    pool.close()


def test_pool_autotune_keeps_states(lbsd):
    probs = tube_set(2, 30, 256, 20000)
    pool = lbsd.Pool(1, 32, 64 << 20, precision="fp32")
    slots = [pool.admit_riemann(nx, xd, L, R, 1000, lam=lam) for (nx, xd, L, R, lam) in probs]
    pool.advance(3)
    before = [pool.moments(s) for s in slots]
    best, ms = pool.autotune(trials=3)
    assert 0 <= best < pool.shapes and pool.shape == best and ms > 0
    assert all(pool.poll(s)[0] == 3 for s in slots)
    for s, b in zip(slots, before):
        assert np.array_equal(pool.moments(s), b)
    pool.close()


def test_serve_loop_results_match_alone(lbsd):
    from paper_1602_02675_amd import serve

    reqs = inputs.serve_requests(11, 6, rate_per_s=200.0, side_lo=32, side_hi=160, steps_lo=5, steps_hi=50)
    refs = [alone(lbsd, 2, r["side"], r["side"], r["x_d"], r["left"], r["right"],
                  inputs.cfl_lambda([r["left"], r["right"]]), r["steps"], "fp32") for r in reqs]
    pool = lbsd.Pool(2, 2, 3 * 2 * 4 * 160 * 160 * 4, precision="fp32")
    pool.use_graph(5)
    got = {}
    res = serve.run(pool, reqs, tick=5, fetch="moments", on_result=lambda i, m: got.__setitem__(i, m))
    assert sorted(got) == list(range(len(reqs)))
    for i, ref in enumerate(refs):
        assert np.array_equal(got[i], ref), i
    lat = res["latency_s"]
    assert np.all(lat > 0) and res["p99_s"] >= res["p50_s"] > 0
    assert res["nups"] > 0 and pool.live == 0
    pool.close()


def test_snapshots_follow_stream_order(lbsd):
    """lb_pool_snapshot / lb_pool_snapshot_read: a snapshot shows the slots
    as they were when it was queued (steps done, status, totals equal to
    lb_pool_totals once synchronised); a slot released and admitted again
    after a snapshot was queued reads as free in it; releases and admissions
    queued behind running steps leave the others' results unchanged."""
    L, R = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1)
    lam = inputs.cfl_lambda([L, R])
    pool = lbsd.Pool(2, 3, 3 * 2 * 4 * 120 * 60 * 8, precision="fp64")
    a = pool.admit_riemann(120, 0.5, L, R, 6, ny=60, lam=lam)
    b = pool.admit_riemann(100, 0.4, L, R, 20, ny=40, lam=lam)
    pool.advance(4)
    pool.snapshot(0)
    pool.advance(4)  # a finishes at 6
    pool.snapshot(1)
    done0, st0, tot0 = pool.snapshot_read(0)
    assert (done0[a], st0[a], done0[b], st0[b]) == (4, 0, 4, 0)
    assert st0[2] == lbsd.LB_POOL_FREE and np.all(np.isnan(tot0[2]))
    done1, st1, tot1 = pool.snapshot_read(1)
    assert (done1[a], st1[a], done1[b], st1[b]) == (6, 1, 8, 0)
    np.testing.assert_array_equal(tot1[a], pool.totals(a))
    ref_a = alone(lbsd, 2, 120, 60, 0.5, L, R, lam, 6, "fp64")
    np.testing.assert_array_equal(pool.moments(a), ref_a)
    # release a and admit another problem into its slot while b's steps are queued
    pool.advance(4)
    pool.snapshot(0)  # queued before the release and the admission
    pool.release(a)
    c = pool.admit_riemann(80, 0.6, L, R, 3, ny=30, lam=lam)
    assert c == a  # the freed slot is reused
    pool.advance(8)
    pool.snapshot(1)
    done0, st0, _ = pool.snapshot_read(0)
    assert st0[c] == lbsd.LB_POOL_FREE  # the new occupant is not in the older snapshot
    assert (done0[b], st0[b]) == (12, 0)
    done1, st1, _ = pool.snapshot_read(1)
    assert (done1[c], st1[c], done1[b], st1[b]) == (3, 1, 20, 1)
    np.testing.assert_array_equal(pool.moments(b), alone(lbsd, 2, 100, 40, 0.4, L, R, lam, 20, "fp64"))
    np.testing.assert_array_equal(pool.moments(c), alone(lbsd, 2, 80, 30, 0.6, L, R, lam, 3, "fp64"))
    with pytest.raises(lbsd.LBError):
        pool.snapshot(2)
    pool.close()
