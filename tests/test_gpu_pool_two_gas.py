"""GPU tests of pools of two-gas problems (lb_pool_create_two_gas), through
the C ABI: every slot (species field rho chi last) equals its lb_solver run
of the same problem bit for bit, on both lattices, across tile shapes, graph
capture and walls; the solver's two-gas parity with the oracle is tested in
test_gpu_two_gas and test_gpu_two_gas2d."""
import numpy as np
import pytest

from paper_1602_02675_amd import inputs

pytestmark = pytest.mark.gpu

G1, G2 = 1.4, 5.0 / 3.0


@pytest.fixture(scope="module")
def lbsd():
    import torch

    assert torch.cuda.is_available()
    from paper_1602_02675_amd import lbsd as m

    return m


def alone(lbsd, dim, nx, ny, x_d, left, right, lam, steps, prec, bc_x="transmissive", bc_y="periodic",
          d0_frac=None):
    s = lbsd.Solver(dim, nx, ny, precision=prec, bc_x=bc_x, bc_y=bc_y, gamma=G1, gamma2=G2, d0_frac=d0_frac)
    s.init_riemann(x_d, left, right, lam=lam)
    s.step(steps)
    out = s.moments()
    s.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pool_1d_two_gas_equals_solver(lbsd, prec):
    SL, SR = inputs.SOD_LEFT, inputs.SOD_RIGHT
    lam = 0.9 / max(abs(u) + np.sqrt(g * p / r) for (r, u, _, p), g in ((SL, G1), (SR, G2)))
    tubes = [(1000, 0.5, "reflecting"), (5, 0.5, "reflecting"), (333, 0.3, "transmissive"),
             (2049, 0.6, "periodic"), (1, 0.5, "transmissive"), (4100, 0.45, "transmissive")]
    steps = 300
    ref = [alone(lbsd, 1, nx, 1, xd, SL, SR, lam, steps, prec, bx) for nx, xd, bx in tubes]
    pool = lbsd.Pool(1, 8, 8 << 20, precision=prec, gamma=G1, gamma2=G2)
    assert pool.nf == 4
    for shape, graph in ((0, 0), (2, 8), (4, 0)):
        slots = [pool.admit_riemann(nx, xd, SL, SR, steps, lam=lam, bc_x=bx) for nx, xd, bx in tubes]
        pool.set_shape(shape)
        pool.use_graph(graph)
        pool.advance(steps + 3)
        for i, sl in enumerate(slots):
            assert pool.poll(sl) == (steps, 1)
            got = pool.moments(sl)
            assert got.shape == (4, 1, tubes[i][0])
            assert np.array_equal(got, ref[i]), (shape, graph, i)
            pool.release(sl)
    pool.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d0_frac", [None, 0.4])
def test_pool_2d_two_gas_equals_solver(lbsd, prec, d0_frac):
    SL, SR = inputs.SOD_LEFT, inputs.SOD_RIGHT
    lam = 0.9 / max(abs(u) + np.sqrt(g * p / r) for (r, u, _, p), g in ((SL, G1), (SR, G2)))
    probs = [(64, 64, "reflecting", "reflecting"), (300, 20, "transmissive", "periodic"),
             (90, 45, "reflecting", "transmissive")]
    steps = 60
    ref = [alone(lbsd, 2, nx, ny, 0.4, SL, SR, lam, steps, prec, bx, by, d0_frac) for nx, ny, bx, by in probs]
    # a non-planar two-gas state: quadrants of alternating gas
    states, center = inputs.quadrant_riemann(5)
    nq, mq = 61, 53
    Ya = inputs.quadrant_moments(states, center, nq, mq, gamma=G1)
    Yb = inputs.quadrant_moments(states, center, nq, mq, gamma=G2)
    X, Yy = np.meshgrid(inputs.node_x(nq), (np.arange(mq) + 0.5) / nq)
    gas1 = (X >= center[0]) == (Yy >= center[1])
    Yq = np.concatenate([np.where(gas1[None], Ya, Yb), (Ya[0] * gas1)[None]], axis=0)
    lq = min(inputs.quadrant_lambda(states, gamma=G1), inputs.quadrant_lambda(states, gamma=G2))
    s = lbsd.Solver(2, nq, mq, precision=prec, bc_x="reflecting", bc_y="reflecting", gamma=G1, gamma2=G2,
                    d0_frac=d0_frac)
    s.init_moments(Yq, lq)
    s.step(25)
    ref_q = s.moments()
    s.close()
    pool = lbsd.Pool(2, 8, 64 << 20, precision=prec, gamma=G1, gamma2=G2, d0_frac=d0_frac)
    assert pool.nf == 5
    for shape in (0, 2):
        slots = [pool.admit_riemann(nx, 0.4, SL, SR, steps, ny=ny, lam=lam, bc_x=bx, bc_y=by)
                 for nx, ny, bx, by in probs]
        sq = pool.admit_moments(Yq, lq, 25, bc_x="reflecting", bc_y="reflecting")
        pool.set_shape(shape)
        pool.advance(steps)
        for i, sl in enumerate(slots):
            assert np.array_equal(pool.moments(sl), ref[i]), (shape, i)
            pool.release(sl)
        assert np.array_equal(pool.moments(sq), ref_q), shape
        pool.release(sq)
    pool.close()


def test_pool_two_gas_admission_checks_species(lbsd):
    nx, ny = 32, 16
    Y = inputs.random_state(71, 2, nx, ny, vel=(-1.0, 1.0), e=(0.1, 1.0))
    pool = lbsd.Pool(2, 2, 8 << 20, precision="fp64", gamma=G1, gamma2=G2)
    with pytest.raises(lbsd.LBError) as ei:
        pool.admit_moments(np.concatenate([Y, 1.5 * Y[:1]], axis=0), 1.0, 5)
    assert ei.value.code == lbsd.LB_ESTATE
    assert pool.live == 0
    sl = pool.admit_moments(np.concatenate([Y, 0.5 * Y[:1]], axis=0), 1.0, 5)
    pool.advance(5)
    assert pool.poll(sl) == (5, 1)
    chi = pool.moments(sl)
    assert np.all(chi[4] >= 0) and np.all(chi[4] <= chi[0] * (1 + 1e-12))
    pool.close()


def test_serve_loop_two_gas_results_match_alone(lbsd):
    """The serving loop on a two-gas FP32 pool: requests admitted as slots
    free up, each result bit-equal to its lb_solver run."""
    from paper_1602_02675_amd import serve

    reqs = inputs.serve_requests(12, 6, rate_per_s=200.0, side_lo=32, side_hi=160, steps_lo=5, steps_hi=50)
    refs = [alone(lbsd, 2, r["side"], r["side"], r["x_d"], r["left"], r["right"],
                  inputs.cfl_lambda([r["left"], r["right"]]), r["steps"], "fp32") for r in reqs]
    pool = lbsd.Pool(2, 2, 3 * 2 * 5 * 160 * 160 * 4, precision="fp32", gamma=G1, gamma2=G2)
    pool.use_graph(5)
    got = {}
    res = serve.run(pool, reqs, tick=5, fetch="moments", on_result=lambda i, m: got.__setitem__(i, m))
    assert sorted(got) == list(range(len(reqs)))
    for i, ref in enumerate(refs):
        assert got[i].shape == (5, reqs[i]["side"], reqs[i]["side"])
        assert np.array_equal(got[i], ref), i
    assert res["nups"] > 0 and pool.live == 0
    pool.close()
