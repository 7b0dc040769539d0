"""Pins of the oracle's per-node equilibrium against what the paper fixes.

Each test checks the oracle (oracle/lb_oracle.c) against something other than
itself: hand-derived tables, the moment identities the equilibrium is built to
satisfy (eq. 16-18, 22, 24-25), the printed lattice speeds (Sec. IV) and an
independent construction of the linear / bilinear split (eq. 28-29) as a hat
function.
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _node(dim, rho, v, E):
    v = list(v)
    return [rho] + [rho * c for c in v] + [rho * E]


def _speed_table(P, node):
    """mass per |c'| and zeta per |c'| for a node at rest (all mass on corner 0)."""
    off, pay = oracle.packets(P, node)
    mass, zeta = {}, {}
    for o, p in zip(off, pay):
        if p[0] == 0.0:
            continue
        sp = int(max(abs(o[0]), abs(o[1])))
        mass[sp] = mass.get(sp, 0.0) + p[0]
        zeta.setdefault(sp, p[-1] / p[0])
    return mass, zeta


@pytest.fixture(scope="module")
def tables():
    return json.load(open(os.path.join(GOLDEN, "equilibrium_tables.json")))


def test_hand_tables(tables):
    g = tables["gamma"]
    for c in tables["cases"]:
        P = oracle.Problem(c["dim"], 4, 4, gamma=g, delta0=c["delta0"])
        rho, v, p = c["rho"], c["v"], c["p"]
        E = c["e"] + 0.5 * sum(x * x for x in v)
        node = _node(c["dim"], rho, v, E)
        L = oracle.levels(P, node)
        assert L["e"] == pytest.approx(c["e"], rel=1e-14)
        assert L["phi"] == pytest.approx(c["phi"], rel=1e-14)
        assert L["A"] == pytest.approx(c["A"], rel=1e-14)
        if not c.get("boundary"):
            assert (L["c1"], L["c2"]) == (c["c1"], c["c2"]), c["name"]
            assert L["d0"] == pytest.approx(c["d0"], rel=1e-14, abs=1e-17)
            assert L["d1"] == pytest.approx(c["d1"], rel=1e-13, abs=1e-17)
            assert L["d2"] == pytest.approx(c["d2"], rel=1e-13, abs=1e-17)
        mass, zeta = _speed_table(P, node)
        for sp, m in c["mass_by_speed"].items():
            assert mass.get(int(sp), 0.0) == pytest.approx(m, rel=1e-13, abs=1e-15), (c["name"], sp)
        for sp, z in c["zeta_by_lane_speed"].items():
            if mass.get(int(sp), 0.0) > 1e-12:
                assert zeta[int(sp)] == pytest.approx(z, rel=1e-13), (c["name"], sp)
        off, pay = oracle.packets(P, node)
        assert pay[:, -1].sum() == pytest.approx(c["sum_m_zeta"], rel=1e-13)
        # pressure from eq. 27
        assert (g - 1.0) * rho * L["e"] == pytest.approx(p, rel=1e-13)


def test_moving_node_split(tables):
    mv = tables["moving"]
    P = oracle.Problem(1, 4)
    off, pay = oracle.packets(P, _node(1, mv["rho"], [mv["u"]], mv["E"]))
    L = oracle.levels(P, _node(1, mv["rho"], [mv["u"]], mv["E"]))
    assert L["f"] == (mv["f"],)
    # corner-0 / corner-1 mass shares of every lane
    lanes = {}
    for o, p in zip(off, pay):
        xi = p[1] / p[0] if p[0] else None
        lanes.setdefault(round(xi, 12) if xi is not None else None, []).append((int(o[0]), p[0]))
    for lane, xi in mv["xi_by_lane"].items():
        got = lanes[round(xi, 12)]
        c = int(lane)
        tot = sum(m for _, m in got)
        by_off = {o: m / tot for o, m in got}
        assert by_off[mv["f"] + c] == pytest.approx(mv["alpha"][0], rel=1e-13)
        assert by_off[mv["f"] + 1 + c] == pytest.approx(mv["alpha"][1], rel=1e-13)
    assert pay[:, 1].sum() == pytest.approx(mv["sum_m_xi"], rel=1e-13)
    assert pay[:, 2].sum() == pytest.approx(mv["sum_m_zeta"], rel=1e-13)
    # mirrored velocity: floor node x - 1 carries 0.3, node x carries 0.7
    Lm = oracle.levels(P, _node(1, mv["rho"], [-mv["u"]], mv["E"]))
    assert Lm["f"] == (mv["mirror_f"],)
    offm, paym = oracle.packets(P, _node(1, mv["rho"], [-mv["u"]], mv["E"]))
    rest = [(int(o[0]), p[0]) for o, p in zip(offm, paym) if abs(p[1] / p[0] - (-mv["u"])) < 1e-12]
    tot = sum(m for _, m in rest)
    by_off = {o: m / tot for o, m in rest}
    assert by_off[-1] == pytest.approx(mv["mirror_alpha"][0], rel=1e-13)
    assert by_off[0] == pytest.approx(mv["mirror_alpha"][1], rel=1e-13)


def test_printed_lattice_speeds_at_sod_states():
    """Sec. IV prints |c'| = 1, 2 for both lattices; eq. 26 reproduces them at
    Sod's states, in lattice units of lambda = 1 and of the CFL rule."""
    const = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    sod = const["sod"]
    for lam in (1.0, 1.0 / np.sqrt(1.4)):
        for dim, key in ((1, "lattice_1d"), (2, "lattice_2d")):
            P = oracle.Problem(dim, 4, 4)
            for rho, p in ((sod["rho_L"], sod["p_L"]), (sod["rho_R"], sod["p_R"])):
                e = p / (0.4 * rho) * lam * lam
                L = oracle.levels(P, _node(dim, rho, [0.0] * dim, e))
                assert [L["c1"], L["c2"]] == const[key]["speeds"][-2:]
                assert list(L["b"]) == const[key]["b"]


def _rand_nodes(dim, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rho = rng.uniform(0.01, 5.0)
        v = rng.uniform(-2.5, 2.5, size=dim)
        e = rng.choice([rng.uniform(0, 0.05), rng.uniform(0, 3), rng.uniform(3, 15)])
        out.append((rho, v, e))
    return out


@pytest.mark.parametrize("dim", [1, 2])
def test_moment_reproduction(dim):
    """eq. 22: the packets of f_eq sum to the node's own moments."""
    for delta0 in ((0.4, 0.5, 0.55) if dim == 1 else (0.0,)):
        P = oracle.Problem(dim, 4, 4, delta0=delta0)
        for rho, v, e in _rand_nodes(dim, 300, 1 + dim):
            node = _node(dim, rho, v, e + 0.5 * float(v @ v))
            off, pay = oracle.packets(P, node)
            assert len(off) == (10 if dim == 1 else 32)
            tot = pay.sum(axis=0)
            scale = np.array([rho] + [rho * (abs(c) + np.sqrt(e) + 1) for c in v] + [node[-1] + rho])
            assert np.all(np.abs(tot - np.array(node)) <= 4e-15 * scale * 8), (tot, node)


@pytest.mark.parametrize("dim", [1, 2])
def test_pressure_tensor_and_weights(dim):
    """eq. 17 with eq. 24-25: sum m (xi - v)(xi - v)^T = p I, all d >= 0,
    sum_v b_v d_v = rho and sum_v b_v d_v c_v^2 = D p."""
    g = 1.4
    P = oracle.Problem(dim, 4, 4, gamma=g)
    for rho, v, e in _rand_nodes(dim, 300, 7 + dim):
        node = _node(dim, rho, v, e + 0.5 * float(v @ v))
        L = oracle.levels(P, node)
        p = (g - 1.0) * rho * L["e"]
        for d in (L["d0"], L["d1"], L["d2"]):
            assert d >= -1e-15 * rho
        b0, b1, b2 = L["b"]
        assert b0 * L["d0"] + b1 * L["d1"] + b2 * L["d2"] == pytest.approx(rho, rel=1e-14)
        assert b1 * L["d1"] * L["c1"] ** 2 + b2 * L["d2"] * L["c2"] ** 2 == pytest.approx(
            dim * p, rel=1e-12, abs=1e-14 * rho)
        assert L["c1"] ** 2 <= L["A"] < L["c2"] ** 2
        off, pay = oracle.packets(P, node)
        m = pay[:, 0]
        xi = pay[:, 1:1 + dim] / np.where(m > 0, m, 1)[:, None]
        dv = xi - np.asarray(v)[None, :]
        T = np.einsum("p,pa,pb->ab", m, dv, dv)
        assert np.allclose(T, p * np.eye(dim), rtol=1e-11, atol=1e-12 * rho)


@pytest.mark.parametrize("dim", [1, 2])
def test_velocity_set_symmetry(dim):
    """eq. 16-18 per level: sum c' = 0, sum c' c' = (b_v / D) c_v^2 I, sum c'c'c' = 0."""
    P = oracle.Problem(dim, 4, 4)
    node = _node(dim, 1.0, [0.0] * dim, 4.0)  # at rest: corner 0 carries the lane, c'_1 >= 1
    L = oracle.levels(P, node)
    assert L["c1"] >= 1
    off, pay = oracle.packets(P, node)
    by_level = {}
    for o, p in zip(off, pay):
        if p[0] == 0.0:
            continue
        c = o[:dim].astype(float)
        sp = int(np.max(np.abs(c)))
        by_level.setdefault(sp, []).append(c)
    b = {0: L["b"][0], L["c1"]: L["b"][1], L["c2"]: L["b"][2]}
    for sp, cs in by_level.items():
        cs = np.array(cs)
        assert len(cs) == b[sp]
        assert np.all(cs.sum(axis=0) == 0)
        assert np.array_equal(np.einsum("ja,jb->ab", cs, cs), (b[sp] / dim) * sp * sp * np.eye(dim))
        assert np.all(np.einsum("ja,jb,jc->abc", cs, cs, cs) == 0)


@pytest.mark.parametrize("dim", [1, 2])
def test_split_is_a_hat_function(dim):
    """eq. 28-29 rebuilt independently: the packet of lane c' lands at the
    continuous point x + v + c' and is shared by the surrounding nodes y with
    weight prod_axis max(0, 1 - |y - (x + v + c')|)."""
    P = oracle.Problem(dim, 4, 4)
    rng = np.random.default_rng(11)
    for _ in range(200):
        rho = rng.uniform(0.1, 2.0)
        v = rng.uniform(-2.2, 2.2, size=dim)
        if rng.random() < 0.2:
            v = np.round(v)  # integer velocities: the far corner gets weight 0
        node = _node(dim, rho, v, 1.0 + 0.5 * float(v @ v))
        off, pay = oracle.packets(P, node)
        m = pay[:, 0]
        xi = pay[:, 1:1 + dim] / np.where(m > 0, m, 1)[:, None]
        # group the packets of each lane: all corners of a lane share xi
        L = oracle.levels(P, node)
        lanes = {}
        for o, mm, x in zip(off, m, xi):
            if mm <= 1e-9 * rho:  # xi = (m xi) / m is only accurate for non-tiny m
                continue
            key = tuple(np.round(x - v, 9))
            lanes.setdefault(key, []).append((o[:dim].astype(float), mm))
        for cprime, pk in lanes.items():
            cp = np.array(cprime)
            lane_mass = sum(mm for _, mm in pk)
            end = v + cp
            if len(pk) < 2 ** dim and np.any(np.abs(end - np.round(end)) > 1e-6):
                continue  # a corner of this lane was filtered as tiny
            share = {}  # lanes with equal c' (c'_1 = 0) coincide: compare per node
            for o, mm in pk:
                share[tuple(o)] = share.get(tuple(o), 0.0) + mm / lane_mass
            for o, sh in share.items():
                w = np.prod(np.maximum(0.0, 1.0 - np.abs(np.array(o) - end)))
                assert sh == pytest.approx(w, abs=1e-13)
            # the mass-weighted mean landing point is x + v + c' (centre of mass)
            com = sum(mm * o for o, mm in pk) / lane_mass
            assert np.allclose(com, end, atol=1e-12)
        assert all(isinstance(f, int) for f in L["f"])


def test_rho_zero_emits_nothing():
    P = oracle.Problem(1, 4)
    off, pay = oracle.packets(P, [0.0, 0.0, 0.0])
    assert len(off) == 0
