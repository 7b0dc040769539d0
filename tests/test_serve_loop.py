"""The serving loop's host logic (paper_1602_02675_amd/serve.py) on a
stand-in pool that follows the snapshot rules of include/lbsd.h on the CPU:
steps are applied when queued, a snapshot records every slot's progress and
admission count when it is queued, and a slot admitted again since then
reads as LB_POOL_FREE in it.  No device work: this checks that every request
is admitted once, collected once with its own result, and that the loop keeps
at most one tick queued ahead of the snapshot it waits for.
"""
import numpy as np
import pytest

from paper_1602_02675_amd import inputs, serve
from paper_1602_02675_amd.lbsd import LB_POOL_FREE


class FakePool:
    def __init__(self, max_slots, arena_bytes):
        self.max_slots, self.arena_bytes = max_slots, arena_bytes
        self.slots = [None] * max_slots  # dict(side, target, done, gen, req) or None
        self.gen = [0] * max_slots
        self.snaps = [None, None]
        self.queued_ticks = 0  # ticks queued after the newest snapshot read
        self.max_ahead = 0
        self.admissions = 0

    def footprint(self, nx, ny):
        return 32 * nx * ny

    def _used(self):
        return sum(self.footprint(q["side"], q["side"]) for q in self.slots if q is not None)

    def admit_riemann(self, side, x_d, left, right, steps, *, ny, lam):
        free = [i for i, q in enumerate(self.slots) if q is None]
        if not free or self._used() + self.footprint(side, ny) > self.arena_bytes:
            return None
        i = free[0]
        self.gen[i] += 1
        self.slots[i] = dict(side=side, target=steps, done=0, gen=self.gen[i], x_d=x_d)
        self.admissions += 1
        return i

    def advance(self, n):
        for q in self.slots:
            if q is not None:
                q["done"] = min(q["target"], q["done"] + n)
        self.queued_ticks += 1
        self.max_ahead = max(self.max_ahead, self.queued_ticks)

    def snapshot(self, buf):
        self.snaps[buf] = [None if q is None else dict(q) for q in self.slots]

    def snapshot_read(self, buf):
        snap = self.snaps[buf]
        self.queued_ticks = max(0, self.queued_ticks - 1)
        done = np.zeros(self.max_slots, dtype=np.int64)
        st = np.full(self.max_slots, LB_POOL_FREE, dtype=np.int32)
        tot = np.full((self.max_slots, 4), np.nan)
        for i, q in enumerate(snap):
            cur = self.slots[i]
            if q is None or cur is None or cur["gen"] != q["gen"]:
                continue
            done[i] = q["done"]
            st[i] = 1 if q["done"] >= q["target"] else 0
            tot[i] = [q["side"], q["done"], q["x_d"], 0.0]
        return done, st, tot

    def release(self, slot):
        assert self.slots[slot] is not None
        self.slots[slot] = None

    def moments(self, slot):
        q = self.slots[slot]
        return np.array([q["side"], q["done"]])

    @property
    def live(self):
        return sum(q is not None for q in self.slots)


@pytest.mark.parametrize("slots,arena_sides,fetch", [(4, 4, "totals"), (2, 1, "totals"), (3, 2, "moments")])
def test_every_request_collected_once_with_its_result(slots, arena_sides, fetch):
    reqs = inputs.serve_requests(5, 40, rate_per_s=2000.0, side_lo=16, side_hi=64, steps_lo=3, steps_hi=60)
    pool = FakePool(slots, arena_sides * 32 * 64 * 64)
    got = {}

    def on_result(i, res):
        assert i not in got
        got[i] = res

    res = serve.run(pool, reqs, tick=7, fetch=fetch, on_result=on_result)
    assert sorted(got) == list(range(len(reqs)))
    assert pool.admissions == len(reqs) and pool.live == 0
    for i, r in enumerate(reqs):
        if fetch == "totals":
            side, done, x_d, _ = got[i]
            assert (side, done, x_d) == (r["side"], r["steps"], r["x_d"])
        else:
            assert list(got[i]) == [r["side"], r["steps"]]
    lat = res["latency_s"]
    assert np.all(lat > 0) and res["p99_s"] >= res["p50_s"] > 0
    # one tick queued ahead of the snapshot being read, never more
    assert pool.max_ahead <= 2


def test_request_that_never_fits_is_refused():
    reqs = inputs.serve_requests(1, 3, rate_per_s=100.0, side_lo=64, side_hi=64)
    pool = FakePool(2, 32 * 32 * 32)
    with pytest.raises(ValueError):
        serve.run(pool, reqs, tick=5)
