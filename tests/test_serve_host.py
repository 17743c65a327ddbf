"""Host logic of the request loop: the footprint pool, percentiles, and the scheduler
driven by a fake executor on a virtual clock (no GPU)."""
import math
import random

import numpy as np
import pytest

from paper_2012_01968_amd.serve import FootprintPool, Request, Server, percentile


# ------------------------------------------------------------------ footprint pool

def test_pool_matches_a_bitmap_model():
    rng = random.Random(3)
    cap, align = 64 * 256, 256
    pool = FootprintPool(cap, align)
    used = np.zeros(cap // align, bool)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            pool.free(off)
            used[off // align: off // align + live.pop(off)] = False
        else:
            nb = rng.randint(1, 9 * align)
            units = -(-nb // align)
            off = pool.alloc(nb)
            # first fit: the lowest start of a free run of `units` slots
            want = None
            for s in range(len(used) - units + 1):
                if not used[s:s + units].any():
                    want = s * align
                    break
            assert off == want
            if off is not None:
                used[off // align: off // align + units] = True
                live[off] = units
        pool.check()
        assert pool.used == used.sum() * align
    for off in list(live):
        pool.free(off)
    pool.check()
    assert pool.largest_free() == pool.capacity and pool.used == 0


def test_pool_rejects_double_free_and_bad_args():
    pool = FootprintPool(4096)
    off = pool.alloc(100)
    pool.free(off)
    with pytest.raises(KeyError):
        pool.free(off)
    with pytest.raises(ValueError):
        FootprintPool(0)
    with pytest.raises(ValueError):
        FootprintPool(4096, 100)


def test_percentile_is_nearest_rank():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 100, 1001):
        xs = rng.random(n).tolist()
        for p in (0, 1, 50, 90, 99, 100):
            assert percentile(xs, p) == np.percentile(xs, p, method="inverted_cdf")
    assert math.isnan(percentile([], 50))


# ------------------------------------------------------------------ scheduler on a virtual clock

class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class FakeExecutor:
    """Completes a batch `fixed + per_word * words` seconds after its launch, or after the
    previous batch on its lane, whichever is later; a result is payload * 3 + rid."""

    def __init__(self, clock, lanes=2, fixed=1e-4, per_word=1e-9, Ns=(16, 32, 64), L_max=8, poison=()):
        self.clock, self.lanes, self.fixed, self.per_word = clock, lanes, fixed, per_word
        self.Ns, self.L_max, self.poison = set(Ns), L_max, set(poison)
        self.lane_free = [0.0] * lanes
        self.results = {}
        self.pool = None
        self.launched = []

    def validate(self, r):
        if r.N not in self.Ns:
            return f"no plan for N={r.N}"
        if not 1 <= r.L <= self.L_max:
            return "bad L"
        return ""

    def footprint(self, r):
        return 8 * r.words

    def start(self, clock):
        self.t0 = clock()
        return self.t0

    def launch(self, lane, batch):
        if any(r.rid in self.poison for r in batch):
            raise RuntimeError("poisoned request")
        now = self.clock()
        if self.pool is not None:
            assert self.pool.used <= self.pool.capacity
        start = max(now, self.lane_free[lane])
        done = start + self.fixed + self.per_word * sum(r.words for r in batch)
        self.lane_free[lane] = done
        for r in batch:
            self.results[r.rid] = np.asarray(r.payload) * 3 + r.rid
        self.launched.append((lane, [r.rid for r in batch], now))
        return done

    def poll(self, tok):
        return self.clock() >= tok

    def finish_time(self, tok):
        return tok - self.t0

    def view(self, r):
        return self.results[r.rid]


def make_requests(n, rate, seed=1, Ns=(16, 32, 64)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    out = []
    for i in range(n):
        N = int(rng.choice(Ns))
        L = int(rng.integers(1, 9))
        out.append(Request(i, N, L, float(t[i]), payload=np.full((2, L, N), i, np.int64)))
    return out


def run(reqs, policy="continuous", capacity=1 << 20, lanes=2, **kw):
    clk = VClock()
    ex = FakeExecutor(clk, lanes=lanes, **kw)
    srv = Server(ex, capacity, policy=policy, clock=clk, sleep=clk.sleep)
    ex.pool = srv.pool
    got = {}
    stats = srv.run(reqs, on_complete=lambda r, v: got.__setitem__(r.rid, v.copy()))
    return stats, got, ex, srv


@pytest.mark.parametrize("policy", ["continuous", "per_request"])
def test_every_request_completes_with_its_own_result(policy):
    reqs = make_requests(300, rate=20000)
    stats, got, ex, srv = run(reqs, policy)
    assert stats.completed == 300 and stats.rejected == stats.failed == 0
    for r in reqs:
        assert r.status == "done" and r.done_t >= r.arrival
        assert np.array_equal(got[r.rid], np.full((2, r.L, r.N), r.rid * 4, np.int64))
    srv.pool.check()
    assert srv.pool.used == 0
    if policy == "per_request":
        assert stats.batches == 300 and all(lane == 0 for lane, _, _ in ex.launched)
    else:
        assert stats.batches < 300 and stats.mean_batch > 1    # arrivals during busy lanes were merged


def test_continuous_batching_keeps_lanes_bounded_and_fifo():
    reqs = make_requests(200, rate=50000, seed=2)
    stats, got, ex, srv = run(reqs, lanes=3, per_word=5e-8)
    order = [rid for _, rids, _ in ex.launched for rid in rids]
    assert order == sorted(order)                               # FIFO admission and launch
    # never more than `lanes` batches in flight: each launch happens once a lane is free
    for k, (lane, rids, t) in enumerate(ex.launched):
        inflight = 0
        for lane2, rids2, t2 in ex.launched[:k]:
            done = max(r.done_t for r in reqs if r.rid in rids2)
            if done + ex.t0 > t:
                inflight += 1
        assert inflight < 3


def test_back_pressure_holds_requests_until_memory_frees():
    reqs = [Request(i, 64, 8, 0.0, payload=np.zeros((2, 8, 64), np.int64)) for i in range(10)]
    per = 8 * 2 * 8 * 64
    stats, got, ex, srv = run(reqs, capacity=3 * per, lanes=4)
    assert stats.completed == 10
    assert srv.pool.peak <= 3 * per
    # at most three requests were admitted at once, so no batch holds more than three
    assert max(len(rids) for _, rids, _ in ex.launched) <= 3


def test_rejections_and_failures_are_isolated():
    reqs = make_requests(60, rate=10000, seed=4)
    reqs.append(Request(100, 128, 2, 0.001))                    # no plan for this N
    reqs.append(Request(101, 16, 40, 0.001))                    # too many limbs
    reqs.append(Request(102, 64, 8, 0.001, polys=2000))         # larger than the arena
    stats, got, ex, srv = run(reqs, policy="per_request", capacity=1 << 20, poison={7})
    by = {r.rid: r for r in reqs}
    assert by[100].status == by[101].status == by[102].status == "rejected"
    assert by[7].status == "failed" and "poisoned" in by[7].error
    assert stats.rejected == 3 and stats.failed == 1 and stats.completed == 59
    for r in reqs:
        if r.status == "done":
            assert np.array_equal(got[r.rid], np.full((2, r.L, r.N), r.rid * 4, np.int64))
    assert srv.pool.used == 0


def test_latency_accounting_on_a_fixed_timeline():
    # one lane, 1 ms per batch, three requests: two together at t=0, one at t=0.5 ms
    reqs = [Request(0, 16, 1, 0.0, payload=np.zeros((2, 1, 16))),
            Request(1, 16, 1, 0.0, payload=np.zeros((2, 1, 16))),
            Request(2, 16, 1, 0.0005, payload=np.zeros((2, 1, 16)))]
    stats, got, ex, srv = run(reqs, lanes=1, fixed=1e-3, per_word=0.0)
    assert [rids for _, rids, _ in ex.launched] == [[0, 1], [2]]
    assert reqs[0].latency == pytest.approx(1e-3, abs=1e-6)
    assert reqs[2].latency == pytest.approx(1.5e-3, abs=1e-4)   # waited for the lane, then 1 ms
    assert stats.p50_ms == pytest.approx(1.0, abs=1e-3)
