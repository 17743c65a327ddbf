"""Serving on the GPU: a request's result is the same when it is served alone and in a
mix of overlapping requests of other sizes, and equals the oracle's negacyclic product
with the resident key (bit-exact)."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")
from paper_2012_01968_amd.serve import GpuExecutor, Request, Server  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)
LOGNS = (10, 12, 14)
L_MAX = 8


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


@pytest.fixture(scope="module")
def setup():
    chain = synth.gen_primes(2000, 1 << max(LOGNS), 60, L_MAX)
    plans, keys, key_coeffs = {}, {}, {}
    for logN in LOGNS:
        N = 1 << logN
        plans[N] = ntt.ntt_plan_create(N, chain)
        coeff = synth.residue_batch(2100 + logN, chain, N, 1).reshape(L_MAX, N)
        key_coeffs[N] = coeff
        keys[N] = dev(oracle.forward(coeff, chain, oracle.roots(chain, N), THREADS))
    yield chain, plans, keys, key_coeffs
    for p in plans.values():
        p.destroy()


def make_requests(chain, n, rate, seed):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    reqs, host = [], {}
    for i in range(n):
        N = 1 << int(rng.choice(LOGNS))
        L = int(rng.integers(1, L_MAX + 1))
        data = synth.residue_batch(seed * 1000 + i, chain[:L], N, 2)
        host[i] = data.reshape(2, L, N)
        reqs.append(Request(i, N, L, float(t[i]), payload=dev(host[i])))
    return reqs, host


def serve(setup, reqs, policy, lanes=2, capacity=64 << 20):
    chain, plans, keys, _ = setup
    ex = GpuExecutor(plans, keys, capacity, lanes=lanes,
                     mode=ntt.BATCH_PLAIN if policy == "per_request" else ntt.BATCH_GROUPED)
    got = {}
    try:
        stats = Server(ex, capacity, policy=policy).run(
            reqs, on_complete=lambda r, v: got.__setitem__(r.rid, v.cpu().numpy().view(np.uint64).copy()))
    finally:
        ex.close()
    return stats, got


def expected(setup, r, data):
    chain, _, _, key_coeffs = setup
    primes = chain[:r.L]
    key = np.tile(key_coeffs[r.N][:r.L], (2, 1))
    return oracle.polymul(data.reshape(2 * r.L, r.N), key, primes, oracle.roots(primes, r.N),
                          THREADS).reshape(2, r.L, r.N)


def test_alone_equals_mix_equals_oracle(setup):
    chain = setup[0]
    reqs, host = make_requests(chain, 40, rate=200000, seed=7)   # arrivals overlap the running batches
    stats, mix = serve(setup, reqs, "continuous", lanes=3, capacity=8 << 20)
    assert stats.completed == 40 and stats.failed == stats.rejected == 0
    assert stats.mean_batch > 1
    for r in reqs:
        alone_req = Request(r.rid, r.N, r.L, 0.0, payload=r.payload)
        _, alone = serve(setup, [alone_req], "continuous", lanes=1)
        assert np.array_equal(alone[r.rid], mix[r.rid]), f"request {r.rid} N={r.N} L={r.L}"
        assert np.array_equal(mix[r.rid], expected(setup, r, host[r.rid])), f"request {r.rid}"


def test_per_request_path_matches(setup):
    chain = setup[0]
    reqs, host = make_requests(chain, 24, rate=100000, seed=8)
    stats, got = serve(setup, reqs, "per_request")
    assert stats.completed == 24 and stats.batches == 24
    for r in reqs:
        assert np.array_equal(got[r.rid], expected(setup, r, host[r.rid])), f"request {r.rid}"


def test_back_pressure_and_rejection_on_device(setup):
    chain = setup[0]
    reqs, host = make_requests(chain, 16, rate=1e6, seed=9)
    reqs.append(Request(99, 1 << 11, 2, 0.0))                        # no plan for this N
    big = max(8 * r.words for r in reqs[:16])
    stats, got = serve(setup, reqs, "continuous", lanes=2, capacity=2 * big + 4096)
    assert stats.completed == 16 and stats.rejected == 1
    assert stats.peak_bytes <= 2 * big + 4096
    for r in reqs[:16]:
        assert np.array_equal(got[r.rid], expected(setup, r, host[r.rid])), f"request {r.rid}"
