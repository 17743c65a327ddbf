"""Bit-exact parity of the HIP path against the CPU oracle, through the C ABI.

Every comparison is exact (tolerance 0): the arithmetic is integer, so exactly one
correct output exists for each (prime, root convention, output order).  Inputs come
from ``synth``; expected values come only from ``oracle``.
"""
import os
import random

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")

THREADS = min(16, os.cpu_count() or 1)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint64)


def make(N, L, P, bits, seed, n_max=None):
    primes = synth.gen_primes(seed, n_max or N, bits, L)
    data = synth.residue_batch(seed, primes, N, P)
    return primes, oracle.roots(primes, N), data


def run_fwd(plan, data):
    d = dev(data)
    ntt.ntt_forward(plan, d)
    torch.cuda.synchronize()
    return host(d)


def run_inv(plan, data):
    d = dev(data)
    ntt.ntt_inverse(plan, d)
    torch.cuda.synchronize()
    return host(d)


def check_fwd_inv(N, L, P, bits, seed, **opts):
    primes, psis, data = make(N, L, P, bits, seed)
    plan = ntt.ntt_plan_create(N, primes, **opts)
    try:
        assert ntt.ntt_plan_get_roots(plan) == psis
        want = oracle.forward(data, primes, psis, THREADS)
        got = run_fwd(plan, data)
        assert np.array_equal(got, want), f"forward mismatch N={N} opts={opts}"
        back = run_inv(plan, want)
        assert np.array_equal(back, data), f"inverse(forward) mismatch N={N} opts={opts}"
        # inverse of arbitrary NTT-domain vectors against the oracle's inverse
        want_i = oracle.inverse(data, primes, psis, THREADS)
        assert np.array_equal(run_inv(plan, data), want_i), f"inverse mismatch N={N} opts={opts}"
    finally:
        plan.destroy()


# ------------------------------------------------------------------ every size

@pytest.mark.parametrize("logN", list(range(1, 18)))
def test_every_size_table(logN):
    N = 1 << logN
    L, P = (3, 2) if logN >= 12 else (5, 3)   # small sizes: ragged vector counts per workgroup
    check_fwd_inv(N, L, P, 60, 100 + logN)


@pytest.mark.parametrize("logN", [11, 12, 13, 14, 15, 16, 17])
@pytest.mark.parametrize("ots", [1, 2])
def test_every_size_ot(logN, ots):
    check_fwd_inv(1 << logN, 3, 2, 60, 200 + logN, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=ots)


@pytest.mark.parametrize("logN,base", [(4, 2), (6, 3), (8, 4), (10, 5)])
def test_ot_small_bases(logN, base):
    check_fwd_inv(1 << logN, 4, 3, 60, 300 + logN, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2, ot_log2_base=base)


# Columns of up to 64 points take the wide 64-column tile when N2 = N / N1 has 64 columns
# (exactly one tile per vector at (12, 6)), the 16-column tile otherwise (N2 = 16, 32 at
# (13, 9), (13, 8); longer columns at (13, 7) and up)
@pytest.mark.parametrize("logN,n1", [(12, 6), (13, -1), (13, 4), (13, 7), (13, 8), (13, 9), (14, 4), (14, 10),
                                     (15, 5), (16, 4), (16, 6), (16, 7), (16, 9), (16, 10), (17, 4), (17, 7),
                                     (17, 9), (17, 10)])
def test_pass_splits(logN, n1):
    check_fwd_inv(1 << logN, 2, 2, 60, 400 + logN, log2_n1=n1, kernel_path=ntt.PATH_SPLIT)
    check_fwd_inv(1 << logN, 2, 1, 60, 450 + logN, log2_n1=n1, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2,
                  kernel_path=ntt.PATH_SPLIT)


# ------------------------------------------------------------------ fused single-launch path

@pytest.mark.parametrize("logN", [13, 14, 15, 16, 17])
@pytest.mark.parametrize("ots", [0, 1, 2])
def test_fused_shapes(logN, ots):
    """Both passes in one persistent launch, per-XCD queues (default split of every fused N)."""
    kw = dict(kernel_path=ntt.PATH_FUSED)
    if ots:
        kw.update(twiddle_mode=ntt.TWIDDLE_OT, ot_stages=ots)
    # 11 limbs x 3 polys: uneven queues across the 8 XCDs (limbs 0-2 give XCDs two limbs)
    check_fwd_inv(1 << logN, 11, 3, 60, 900 + logN + 10 * ots, **kw)


@pytest.mark.parametrize("grid,lag", [(1, 4), (3, 1), (8, 2), (24, 100), (1024, 1)])
def test_fused_grids_and_lags(grid, lag, monkeypatch):
    """Tiny grids leave XCDs without workgroups (their queues are drained by the last
    workgroup out); any lag keeps the order; repeated launches reuse the reset counters."""
    monkeypatch.setenv("NTT_FUSED_GRID", str(grid))
    monkeypatch.setenv("NTT_FUSED_LAG", str(lag))
    N, L, P = 1 << 14, 9, 2
    primes, psis, data = make(N, L, P, 60, 950 + grid)
    plan = ntt.ntt_plan_create(N, primes, kernel_path=ntt.PATH_FUSED)
    try:
        assert ntt.ntt_plan_get_info(plan)["kernel_path"] == ntt.PATH_FUSED
        want = oracle.forward(data, primes, psis, THREADS)
        d = dev(data)
        for _ in range(3):
            ntt.ntt_forward(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want)
            ntt.ntt_inverse(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), data)
    finally:
        plan.destroy()


def test_fused_and_split_agree_across_streams():
    N, L, P = 1 << 16, 6, 2
    primes, psis, data = make(N, L, P, 60, 990)
    fused = ntt.ntt_plan_create(N, primes, kernel_path=ntt.PATH_FUSED)
    split = ntt.ntt_plan_create(N, primes, kernel_path=ntt.PATH_SPLIT)
    try:
        want = oracle.forward(data, primes, psis, THREADS)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        d1, d2, d3 = dev(data), dev(data), dev(data)
        torch.cuda.synchronize()
        ntt.ntt_forward(fused, d1, stream=s1)
        ntt.ntt_forward(fused, d2, stream=s2)     # same plan, other stream: ordered by the library
        ntt.ntt_forward(split, d3, stream=s2)
        torch.cuda.synchronize()
        for d in (d1, d2, d3):
            assert np.array_equal(host(d), want)
    finally:
        fused.destroy()
        split.destroy()


# ------------------------------------------------------------------ edge values

@pytest.mark.parametrize("bits", [31, 54, 59, 60, 61, 62])
def test_prime_widths(bits):
    # primes below 2^60 take the estimated-quotient arithmetic; 61- and 62-bit primes the exact one,
    # whose lazy ranges reach their limit (4q < 2^64) at 62 bits
    check_fwd_inv(1 << 16, 3, 2, bits, 500 + bits)
    check_fwd_inv(1 << 12, 3, 2, bits, 520 + bits, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2)


# 62-bit primes take the exact-quotient arithmetic, 60-bit ones the estimated quotient with its
# lazy ranges (float quotient in the forward final reduction, per-register inverse bounds)
@pytest.mark.parametrize("logN,bits,opts", [
    (12, 62, {}), (16, 62, {}), (12, 60, {}), (16, 60, {}), (16, 60, dict(log2_n1=6)),
    (16, 60, dict(log2_n1=6, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2)), (17, 60, dict(log2_n1=7))])
def test_extreme_inputs(logN, bits, opts):
    N = 1 << logN
    primes = synth.gen_primes(600, N, bits, 2)
    psis = oracle.roots(primes, N)
    plan = ntt.ntt_plan_create(N, primes, **opts)
    try:
        zeros = np.zeros((1, 2, N), dtype=np.uint64)
        assert not run_fwd(plan, zeros).any()
        top = np.empty((1, 2, N), dtype=np.uint64)
        for l, q in enumerate(primes):
            top[0, l] = q - 1
        assert np.array_equal(run_fwd(plan, top), oracle.forward(top, primes, psis))
        assert np.array_equal(run_inv(plan, top), oracle.inverse(top, primes, psis))
        e0 = zeros.copy()
        e0[0, :, 0] = 1
        assert np.array_equal(run_fwd(plan, e0), np.ones_like(e0))
        assert np.array_equal(run_inv(plan, np.ones_like(e0)), e0)
    finally:
        plan.destroy()


# ------------------------------------------------------------------ products

@pytest.mark.parametrize("logN", [3, 10, 12, 16])
def test_pointwise_and_polymul(logN):
    N = 1 << logN
    L = 3
    primes, psis, a = make(N, L, 2, 60, 700 + logN)
    b = synth.residue_batch(701 + logN, primes, N, 2)
    b[0, :, :4] = np.array(primes, dtype=np.uint64)[:, None] - np.uint64(1)   # q - 1 edge values
    plan = ntt.ntt_plan_create(N, primes)
    try:
        da, db, dc = dev(a), dev(b), dev(np.zeros_like(a))
        ntt.ntt_pointwise_mul(plan, da, db, dc)
        torch.cuda.synchronize()
        assert np.array_equal(host(dc), oracle.pointwise(a, b, primes))
        ntt.ntt_polymul_negacyclic(plan, da, db, dc)
        torch.cuda.synchronize()
        want = oracle.polymul(a, b, primes, psis, THREADS)
        assert np.array_equal(host(dc), want)
        assert np.array_equal(host(da), a) and np.array_equal(host(db), b)   # inputs untouched
        if N <= 1 << 10:
            for l, q in enumerate(primes):
                assert host(dc)[1, l].tolist() == oracle.schoolbook(a[1, l], b[1, l], q).tolist()
        ntt.ntt_polymul_negacyclic(plan, da, db, da)   # in place on a
        torch.cuda.synchronize()
        assert np.array_equal(host(da), want)
    finally:
        plan.destroy()


@pytest.mark.parametrize("logN,bits,opts", [
    (8, 62, {}),                                                     # single pass, exact quotients
    (13, 60, dict(twiddle_mode=2, ot_stages=2, log2_n1=-1)),         # single pass with OT
    (13, 61, dict(log2_n1=6)),
    (14, 60, dict(twiddle_mode=2, ot_stages=1)),
    (16, 62, dict(twiddle_mode=2, ot_stages=2, ot_log2_base=8)),
    (17, 60, dict(log2_n1=10)),
    (16, 60, dict(kernel_path=2)),                                   # fused-path plan: separate launches
])
def test_polymul_paths(logN, bits, opts):
    """The product's launch sequences: NTT(b) out of place, a's forward column pass out of
    place, then one launch for the row passes with the key product, then the inverse column
    pass (or a single launch at single-pass sizes)."""
    N, L, P = 1 << logN, 3, 2
    primes, psis, a = make(N, L, P, bits, 750 + logN)
    b = synth.residue_batch(751 + logN, primes, N, P)
    plan = ntt.ntt_plan_create(N, primes, **opts)
    try:
        da, db, dc = dev(a), dev(b), dev(np.zeros_like(a))
        ntt.ntt_polymul_negacyclic(plan, da, db, dc)
        torch.cuda.synchronize()
        want = oracle.polymul(a, b, primes, psis, THREADS)
        assert np.array_equal(host(dc), want), f"N=2^{logN} {opts}"
        assert np.array_equal(host(da), a) and np.array_equal(host(db), b)
        ntt.ntt_polymul_negacyclic(plan, da, db, da)   # in place on a
        torch.cuda.synchronize()
        assert np.array_equal(host(da), want)
    finally:
        plan.destroy()


# ------------------------------------------------------------------ benchmark workloads at full size

def test_config1_plain_small():
    """N=2^12, L=4 primes of 54 bits (seed 1): forward+inverse of one polynomial and the
    negacyclic product of two."""
    N, L = 1 << 12, 4
    primes, psis, data = make(N, L, 2, 54, 1)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        f = run_fwd(plan, data[:1])
        assert np.array_equal(f, oracle.forward(data[:1], primes, psis))
        assert np.array_equal(run_inv(plan, f), data[:1])
        da, db, dc = dev(data[:1]), dev(data[1:]), dev(np.zeros_like(data[:1]))
        ntt.ntt_polymul_negacyclic(plan, da, db, dc)
        torch.cuda.synchronize()
        got = host(dc)
        for l, q in enumerate(primes):
            assert got[0, l].tolist() == oracle.schoolbook(data[0, l], data[1, l], q).tolist()
    finally:
        plan.destroy()


@pytest.mark.parametrize("mode", ["table", "ot"])
def test_config2_full(mode):
    """N=2^16, L=45 primes in [2^59, 2^60) (seed 2), one ciphertext (2 polys): forward then inverse."""
    N, L, P = 1 << 16, 45, 2
    primes, psis, data = make(N, L, P, 60, 2)
    opts = {} if mode == "table" else dict(twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2)
    plan = ntt.ntt_plan_create(N, primes, **opts)
    try:
        d = dev(data)
        ntt.ntt_forward(plan, d)
        torch.cuda.synchronize()
        f = host(d)
        assert np.array_equal(f, oracle.forward(data, primes, psis, THREADS))
        rnd = random.Random(2)
        for _ in range(8):   # slots checked against the definition itself (Horner), not Algorithm 1
            p, l, i = rnd.randrange(P), rnd.randrange(L), rnd.randrange(N)
            assert int(f[p, l, i]) == oracle.forward_at(data[p, l], primes[l], psis[l], i)
        ntt.ntt_inverse(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), data)
    finally:
        plan.destroy()


def _bench_module():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_config2_bench_plans():
    """Every plan the headline measurement times, built as it builds them, on its own inputs
    (N=2^16, L=45, 2 polys): the four named variants at the default split and the tuner's cached
    plan for the shape.  Each is driven the three ways the measurement drives it (one call per
    step, one call per pass, one call per polynomial) and checked against one oracle forward."""
    b = _bench_module()
    W = b.WORKLOAD
    N, L, P = W["N"], W["L"], W["P"]
    primes = synth.gen_primes(W["seed"], N, W["bits"], L)
    data = synth.residue_batch(W["seed"], primes, N, P)
    psis = oracle.roots(primes, N)
    want = oracle.forward(data, primes, psis, THREADS)
    plans = {name: dict(opts, log2_n1=0) for name, opts in b.VARIANTS.items()}
    from paper_2012_01968_amd import autotune
    entry = autotune.lookup(N, primes, P)
    if entry is not None:        # present whenever the cache was refreshed for these kernel sources
        plans["tuned"] = entry["opts"]
    for name, opts in plans.items():
        plan = ntt.ntt_plan_create(N, primes, **opts)
        try:
            assert ntt.ntt_plan_get_roots(plan) == psis
            d = dev(data)
            ntt.ntt_forward(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want), f"{name}: forward"
            ntt.ntt_inverse(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), data), f"{name}: inverse(forward)"
            npass = ntt.ntt_plan_num_passes(plan)
            for p in range(npass):
                ntt.ntt_forward_pass(plan, d, p)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want), f"{name}: forward by passes"
            for p in range(npass):
                ntt.ntt_inverse_pass(plan, d, p)
            for i in range(P):
                ntt.ntt_forward(plan, d[i])
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want), f"{name}: forward per polynomial"
        finally:
            plan.destroy()


def test_config3_full_polymul():
    """N=2^17, L=60 (seed 3), 4 polys: forward x4, products p0*p2 and p1*p3, inverse x2, OT on."""
    N, L, P = 1 << 17, 60, 4
    primes, psis, data = make(N, L, P, 60, 3)
    plan = ntt.ntt_plan_create(N, primes, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2)
    try:
        d = dev(data)
        ntt.ntt_forward(plan, d)
        prod = torch.empty_like(d[:2])
        ntt.ntt_pointwise_mul(plan, d[:2], d[2:], prod)
        ntt.ntt_inverse(plan, prod)
        torch.cuda.synchronize()
        got = host(prod)
        f = host(d)
        rnd = random.Random(3)
        for _ in range(6):
            p, l, i = rnd.randrange(P), rnd.randrange(L), rnd.randrange(N)
            assert int(f[p, l, i]) == oracle.forward_at(data[p, l], primes[l], psis[l], i)
        want = oracle.polymul(data[:2], data[2:], primes, psis, THREADS)
        assert np.array_equal(got, want)
    finally:
        plan.destroy()


def test_plan_reuse_across_streams():
    N, L = 1 << 14, 4
    primes, psis, data = make(N, L, 2, 60, 800)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        want = oracle.forward(data, primes, psis)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        d1, d2 = dev(data), dev(data)
        torch.cuda.synchronize()
        ntt.ntt_forward(plan, d1, stream=s1)
        ntt.ntt_forward(plan, d2, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(host(d1), want) and np.array_equal(host(d2), want)
    finally:
        plan.destroy()


def test_round_robin_steps_on_two_streams():
    """The bench's schedule: independent forward + inverse steps over copies, step i on stream
    i mod 2 with no wait between steps; every copy ends as it started, and a forward run on one
    stream while the other keeps stepping matches the oracle."""
    N, L, P = 1 << 16, 6, 2
    primes, psis, data = make(N, L, P, 60, 810)
    plan = ntt.ntt_plan_create(N, primes, log2_n1=6, col_width=32)
    try:
        want = oracle.forward(data, primes, psis, THREADS)
        sts = [torch.cuda.Stream(), torch.cuda.Stream()]
        copies = [dev(data) for _ in range(6)]
        torch.cuda.synchronize()
        for i in range(24):
            st = sts[i % 2]
            ntt.ntt_forward(plan, copies[i % 6], stream=st)
            ntt.ntt_inverse(plan, copies[i % 6], stream=st)
        fwd = dev(data)
        torch.cuda.synchronize()
        for i in range(8):
            ntt.ntt_forward(plan, copies[2 * i % 6 + 1], stream=sts[1])
            ntt.ntt_inverse(plan, copies[2 * i % 6 + 1], stream=sts[1])
            if i == 3:
                ntt.ntt_forward(plan, fwd, stream=sts[0])
        torch.cuda.synchronize()
        for c in copies:
            assert np.array_equal(host(c), data)
        assert np.array_equal(host(fwd), want)
    finally:
        plan.destroy()


# ------------------------------------------------------------------ batches of uneven jobs

@pytest.mark.parametrize("mode", ["plain", "grouped", "graph", "branched"])
def test_batch_uneven_jobs(mode):
    """Jobs of several N and limb counts (prefixes of one prime chain), mixed ops, in one
    batch; every job is checked against the oracle and the three run modes agree."""
    n_max = 1 << 16
    chain = synth.gen_primes(1000, n_max, 60, 6)
    plans = {logN: ntt.ntt_plan_create(1 << logN, chain) for logN in (4, 10, 13, 16)}
    spec = [(4, 1, 2, ntt.OP_FORWARD), (10, 3, 1, ntt.OP_FORWARD_INVERSE), (13, 6, 2, ntt.OP_INVERSE),
            (16, 2, 1, ntt.OP_FORWARD), (16, 5, 2, ntt.OP_FORWARD_INVERSE), (10, 6, 3, ntt.OP_INVERSE),
            (13, 1, 1, ntt.OP_FORWARD), (4, 6, 1, ntt.OP_FORWARD_INVERSE)]
    try:
        jobs, bufs, want = [], [], []
        for k, (logN, limbs, polys, op) in enumerate(spec):
            N = 1 << logN
            primes = chain[:limbs]
            data = synth.residue_batch(1100 + k, primes, N, polys)
            psis = oracle.roots(primes, N)
            if op == ntt.OP_FORWARD:
                w = oracle.forward(data, primes, psis, THREADS)
            elif op == ntt.OP_INVERSE:
                w = oracle.inverse(data, primes, psis, THREADS)
            else:
                w = data.copy()
            d = dev(data)
            bufs.append(d)
            want.append(w)
            jobs.append((plans[logN], d, polys, limbs if limbs < len(chain) else 0, op))
        batch = ntt.ntt_batch_create(jobs)
        m = {"plain": ntt.BATCH_PLAIN, "grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH,
             "branched": ntt.BATCH_GRAPH_BRANCHED}[mode]
        ntt.ntt_batch_run(batch, m)
        torch.cuda.synchronize()
        for d, w in zip(bufs, want):
            assert np.array_equal(host(d), w)
        if mode in ("graph", "branched"):   # replays: forward-only jobs advance, round-trip jobs stay put
            for _ in range(3):
                ntt.ntt_batch_run(batch, m)
                torch.cuda.synchronize()
            for (logN, limbs, polys, op), d, w in zip(spec, bufs, want):
                if op == ntt.OP_FORWARD_INVERSE:
                    assert np.array_equal(host(d), w)
        batch.destroy()
    finally:
        for p in plans.values():
            p.destroy()


@pytest.mark.parametrize("mode", ["plain", "grouped", "graph", "branched"])
def test_batch_mulkey_jobs(mode):
    """Forward, product with a resident NTT-domain key, inverse, as one job: the result is
    the negacyclic product with the key polynomial, per limb (schoolbook-checked on a small
    case, oracle NTT product on the rest)."""
    n_max = 1 << 15
    chain = synth.gen_primes(1200, n_max, 60, 8)
    plans = {logN: ntt.ntt_plan_create(1 << logN, chain) for logN in (5, 12, 15)}
    spec = [(5, 3, 2), (12, 8, 1), (15, 5, 2), (12, 2, 3), (15, 8, 1)]
    try:
        jobs, bufs, want = [], [], []
        keys = {}
        for logN in plans:
            N = 1 << logN
            coeff = synth.residue_batch(1300 + logN, chain, N, 1)
            keys[logN] = (coeff, oracle.forward(coeff, chain, oracle.roots(chain, N), THREADS),)
        for k, (logN, limbs, polys) in enumerate(spec):
            N = 1 << logN
            primes = chain[:limbs]
            psis = oracle.roots(primes, N)
            data = synth.residue_batch(1400 + k, primes, N, polys)
            coeff, key_ntt = keys[logN]
            key_coeff = coeff.reshape(len(chain), N)[:limbs]
            w = oracle.polymul(data.reshape(polys * limbs, N), np.tile(key_coeff, (polys, 1)), primes, psis,
                               THREADS).reshape(data.shape)
            if logN == 5:   # pin the small case to the schoolbook product as well
                a = data.reshape(polys, limbs, N)
                for p in range(polys):
                    for l in range(limbs):
                        sb = oracle.schoolbook(a[p, l], key_coeff[l], primes[l])
                        assert np.array_equal(w.reshape(polys, limbs, N)[p, l], sb)
            d = dev(data)
            dk = dev(key_ntt.reshape(len(chain), N)[:limbs])
            bufs.append((d, dk))
            want.append(w)
            jobs.append((plans[logN], d, polys, limbs if limbs < len(chain) else 0,
                         ntt.OP_FORWARD | ntt.OP_MULKEY | ntt.OP_INVERSE, dk))
        batch = ntt.ntt_batch_create(jobs)
        m = {"plain": ntt.BATCH_PLAIN, "grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH,
             "branched": ntt.BATCH_GRAPH_BRANCHED}[mode]
        ntt.ntt_batch_run(batch, m)
        torch.cuda.synchronize()
        for (d, _), w in zip(bufs, want):
            assert np.array_equal(host(d), w)
        batch.destroy()
    finally:
        for p in plans.values():
            p.destroy()


def test_batch_assign_reuse():
    """One batch object, reassigned on a stream to job sets of growing and shrinking size;
    each run matches the oracle, and a graph captured before a reassign is not reused."""
    chain = synth.gen_primes(1500, 1 << 13, 60, 4)
    plans = {logN: ntt.ntt_plan_create(1 << logN, chain) for logN in (11, 13)}
    st = torch.cuda.Stream()
    rounds = [[(11, 2, 1)], [(13, 4, 3), (11, 4, 2), (11, 1, 5)], [(13, 1, 1)], [(11, 3, 40), (13, 4, 9)]]
    batch = None
    try:
        for r, spec in enumerate(rounds):
            jobs, bufs, want = [], [], []
            for k, (logN, limbs, polys) in enumerate(spec):
                N = 1 << logN
                primes = chain[:limbs]
                data = synth.residue_batch(1600 + 10 * r + k, primes, N, polys)
                want.append(oracle.forward(data, primes, oracle.roots(primes, N), THREADS))
                d = dev(data)
                bufs.append(d)
                jobs.append((plans[logN], d, polys, limbs if limbs < len(chain) else 0, ntt.OP_FORWARD))
            torch.cuda.synchronize()
            if batch is None:
                batch = ntt.ntt_batch_create(jobs)
            else:
                ntt.ntt_batch_assign(batch, jobs, st)
            ntt.ntt_batch_run(batch, ntt.BATCH_GRAPH if r % 2 else ntt.BATCH_GROUPED, st)
            st.synchronize()
            for d, w in zip(bufs, want):
                assert np.array_equal(host(d), w), f"round {r}"
    finally:
        if batch is not None:
            batch.destroy()
        for p in plans.values():
            p.destroy()


def test_config3_polymul_entry_point():
    """N=2^17, L=60 (seed 3), OT on: the negacyclic product of two 2-polynomial operands through
    ntt_polymul_negacyclic, against the oracle."""
    N, L = 1 << 17, 60
    primes, psis, data = make(N, L, 4, 60, 3)
    plan = ntt.ntt_plan_create(N, primes, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2)
    try:
        da, db = dev(data[:2]), dev(data[2:])
        dc = torch.empty_like(da)
        ntt.ntt_polymul_negacyclic(plan, da, db, dc)
        torch.cuda.synchronize()
        assert np.array_equal(host(dc), oracle.polymul(data[:2], data[2:], primes, psis, THREADS))
    finally:
        plan.destroy()


@pytest.mark.parametrize("mode", ["plain", "grouped", "graph", "branched"])
def test_batch_mulkey_ot_and_wide_plans(mode):
    """Forward, key product, inverse jobs on OT plans (single pass and split) and on a plan of
    61-bit primes (exact quotients), with limb prefixes; every result against the oracle."""
    specs = [  # (logN, bits, plan options, [(limbs, polys), ...])
        (12, 60, dict(twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2), [(3, 2), (1, 1)]),
        (14, 60, dict(twiddle_mode=ntt.TWIDDLE_OT, ot_stages=1, ot_log2_base=8), [(4, 1), (2, 3)]),
        (13, 61, dict(log2_n1=6), [(4, 2)]),
    ]
    plans, jobs, bufs, want = [], [], [], []
    try:
        for si, (logN, bits, opts, shapes) in enumerate(specs):
            N = 1 << logN
            chain = synth.gen_primes(1700 + si, N, bits, 4)
            plan = ntt.ntt_plan_create(N, chain, **opts)
            plans.append(plan)
            key_coeff = synth.residue_batch(1710 + si, chain, N, 1).reshape(4, N)
            key_ntt = oracle.forward(key_coeff, chain, oracle.roots(chain, N), THREADS)
            dk = dev(key_ntt)
            for k, (limbs, polys) in enumerate(shapes):
                primes = chain[:limbs]
                data = synth.residue_batch(1720 + 10 * si + k, primes, N, polys)
                w = oracle.polymul(data.reshape(polys * limbs, N), np.tile(key_coeff[:limbs], (polys, 1)), primes,
                                   oracle.roots(primes, N), THREADS).reshape(data.shape)
                d = dev(data)
                bufs.append((d, dk))
                want.append(w)
                jobs.append((plan, d, polys, limbs if limbs < 4 else 0,
                             ntt.OP_FORWARD | ntt.OP_MULKEY | ntt.OP_INVERSE, dk))
        batch = ntt.ntt_batch_create(jobs)
        m = {"plain": ntt.BATCH_PLAIN, "grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH,
             "branched": ntt.BATCH_GRAPH_BRANCHED}[mode]
        ntt.ntt_batch_run(batch, m)
        torch.cuda.synchronize()
        for (d, _), w in zip(bufs, want):
            assert np.array_equal(host(d), w)
        batch.destroy()
    finally:
        for p in plans:
            p.destroy()


@pytest.mark.parametrize("mode", ["grouped", "graph", "branched"])
def test_config4_full_uneven_batch(mode):
    """The full uneven workload (256 polys, N from 2^13 to 2^17, L uniform in [4, 60], seed 4)
    with the plans the benchmark builds for it (the tuner's cached choice per size, else the
    default): forward NTT of every polynomial in one batch against the oracle, then forward +
    inverse jobs returning every polynomial unchanged."""
    b = _bench_module()
    cfg = b.UNEVEN
    chain, logNs, Ls = b.uneven_jobs(cfg)
    Lmax = cfg["L"][1]
    from paper_2012_01968_amd import autotune
    plans, src, want = {}, {}, {}
    try:
        for k in cfg["logNs"]:
            k = int(k)
            polys_k = max(1, -(-int(Ls[logNs == k].sum()) // Lmax))
            entry = autotune.lookup(1 << k, chain, polys_k)
            plans[k] = ntt.ntt_plan_create(1 << k, chain, **(entry["opts"] if entry else {}))
            s = synth.residue_batch(cfg["seed"] + k, chain, 1 << k, 1).reshape(Lmax, 1 << k)
            src[k] = s
            want[k] = oracle.forward(s, chain, oracle.roots(chain, 1 << k), THREADS)
        m = {"grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH, "branched": ntt.BATCH_GRAPH_BRANCHED}[mode]
        for op in (ntt.OP_FORWARD, ntt.OP_FORWARD_INVERSE):
            bufs, jobs = [], []
            for k, L in zip(logNs.tolist(), Ls.tolist()):
                d = dev(src[k][:L])
                bufs.append(d)
                jobs.append((plans[k], d, 1, L if L < Lmax else 0, op))
            batch = ntt.ntt_batch_create(jobs)
            ntt.ntt_batch_run(batch, m)
            torch.cuda.synchronize()
            for i, (d, k, L) in enumerate(zip(bufs, logNs.tolist(), Ls.tolist())):
                expect = want[k][:L] if op == ntt.OP_FORWARD else src[k][:L]
                assert np.array_equal(host(d), expect), f"poly {i}: N=2^{k} L={L} op={op}"
            batch.destroy()
            del bufs
    finally:
        for p in plans.values():
            p.destroy()
