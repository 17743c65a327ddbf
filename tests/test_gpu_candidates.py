"""Every plan the tuner can choose, against the CPU oracle.

For each transform size N = 2^1 .. 2^17 and two prime widths (60-bit primes take the
estimated-quotient arithmetic, 62-bit primes the exact one), every option set that
``autotune.candidates(N)`` enumerates is built and its forward transform (Algorithm 1),
its inverse and its negacyclic product (Section III-A) are compared element by element
with the oracle on the same seeded inputs.  This covers every split N1 x N2 (including the
2^11-point rows of N1 = 2^6 at N = 2^17), the key-product row kernel at every row length,
every OT depth and digit base, and the fused launch where its shape exists.  Tolerance 0:
the arithmetic is exact.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")
from paper_2012_01968_amd import autotune  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)
L, P = 3, 2


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("bits", [60, 62])
@pytest.mark.parametrize("logN", list(range(1, 18)))
def test_every_candidate_plan(logN, bits):
    N = 1 << logN
    seed = 3000 + 100 * bits + logN
    primes = synth.gen_primes(seed, N, bits, L)
    psis = oracle.roots(primes, N)
    a = synth.residue_batch(seed, primes, N, P)
    b = synth.residue_batch(seed + 1, primes, N, P)
    # extreme operands in the first vector of b: q - 1 everywhere
    b[0, 0, :] = np.uint64(primes[0] - 1)
    want_f = oracle.forward(a, primes, psis, THREADS)
    want_i = oracle.inverse(a, primes, psis, THREADS)
    want_m = oracle.polymul(a, b, primes, psis, THREADS)
    da, db = dev(a), dev(b)
    checked, refused = [], []
    for opts in autotune.candidates(N):
        try:
            plan = ntt.ntt_plan_create(N, primes, **opts)
        except ntt.NttError as e:
            # the fused launch exists only for primes below 2^60; nothing else may be refused
            assert bits > 60 and opts.get("kernel_path") == ntt.PATH_FUSED, f"{opts}: {e}"
            refused.append(opts)
            continue
        try:
            assert ntt.ntt_plan_get_roots(plan) == psis
            d = da.clone()
            ntt.ntt_forward(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want_f), f"N=2^{logN} q<2^{bits} {opts}: forward"
            ntt.ntt_inverse(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), a), f"N=2^{logN} q<2^{bits} {opts}: inverse(forward)"
            d = da.clone()
            ntt.ntt_inverse(plan, d)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), want_i), f"N=2^{logN} q<2^{bits} {opts}: inverse"
            c = torch.empty_like(da)
            ntt.ntt_polymul_negacyclic(plan, da, db, c)
            torch.cuda.synchronize()
            assert np.array_equal(host(c), want_m), f"N=2^{logN} q<2^{bits} {opts}: product"
            assert np.array_equal(host(da), a) and np.array_equal(host(db), b), "operands changed"
            checked.append(opts)
        finally:
            plan.destroy()
    assert checked, "no candidate plan was built"
    # at 60 bits the sweep must reach every candidate
    if bits == 60:
        assert not refused


@pytest.mark.parametrize("logN", list(range(1, 18)))
def test_every_tile_shape(logN):
    """Every tile shape the tuner's second round can choose (values per lane and workgroup
    lanes of the row pass, column tile width), on every split of N and with table, one-stage
    and two-stage OT twiddles (60-bit primes): forward, inverse and negacyclic product against
    the oracle.  Together these reach every row, key-product and column kernel instance that
    a tile option selects."""
    N = 1 << logN
    seed = 5000 + logN
    primes = synth.gen_primes(seed, N, 60, L)
    psis = oracle.roots(primes, N)
    a = synth.residue_batch(seed, primes, N, P)
    b = synth.residue_batch(seed + 1, primes, N, P)
    b[1, 2, :] = np.uint64(primes[2] - 1)
    want_f = oracle.forward(a, primes, psis, THREADS)
    want_i = oracle.inverse(a, primes, psis, THREADS)
    want_m = oracle.polymul(a, b, primes, psis, THREADS)
    da, db = dev(a), dev(b)
    checked = 0
    bases = [c for c in autotune.candidates(N) if c["kernel_path"] == ntt.PATH_SPLIT and
             (c["twiddle_mode"] == ntt.TWIDDLE_TABLE or c.get("ot_log2_base") == min(10, logN - 1))]
    for base in bases:
        for opts in autotune.tile_candidates(N, base)[1:]:
            plan = ntt.ntt_plan_create(N, primes, **opts)
            try:
                info = ntt.ntt_plan_get_info(plan)
                assert (info["r1"], info["wg_size"], info["col_width"]) == \
                    (opts.get("r1", 0), opts.get("wg_size", 0), opts.get("col_width", 0))
                d = da.clone()
                ntt.ntt_forward(plan, d)
                torch.cuda.synchronize()
                assert np.array_equal(host(d), want_f), f"N=2^{logN} {opts}: forward"
                ntt.ntt_inverse(plan, d)
                torch.cuda.synchronize()
                assert np.array_equal(host(d), a), f"N=2^{logN} {opts}: inverse(forward)"
                d = da.clone()
                ntt.ntt_inverse(plan, d)
                torch.cuda.synchronize()
                assert np.array_equal(host(d), want_i), f"N=2^{logN} {opts}: inverse"
                c = torch.empty_like(da)
                ntt.ntt_polymul_negacyclic(plan, da, db, c)
                torch.cuda.synchronize()
                assert np.array_equal(host(c), want_m), f"N=2^{logN} {opts}: product"
                checked += 1
            finally:
                plan.destroy()
    assert checked > 0


@pytest.mark.parametrize("mode", ["poison", "reverse", "poison,reverse"])
def test_debug_modes_change_nothing(mode, monkeypatch):
    """With the split passes' LDS poisoned before use and with their workgroups taking tiles
    in reverse order, every split and tile shape at N = 2^10, 2^13 and 2^16 still matches the
    oracle: no exchange reads a slot it did not write and no tile depends on another."""
    monkeypatch.setenv("NTT_DEBUG", mode)
    for logN in (10, 13, 16):
        N = 1 << logN
        seed = 6000 + logN
        primes = synth.gen_primes(seed, N, 60, L)
        psis = oracle.roots(primes, N)
        a = synth.residue_batch(seed, primes, N, P)
        b = synth.residue_batch(seed + 1, primes, N, P)
        want_f = oracle.forward(a, primes, psis, THREADS)
        want_m = oracle.polymul(a, b, primes, psis, THREADS)
        da, db = dev(a), dev(b)
        for base in autotune.candidates(N):
            if base["kernel_path"] != ntt.PATH_SPLIT or base.get("ot_log2_base", 10) != 10:
                continue
            for opts in autotune.tile_candidates(N, base):
                plan = ntt.ntt_plan_create(N, primes, **opts)
                try:
                    d = da.clone()
                    ntt.ntt_forward(plan, d)
                    torch.cuda.synchronize()
                    assert np.array_equal(host(d), want_f), f"{mode} N=2^{logN} {opts}: forward"
                    ntt.ntt_inverse(plan, d)
                    torch.cuda.synchronize()
                    assert np.array_equal(host(d), a), f"{mode} N=2^{logN} {opts}: inverse(forward)"
                    c = torch.empty_like(da)
                    ntt.ntt_polymul_negacyclic(plan, da, db, c)
                    torch.cuda.synchronize()
                    assert np.array_equal(host(c), want_m), f"{mode} N=2^{logN} {opts}: product"
                finally:
                    plan.destroy()


@pytest.mark.parametrize("mode", ["", "poison", "reverse"])
def test_key_product_rows_of_128_points(mode, monkeypatch):
    """Products whose row passes are 128 points at 4 values per lane (32 lanes, two rows per
    wave) with one OT stage, for every N1 from 2^6 to 2^10 and every row workgroup size, plus
    the 8-value and two-stage neighbours, in each debug mode.  This is the shape that an
    earlier form of the conditional subtraction computed wrongly at N1 >= 2^8."""
    monkeypatch.setenv("NTT_DEBUG", mode)
    for logN in (13, 14, 15, 16, 17):
        N, n1 = 1 << logN, logN - 7
        primes = synth.gen_primes(5000 + logN, N, 60, L)
        psis = oracle.roots(primes, N)
        a = synth.residue_batch(5000 + logN, primes, N, P)
        b = synth.residue_batch(5001 + logN, primes, N, P)
        want = oracle.polymul(a, b, primes, psis, THREADS)
        for r1, wg, ots in ((4, 128, 1), (4, 64, 1), (4, 256, 1), (8, 128, 1), (4, 128, 2)):
            plan = ntt.ntt_plan_create(N, primes, log2_n1=n1, kernel_path=ntt.PATH_SPLIT, r1=r1, wg_size=wg,
                                       twiddle_mode=ntt.TWIDDLE_OT, ot_stages=ots, ot_log2_base=10)
            try:
                c = torch.empty_like(dev(a))
                ntt.ntt_polymul_negacyclic(plan, dev(a), dev(b), c)
                torch.cuda.synchronize()
                assert np.array_equal(host(c), want), f"N=2^{logN} n1={n1} r1={r1} wg={wg} ots={ots} {mode}"
            finally:
                plan.destroy()
