"""The product entry point that allocates nothing, against the allocating one.

ntt_polymul_negacyclic_noalloc keeps NTT(b) in the library's fixed device array instead of a
plan-owned buffer; it must give exactly the same residues as ntt_polymul_negacyclic (and as the
oracle's negacyclic product, Section III-A) on two calls in a row, the second with a smaller
batch, and refuse a batch larger than its array.  Tolerance 0: the arithmetic is exact.
"""
import os

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


@pytest.mark.parametrize("logN,L,opts", [
    (16, 6, dict(log2_n1=6)),                                            # split, 2^10-point rows
    (17, 4, dict(log2_n1=6, twiddle_mode=2, ot_stages=1)),               # 2^11-point rows, OT
    (12, 3, dict()),                                                     # one pass
    (14, 3, dict(kernel_path=2, log2_n1=7)),                             # fused launch
])
def test_noalloc_matches_the_allocating_product(logN, L, opts):
    N = 1 << logN
    seed = 7100 + logN
    primes = synth.gen_primes(seed, N, 60, L)
    psis = oracle.roots(primes, N)
    plan = ntt.ntt_plan_create(N, primes, **opts)
    try:
        for polys in (3, 1):            # the second call on a smaller batch
            a = synth.residue_batch(seed + polys, primes, N, polys)
            b = synth.residue_batch(seed + 10 + polys, primes, N, polys)
            da, db = dev(a), dev(b)
            c_ref, c_new = torch.empty_like(da), torch.full_like(da, -1)
            ntt.ntt_polymul_negacyclic(plan, da, db, c_ref)
            ntt.ntt_polymul_negacyclic_noalloc(plan, da, db, c_new)
            torch.cuda.synchronize()
            got = host(c_new)
            assert np.array_equal(got, host(c_ref)), f"N=2^{logN} P={polys} {opts}: differs from the allocating call"
            if polys == 1 or logN <= 14:
                assert np.array_equal(got, oracle.polymul(a, b, primes, psis, THREADS)), "differs from the oracle"
            assert np.array_equal(host(da), a) and np.array_equal(host(db), b), "operands changed"
    finally:
        plan.destroy()


def test_noalloc_in_place_and_limit():
    N, L = 1 << 13, 2
    primes = synth.gen_primes(7200, N, 60, L)
    psis = oracle.roots(primes, N)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        a = synth.residue_batch(7201, primes, N, 2)
        b = synth.residue_batch(7202, primes, N, 2)
        da, db = dev(a), dev(b)
        ntt.ntt_polymul_negacyclic_noalloc(plan, da, db, da)       # c aliases a
        torch.cuda.synchronize()
        assert np.array_equal(host(da), oracle.polymul(a, b, primes, psis, THREADS))
        limit = ntt.ntt_polymul_noalloc_max_words()
        assert limit == 1 << 23
        polys = limit // (L * N) + 1                                # one polynomial too many
        big = torch.zeros((polys, L, N), dtype=torch.int64, device="cuda")
        with pytest.raises(ntt.NttError, match="no-allocation limit"):
            ntt.ntt_polymul_negacyclic_noalloc(plan, big, big.clone(), big)
    finally:
        plan.destroy()
