"""RNS <-> integer conversion (Section III-B) against the CPU oracle (Python big integers),
element by element: decomposition of integers below Q and of wider words, reconstruction of
random residues, round trips, extreme values, and prime chains of 1 to 128 primes."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("L,bits,logN", [(1, 60, 4), (2, 61, 10), (3, 40, 11), (45, 60, 10), (60, 60, 8),
                                         (7, 62, 12), (64, 60, 6)])
def test_decompose_and_reconstruct(L, bits, logN):
    N, P = 1 << logN, 2
    primes = synth.gen_primes(9000 + L + bits, N, bits, L)
    Q = 1
    for q in primes:
        Q *= q
    plan = ntt.ntt_plan_create(N, primes)
    try:
        W = ntt.ntt_crt_words(plan)
        assert W == oracle.crt_words(primes)
        words = np.stack([synth.uniform_wide(9100 + L, p, Q, N) for p in range(P)])
        words[0, :, 0] = synth.ints_to_words([Q - 1], W)[:, 0]      # the largest value
        words[0, :, 1] = 0
        res = torch.empty((P, L, N), dtype=torch.int64, device="cuda")
        ntt.ntt_rns_decompose(plan, dev(words), W, res)
        torch.cuda.synchronize()
        want_res = oracle.rns_decompose_words(words, primes)
        assert np.array_equal(host(res), want_res), "decompose"
        out = torch.empty((P, W, N), dtype=torch.int64, device="cuda")
        ntt.ntt_crt_reconstruct(plan, res, out)
        torch.cuda.synchronize()
        assert np.array_equal(host(out), words), "reconstruct(decompose(x)) = x"
        # reconstruction of arbitrary residues (every residue q - 1 in one coefficient)
        r = synth.residue_batch(9200 + L, primes, N, P)
        r[1, :, 5] = np.array(primes, dtype=np.uint64) - np.uint64(1)
        ntt.ntt_crt_reconstruct(plan, dev(r), out)
        torch.cuda.synchronize()
        assert np.array_equal(host(out), oracle.crt_reconstruct_words(r, primes)), "reconstruct"
    finally:
        plan.destroy()


def test_decompose_wide_words():
    """Integers wider than Q (up to 2^(64*8)) reduce like any other."""
    N, L = 1 << 9, 5
    primes = synth.gen_primes(9300, N, 60, L)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        Wx = 8
        words = np.stack([synth.uniform_wide(9301, p, 1 << (64 * Wx), N) for p in range(2)])
        words[1, :, 3] = np.uint64(0xFFFFFFFFFFFFFFFF)
        res = torch.empty((2, L, N), dtype=torch.int64, device="cuda")
        ntt.ntt_rns_decompose(plan, dev(words), Wx, res)
        torch.cuda.synchronize()
        assert np.array_equal(host(res), oracle.rns_decompose_words(words, primes))
    finally:
        plan.destroy()


def test_conversions_with_the_transform():
    """Integers -> residues -> forward NTT -> product with a key -> inverse -> integers equals
    the negacyclic product of the integer polynomials modulo Q (the path between the two
    conversions), checked through the oracle."""
    N, L = 1 << 10, 6
    primes = synth.gen_primes(9400, N, 60, L)
    Q = 1
    for q in primes:
        Q *= q
    plan = ntt.ntt_plan_create(N, primes)
    try:
        W = ntt.ntt_crt_words(plan)
        a = synth.uniform_wide(9401, 0, Q, N)[None]
        b = synth.uniform_wide(9402, 0, Q, N)[None]
        ra = torch.empty((1, L, N), dtype=torch.int64, device="cuda")
        rb = torch.empty_like(ra)
        ntt.ntt_rns_decompose(plan, dev(a), W, ra)
        ntt.ntt_rns_decompose(plan, dev(b), W, rb)
        rc = torch.empty_like(ra)
        ntt.ntt_polymul_negacyclic(plan, ra, rb, rc)
        out = torch.empty((1, W, N), dtype=torch.int64, device="cuda")
        ntt.ntt_crt_reconstruct(plan, rc, out)
        torch.cuda.synchronize()
        psis = oracle.roots(primes, N)
        want_res = oracle.polymul(oracle.rns_decompose_words(a, primes), oracle.rns_decompose_words(b, primes),
                                  primes, psis)
        assert np.array_equal(host(out), oracle.crt_reconstruct_words(want_res, primes))
    finally:
        plan.destroy()


def test_reconstruct_refuses_more_than_64_primes():
    N = 1 << 6
    primes = synth.gen_primes(9500, N, 60, 65)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        x = torch.zeros((1, 65, N), dtype=torch.int64, device="cuda")
        out = torch.zeros((1, ntt.ntt_crt_words(plan), N), dtype=torch.int64, device="cuda")
        with pytest.raises(ntt.NttError, match="NTT_ERR_UNSUPPORTED"):
            ntt.ntt_crt_reconstruct(plan, x, out)
    finally:
        plan.destroy()
