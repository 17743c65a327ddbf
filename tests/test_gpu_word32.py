"""The 32-bit word path (primes below 2^30) against the CPU oracle, element by element:
forward, inverse, element-wise and negacyclic products at every size and every column/row
split it has, extreme operands, and refusal of 64-bit calls on 32-bit plans."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")

THREADS = min(16, os.cpu_count() or 1)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int32)).to("cuda")


def host32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint64)


def check(N, L, P, seed, **opts):
    primes = synth.gen_primes(seed, N, 30, L)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(seed, primes, N, P)
    data[0, 0, :3] = np.uint64(primes[0] - 1)          # extreme operands
    plan = ntt.ntt_plan_create(N, primes, word_bits=32, **opts)
    try:
        assert ntt.ntt_plan_word_bits(plan) == 32
        assert ntt.ntt_plan_get_roots(plan) == psis
        want = oracle.forward(data, primes, psis, THREADS)
        d = dev32(data)
        ntt.ntt_forward_u32(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host32(d), want), f"forward N={N} {opts}"
        ntt.ntt_inverse_u32(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host32(d), data), f"inverse(forward) N={N} {opts}"
        d = dev32(data)
        ntt.ntt_inverse_u32(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host32(d), oracle.inverse(data, primes, psis, THREADS)), f"inverse N={N} {opts}"
        b = synth.residue_batch(seed + 1, primes, N, P)
        c = torch.empty_like(d)
        ntt.ntt_pointwise_mul_u32(plan, dev32(data), dev32(b), c)
        torch.cuda.synchronize()
        assert np.array_equal(host32(c), oracle.pointwise(data, b, primes)), "pointwise"
        ntt.ntt_polymul_negacyclic_u32(plan, dev32(data), dev32(b), c)
        torch.cuda.synchronize()
        assert np.array_equal(host32(c), oracle.polymul(data, b, primes, psis, THREADS)), "product"
    finally:
        plan.destroy()


@pytest.mark.parametrize("logN", list(range(1, 18)))
def test_word32_every_size(logN):
    check(1 << logN, 3, 2, 8000 + logN)


@pytest.mark.parametrize("logN,n1", [(10, 5), (12, 6), (13, 5), (13, 8), (15, 10), (16, 6), (16, 10), (17, 5),
                                     (17, 7), (17, 10), (12, -1)])
def test_word32_splits(logN, n1):
    check(1 << logN, 2, 3, 8100 + logN + n1, log2_n1=n1)


def test_word32_plan_rules():
    N = 1 << 12
    q30 = synth.gen_primes(8200, N, 30, 2)
    q31 = synth.gen_primes(8201, N, 31, 1)
    with pytest.raises(ntt.NttError, match="NTT_ERR_PRIME"):
        ntt.ntt_plan_create(N, q31, word_bits=32)
    with pytest.raises(ntt.NttError, match="NTT_ERR_UNSUPPORTED"):
        ntt.ntt_plan_create(N, q30, word_bits=32, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=1)
    plan = ntt.ntt_plan_create(N, q30, word_bits=32)
    try:
        x64 = torch.zeros((1, 2, N), dtype=torch.int64, device="cuda")
        with pytest.raises(ntt.NttError, match="32-bit words"):
            ntt.ntt_forward(plan, x64)
        with pytest.raises(ntt.NttError):
            ntt.ntt_batch_create([(plan, x64, 1, 0, ntt.OP_FORWARD)])
    finally:
        plan.destroy()
    plan64 = ntt.ntt_plan_create(N, q30)
    try:
        with pytest.raises(ntt.NttError, match="64-bit words"):
            ntt.ntt_forward_u32(plan64, torch.zeros((1, 2, N), dtype=torch.int32, device="cuda"))
    finally:
        plan64.destroy()
