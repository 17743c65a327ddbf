"""The natural-order option (Section III-C): plans created with ORDER_NATURAL return A_k in
slot k.  Compared element by element with the oracle: the forward output with the oracle's
bit-reversed output put in natural order (and, at small N, with the natural-order definition
itself), the inverse of natural-order input, the passes one by one, products, and batches
(including key products with natural-order keys)."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import ntt_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")

THREADS = min(16, os.cpu_count() or 1)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint64)


CASES = [  # (logN, plan options)
    (1, {}), (2, {}), (3, {}), (5, {}), (8, {}), (9, {}), (10, {}), (11, {}), (12, {}),
    (13, dict(log2_n1=-1)), (13, {}), (14, dict(twiddle_mode=2, ot_stages=1)), (15, {}),
    (16, {}), (16, dict(log2_n1=6, twiddle_mode=2, ot_stages=2)), (16, dict(kernel_path=2)), (17, {}),
    (17, dict(log2_n1=6)),
]


@pytest.mark.parametrize("logN,opts", CASES)
def test_natural_forward_inverse(logN, opts):
    N, L, P = 1 << logN, 3, 2
    primes = synth.gen_primes(5000 + logN, N, 60, L)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(5000 + logN, primes, N, P)
    plan = ntt.ntt_plan_create(N, primes, order=ntt.ORDER_NATURAL, **opts)
    try:
        assert ntt.ntt_plan_order(plan) == ntt.ORDER_NATURAL
        want = oracle.natural_order(oracle.forward(data, primes, psis, THREADS))
        if N <= 64:
            for l, q in enumerate(primes):
                assert want[0, l].tolist() == O.forward_natural_definition(data[0, l].tolist(), q, psis[l])
        d = dev(data)
        ntt.ntt_forward(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), want), "forward"
        ntt.ntt_inverse(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), data), "inverse(forward)"
        # inverse of arbitrary natural-order input: the oracle's inverse of the same values
        # put back in bit-reversed order (the permutation is its own inverse)
        d = dev(data)
        ntt.ntt_inverse(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), oracle.inverse(oracle.natural_order(data), primes, psis, THREADS)), "inverse"
        # pass by pass
        npass = ntt.ntt_plan_num_passes(plan)
        d = dev(data)
        for p in range(npass):
            ntt.ntt_forward_pass(plan, d, p)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), want), "forward by passes"
        for p in range(npass):
            ntt.ntt_inverse_pass(plan, d, p)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), data), "inverse by passes"
        # the product does not depend on the order
        b = synth.residue_batch(5100 + logN, primes, N, P)
        c = torch.empty_like(d)
        ntt.ntt_polymul_negacyclic(plan, dev(data), dev(b), c)
        torch.cuda.synchronize()
        assert np.array_equal(host(c), oracle.polymul(data, b, primes, psis, THREADS)), "product"
    finally:
        plan.destroy()


@pytest.mark.parametrize("mode", ["plain", "grouped", "graph"])
def test_natural_batches(mode):
    """Forward, inverse and forward + key + inverse jobs on natural-order plans (keys in
    natural order), mixed with a bit-reversed plan, in one batch."""
    chain = synth.gen_primes(5200, 1 << 14, 60, 4)
    nat = {k: ntt.ntt_plan_create(1 << k, chain, order=ntt.ORDER_NATURAL) for k in (9, 14)}
    brv = ntt.ntt_plan_create(1 << 14, chain)
    m = {"plain": ntt.BATCH_PLAIN, "grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH}[mode]
    try:
        jobs, bufs, want = [], [], []
        for i, (k, limbs, op, plan) in enumerate([(9, 2, ntt.OP_FORWARD, nat[9]), (14, 4, ntt.OP_INVERSE, nat[14]),
                                                  (14, 3, ntt.OP_FORWARD | ntt.OP_MULKEY | ntt.OP_INVERSE, nat[14]),
                                                  (14, 2, ntt.OP_FORWARD | ntt.OP_MULKEY | ntt.OP_INVERSE, brv),
                                                  (9, 4, ntt.OP_FORWARD_INVERSE, nat[9])]):
            N = 1 << k
            primes = chain[:limbs]
            psis = oracle.roots(primes, N)
            data = synth.residue_batch(5210 + i, primes, N, 2)
            key = None
            if op == ntt.OP_FORWARD:
                w = oracle.natural_order(oracle.forward(data, primes, psis, THREADS))
            elif op == ntt.OP_INVERSE:
                w = oracle.inverse(oracle.natural_order(data), primes, psis, THREADS)
            elif op == ntt.OP_FORWARD_INVERSE:
                w = data.copy()
            else:
                kc = synth.residue_batch(5230 + i, primes, N, 1).reshape(limbs, N)
                kf = oracle.forward(kc, primes, psis, THREADS)
                key = dev(oracle.natural_order(kf) if plan is not brv else kf)
                w = oracle.polymul(data.reshape(2 * limbs, N), np.tile(kc, (2, 1)), primes, psis,
                                   THREADS).reshape(data.shape)
            d = dev(data)
            bufs.append(d)
            want.append(w)
            job = (plan, d, 2, limbs if limbs < 4 else 0, op)
            jobs.append(job + ((key,) if key is not None else ()))
        batch = ntt.ntt_batch_create(jobs)
        ntt.ntt_batch_run(batch, m)
        torch.cuda.synchronize()
        for i, (d, w) in enumerate(zip(bufs, want)):
            assert np.array_equal(host(d), w), f"job {i}"
        batch.destroy()
    finally:
        for p in list(nat.values()) + [brv]:
            p.destroy()
