"""The ablation-ladder paths (Section VI-A, VI-B; Table II) against the CPU oracle: the
radix-2 path (one launch per stage) and the register-only path at radix 2^2 .. 2^5 (one
launch per group of stages, a shorter last group where log2 N is not a multiple), forward,
inverse, pass by pass, products and batches, for both arithmetic policies.  Exact: tolerance 0."""
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


PATHS = [dict(kernel_path=3)] + [dict(kernel_path=4, log2_radix=k) for k in (2, 3, 4, 5)]


@pytest.mark.parametrize("bits", [60, 62])
@pytest.mark.parametrize("logN", [1, 2, 3, 4, 5, 7, 10, 13, 16, 17])
@pytest.mark.parametrize("path", PATHS, ids=lambda o: f"radix{1 << o.get('log2_radix', 1)}")
def test_ablation_paths(logN, bits, path):
    N, L, P = 1 << logN, 2, 2
    seed = 6000 + logN + bits
    primes = synth.gen_primes(seed, N, bits, L)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(seed, primes, N, P)
    plan = ntt.ntt_plan_create(N, primes, **path)
    try:
        k = path.get("log2_radix", 1)
        assert ntt.ntt_plan_log2_radix(plan) == k
        assert ntt.ntt_plan_num_passes(plan) == -(-logN // k)
        want = oracle.forward(data, primes, psis, THREADS)
        d = dev(data)
        ntt.ntt_forward(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), want), "forward"
        ntt.ntt_inverse(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), data), "inverse(forward)"
        d = dev(data)
        ntt.ntt_inverse(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), oracle.inverse(data, primes, psis, THREADS)), "inverse"
        d = dev(data)
        for p in range(ntt.ntt_plan_num_passes(plan)):
            ntt.ntt_forward_pass(plan, d, p)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), want), "forward by passes"
        if logN >= 10:
            b = synth.residue_batch(seed + 1, primes, N, P)
            c = torch.empty_like(d)
            ntt.ntt_polymul_negacyclic(plan, dev(data), dev(b), c)
            torch.cuda.synchronize()
            assert np.array_equal(host(c), oracle.polymul(data, b, primes, psis, THREADS)), "product"
    finally:
        plan.destroy()


@pytest.mark.parametrize("mode", ["plain", "grouped", "graph"])
def test_ablation_paths_in_batches(mode):
    chain = synth.gen_primes(6100, 1 << 15, 60, 3)
    plans = {"r2": ntt.ntt_plan_create(1 << 11, chain, kernel_path=ntt.PATH_RADIX2),
             "r16": ntt.ntt_plan_create(1 << 15, chain, kernel_path=ntt.PATH_REGISTER, log2_radix=4)}
    m = {"plain": ntt.BATCH_PLAIN, "grouped": ntt.BATCH_GROUPED, "graph": ntt.BATCH_GRAPH}[mode]
    try:
        jobs, bufs, want = [], [], []
        for i, (name, logN, limbs, op) in enumerate([("r2", 11, 2, ntt.OP_FORWARD), ("r16", 15, 3, ntt.OP_INVERSE),
                                                    ("r16", 15, 2, ntt.OP_FORWARD | ntt.OP_MULKEY | ntt.OP_INVERSE)]):
            N = 1 << logN
            primes = chain[:limbs]
            psis = oracle.roots(primes, N)
            data = synth.residue_batch(6110 + i, primes, N, 2)
            key = None
            if op == ntt.OP_FORWARD:
                w = oracle.forward(data, primes, psis, THREADS)
            elif op == ntt.OP_INVERSE:
                w = oracle.inverse(data, primes, psis, THREADS)
            else:
                kc = synth.residue_batch(6120 + i, primes, N, 1).reshape(limbs, N)
                key = dev(oracle.forward(kc, primes, psis, THREADS))
                w = oracle.polymul(data.reshape(2 * limbs, N), np.tile(kc, (2, 1)), primes, psis,
                                   THREADS).reshape(data.shape)
            d = dev(data)
            bufs.append(d)
            want.append(w)
            jobs.append((plans[name], d, 2, limbs if limbs < 3 else 0, op) + ((key,) if key is not None else ()))
        batch = ntt.ntt_batch_create(jobs)
        ntt.ntt_batch_run(batch, m)
        torch.cuda.synchronize()
        for i, (d, w) in enumerate(zip(bufs, want)):
            assert np.array_equal(host(d), w), f"job {i}"
        batch.destroy()
    finally:
        for p in plans.values():
            p.destroy()
