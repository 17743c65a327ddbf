"""The boundary's lifetime and concurrency rules on the device, through the C ABI:

* a plan destroyed by its creator while a batch still names it keeps working for that batch
  (and only for it), and is freed when the batch lets go;
* products on several streams of one plan each use their own scratch and all match the
  oracle, also when they run at the same time and when one stream's scratch grows;
* use_autotune=1 takes the tuner's file entry for a cached shape;
* the measurement's yardstick copy (ntt_device_copy) moves every byte.

Every result is compared with the CPU oracle, element by element.
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


def test_plan_destroyed_while_a_batch_holds_it():
    N, L = 1 << 14, 3
    primes = synth.gen_primes(4100, N, 60, L)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(4100, primes, N, 2)
    want = oracle.forward(data, primes, psis, THREADS)
    plan = ntt.ntt_plan_create(N, primes)
    d = dev(data)
    batch = ntt.ntt_batch_create([(plan, d, 2, 0, ntt.OP_FORWARD)])
    handle = plan.handle
    plan.destroy()                                     # the batch still holds it
    # direct calls on the handle are refused (before any launch); the batch still runs it
    assert ntt._lib.ntt_forward(handle, d.data_ptr(), 2, None) == -1
    assert ntt._lib.ntt_plan_tuned(handle) == -1
    ntt.ntt_batch_run(batch, ntt.BATCH_GROUPED)
    torch.cuda.synchronize()
    assert np.array_equal(host(d), want)
    d.copy_(dev(data))
    ntt.ntt_batch_run(batch, ntt.BATCH_GRAPH)
    torch.cuda.synchronize()
    assert np.array_equal(host(d), want)
    batch.destroy()                                    # last reference: the plan is freed here


def test_destroy_twice_while_held_is_reported():
    N = 1 << 10
    primes = synth.gen_primes(4200, N, 60, 2)
    plan = ntt.ntt_plan_create(N, primes)
    d = dev(synth.residue_batch(4200, primes, N, 1))
    batch = ntt.ntt_batch_create([(plan, d, 1, 0, ntt.OP_FORWARD)])
    handle = plan.handle
    plan.destroy()
    rc = ntt._lib.ntt_plan_destroy(handle)             # second destroy: the batch keeps the plan alive
    assert rc == -1
    batch.destroy()


def test_reassign_releases_the_old_plans():
    """A batch reassigned to jobs of another plan lets go of the first; a plan destroyed by its
    creator and then dropped from the batch is freed, and the batch keeps working."""
    N1, N2 = 1 << 12, 1 << 13
    chain = synth.gen_primes(4300, N2, 60, 2)
    p1 = ntt.ntt_plan_create(N1, chain)
    p2 = ntt.ntt_plan_create(N2, chain)
    a = synth.residue_batch(4300, chain, N1, 1)
    b = synth.residue_batch(4301, chain, N2, 1)
    da, db = dev(a), dev(b)
    batch = ntt.ntt_batch_create([(p1, da, 1, 0, ntt.OP_FORWARD)])
    p1.destroy()
    ntt.ntt_batch_assign(batch, [(p2, db, 1, 0, ntt.OP_FORWARD)])   # p1 freed here
    ntt.ntt_batch_run(batch, ntt.BATCH_GROUPED)
    torch.cuda.synchronize()
    assert np.array_equal(host(db), oracle.forward(b, chain, oracle.roots(chain, N2), THREADS))
    batch.destroy()
    p2.destroy()


def test_products_on_several_streams():
    """Products of one plan on three streams at once, each with its own scratch; then one
    stream's scratch grows (a larger batch) while the others still run."""
    N, L = 1 << 15, 4
    primes = synth.gen_primes(4400, N, 60, L)
    psis = oracle.roots(primes, N)
    plan = ntt.ntt_plan_create(N, primes)
    try:
        streams = [torch.cuda.Stream() for _ in range(3)]
        cases = []
        for k, st in enumerate(streams):
            P = 1 + k
            a = synth.residue_batch(4410 + k, primes, N, P)
            b = synth.residue_batch(4420 + k, primes, N, P)
            cases.append((st, dev(a), dev(b), torch.empty((P, L, N), dtype=torch.int64, device="cuda"),
                          oracle.polymul(a, b, primes, psis, THREADS)))
        torch.cuda.synchronize()
        for _ in range(2):
            for st, da, db, dc, _ in cases:
                ntt.ntt_polymul_negacyclic(plan, da, db, dc, stream=st)
        # grow the first stream's scratch: a 4-polynomial product on it
        a4 = synth.residue_batch(4430, primes, N, 4)
        b4 = synth.residue_batch(4431, primes, N, 4)
        da4, db4 = dev(a4), dev(b4)
        torch.cuda.synchronize()
        dc4 = torch.empty_like(da4)
        ntt.ntt_polymul_negacyclic(plan, da4, db4, dc4, stream=streams[0])
        for st, da, db, dc, _ in cases[1:]:
            ntt.ntt_polymul_negacyclic(plan, da, db, dc, stream=st)
        torch.cuda.synchronize()
        for _, _, _, dc, want in cases:
            assert np.array_equal(host(dc), want)
        assert np.array_equal(host(dc4), oracle.polymul(a4, b4, primes, psis, THREADS))
    finally:
        plan.destroy()


def test_use_autotune_takes_the_cached_choice():
    """For the headline shape the tuner's file has an entry for these kernels; a plan created
    with use_autotune=1 and tune_polys=2 takes exactly that entry's options."""
    from paper_2012_01968_amd import autotune
    N, L, P = 1 << 16, 45, 2
    primes = synth.gen_primes(2, N, 60, L)
    entry = autotune.lookup(N, primes, P)
    if entry is None:
        pytest.skip("the tuner's cache has no entry for these kernel sources on this device")
    plan = ntt.ntt_plan_create(N, primes, use_autotune=1, tune_polys=P)
    try:
        assert ntt.ntt_plan_tuned(plan)
        info = ntt.ntt_plan_get_info(plan)
        o = entry["opts"]
        assert info["log2_n1"] == o["log2_n1"]
        assert info["kernel_path"] == o["kernel_path"]
        assert info["twiddle_mode"] == o["twiddle_mode"]
        if o["twiddle_mode"] == ntt.TWIDDLE_OT:
            assert info["ot_stages"] == o["ot_stages"]
        data = synth.residue_batch(2, primes, N, P)
        d = dev(data)
        ntt.ntt_forward(plan, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), oracle.forward(data, primes, oracle.roots(primes, N), THREADS))
    finally:
        plan.destroy()
    # a shape with no entry keeps the defaults and says so
    small = ntt.ntt_plan_create(1 << 5, synth.gen_primes(7, 1 << 5, 60, 2), use_autotune=1)
    try:
        assert not ntt.ntt_plan_tuned(small)
    finally:
        small.destroy()


def test_device_copy():
    """The measurement's yardstick copy moves every byte, at sizes that leave a partial block."""
    for n in (2, 4096 * 2 + 6, 47185920 // 8):
        src = torch.randint(-(1 << 62), 1 << 62, (n,), dtype=torch.int64, device="cuda")
        dst = torch.zeros_like(src)
        ntt.ntt_device_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
