"""The tuner on the GPU: every candidate agrees bit for bit, the choice is cached, and the
tuned plan matches the oracle."""
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


@pytest.mark.parametrize("logN,L,P", [(12, 3, 2), (14, 4, 1)])
def test_tune_caches_and_matches_oracle(tmp_path, logN, L, P):
    N = 1 << logN
    primes = synth.gen_primes(3000 + logN, N, 60, L)
    path = str(tmp_path / "tune.json")
    e = autotune.tune(N, primes, P, steps=2, warmup=1, path=path)
    # every first-round candidate, then the tile shapes of the fastest split plans
    first = autotune.candidates(N)
    assert e["dropped"] == [] and len(e["tried"]) > len(first)
    tried = [t["opts"] for t in e["tried"]]
    assert all(c in tried for c in first)
    assert any("r1" in o or "wg_size" in o or "col_width" in o for o in tried)
    assert e["us"] == min(t["us"] for t in e["tried"])
    assert autotune.tune(N, primes, P, path=path) == e                # served from the cache
    plan = autotune.plan_create_tuned(N, primes, P, path=path)
    try:
        data = synth.residue_batch(3100 + logN, primes, N, P)
        d = torch.from_numpy(data.view(np.int64)).to("cuda")
        ntt.ntt_forward(plan, d)
        torch.cuda.synchronize()
        want = oracle.forward(data, primes, oracle.roots(primes, N), THREADS)
        assert np.array_equal(d.cpu().numpy().view(np.uint64), want)
    finally:
        plan.destroy()
