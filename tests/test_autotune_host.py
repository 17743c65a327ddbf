"""Host side of the tuner: the candidate space follows the library's shape rules, and the
cache file round-trips (no GPU)."""
import json

import pytest

from paper_2012_01968_amd import PATH_FUSED, PATH_SPLIT, TWIDDLE_OT, TWIDDLE_TABLE
from paper_2012_01968_amd import autotune as at


def test_candidates_follow_the_shape_rules():
    for logN in range(1, 18):
        cands = at.candidates(1 << logN)
        assert cands, logN
        keys = {tuple(sorted(c.items())) for c in cands}
        assert len(keys) == len(cands)                          # no duplicates
        for c in cands:
            n1 = c["log2_n1"]
            rows = logN if n1 < 0 else logN - n1
            if n1 < 0:
                assert logN <= 13
            else:
                assert 4 <= n1 <= 10 and 4 <= rows <= 13
            if c["twiddle_mode"] == TWIDDLE_OT:
                assert c["ot_stages"] in (1, 2) and rows > c["ot_stages"] and c["ot_log2_base"] < logN
            else:
                assert c["twiddle_mode"] == TWIDDLE_TABLE and "ot_stages" not in c
            if c["kernel_path"] == PATH_FUSED:
                assert (n1, rows) in at.FUSED_SHAPES
            else:
                assert c["kernel_path"] == PATH_SPLIT
    c16 = at.candidates(1 << 16)
    assert {c["log2_n1"] for c in c16} == {6, 7, 8, 9, 10} | {x for x in range(4, 11) if 16 - x <= 13}
    assert any(c["kernel_path"] == PATH_FUSED for c in c16)
    assert all(c["log2_n1"] > 0 for c in at.candidates(1 << 17))
    assert {c["log2_n1"] for c in at.candidates(1 << 4)} == {-1}
    for bad in (0, 3, 1 << 18):
        with pytest.raises(ValueError):
            at.candidates(bad)


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "cache.json")
    assert at._load(p) == {"version": 1, "entries": {}}
    cache = at._load(p)
    key = at._key("gfx950:256CU", 1 << 16, [(1 << 59) + 1, (1 << 58) + 1], 2)
    assert key.endswith("|N=65536|L=2|P=2|qbits=60") and at.source_hash() in key
    cache["entries"][key] = {"opts": {"log2_n1": 8, "kernel_path": PATH_SPLIT, "twiddle_mode": TWIDDLE_TABLE},
                             "us": 1.0}
    at._store(p, cache)
    assert at._load(p) == cache
    (tmp_path / "bad.json").write_text("{not json")
    assert at._load(str(tmp_path / "bad.json"))["entries"] == {}
    (tmp_path / "old.json").write_text(json.dumps({"version": 0, "entries": {"x": 1}}))
    assert at._load(str(tmp_path / "old.json"))["entries"] == {}


def test_source_hash_tracks_the_kernel_sources():
    h = at.source_hash()
    assert len(h) == 16 and h == at.source_hash()


def test_committed_cache_holds_the_headline_shape():
    """The shipped cache has a plan for N=2^16, L=45 (60-bit primes), 2 polys on a 256-CU gfx950
    for the kernel sources as they stand, so the measurement and its full-size parity test use
    that plan instead of tuning anew."""
    import synth
    primes = synth.gen_primes(2, 1 << 16, 60, 45)
    with open(at.cache_path()) as f:
        entries = json.load(f)["entries"]
    key = at._key("gfx950:256CU", 1 << 16, primes, 2)
    assert key in entries, "tune cache is stale for the current kernel sources"
    assert at.source_hash() in key
    opts = entries[key]["opts"]
    assert opts in at.candidates(1 << 16)
