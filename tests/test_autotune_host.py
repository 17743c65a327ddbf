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


def test_tile_candidates_are_distinct_kernel_shapes():
    """The second tuning round's tile shapes: the default first, every r1 / wg_size / col_width
    value one the library accepts, and no two candidates that launch the same kernel shape
    (same values per lane, rows per workgroup and effective column width)."""
    for logN in range(1, 18):
        N = 1 << logN
        for opts in at.candidates(N):
            tiles = at.tile_candidates(N, opts)
            assert tiles[0] == opts
            if opts["kernel_path"] == PATH_FUSED:
                assert tiles == [opts]
                continue
            n1 = opts["log2_n1"] if opts["log2_n1"] > 0 else 0
            logm = logN - n1
            shapes = set()
            for t in tiles:
                assert {k: v for k, v in t.items() if k not in ("r1", "wg_size", "col_width")} == opts
                r1, wg, cw = t.get("r1", 8), t.get("wg_size", 128), t.get("col_width", 0)
                assert r1 in (4, 8) and wg in (64, 128, 256) and cw in (0, 16, 32, 64, 128, 256)
                if n1 == 0:
                    assert cw == 0
                lr = r1.bit_length() - 1
                rows_t = (1 << logm) >> min(lr, logm)
                assert rows_t <= 1024
                w = at._col_width(logN, n1, cw) if n1 else 0
                if cw:
                    assert (1 << (logN - n1)) >= w
                shapes.add((lr, max(1, wg // rows_t), w))
            assert len(shapes) == len(tiles)
    # N = 2^16, N1 = 64: 1024-point rows (128 lanes at r1 = 8, 256 at r1 = 4), 64-point columns
    t16 = at.tile_candidates(1 << 16, dict(log2_n1=6, kernel_path=PATH_SPLIT, twiddle_mode=TWIDDLE_TABLE))
    assert {(t.get("r1", 8), t.get("wg_size", 128)) for t in t16} == {(8, 128), (8, 256), (4, 128)}
    assert at._col_width(16, 6, 0) == 64 and at._col_width(16, 6, 16) == 16 and at._col_width(16, 10, 64) == 8


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
    # a first-round option set, or one of the tile shapes of one
    assert any(opts in at.tile_candidates(1 << 16, c) for c in at.candidates(1 << 16))
