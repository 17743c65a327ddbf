"""Per-shape choice of the plan options by measurement.

For a transform size N, a prime chain and a batch width (polynomials per call), the
tuner times forward+inverse round trips of every plan option set that the library
supports for that N:

* the split N = N1 x N2 between the column and the row pass (or one pass for N <= 2^13),
  as in the paper's choice of kernel sizes for its two-kernel NTT (Section VI-C);
* stored twiddle tables, or on-the-fly twiddling on the last one or two stages with a
  digit base of 2^8, 2^10 or 2^12 (Section VII);
* the two-launch path, or the single persistent launch where that shape exists.

A second round then takes the fastest few split plans of the first and tries their tile
shapes: values per lane of the row pass (the per-thread NTT size of Section VI-C: 4 or 8),
row-pass workgroup lanes (64, 128 or 256) and column-pass tile width (16 to 256 adjacent
columns), each distinct kernel shape once.  Every candidate's forward transform, inverse
and negacyclic product are compared bit for bit with those of the default plan on the same
inputs (all of them compute the same exact residues), and its inverse must undo its
forward transform; a candidate that fails any of these is dropped and reported.

Results are cached in a JSON file keyed by the device, a hash of the kernel sources and
the shape, so a shape is measured once per library build.  The cache is
``$NTT_TUNE_CACHE`` if set, else ``tune_cache.json`` next to this file.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import (PATH_FUSED, PATH_SPLIT, TWIDDLE_OT, TWIDDLE_TABLE, NttError, ntt_forward, ntt_inverse,
               ntt_plan_create, ntt_plan_get_info, ntt_polymul_negacyclic)

__all__ = ["candidates", "tile_candidates", "source_hash", "cache_path", "flat_path", "flat_lines", "lookup",
           "tune", "plan_create_tuned"]

_HERE = os.path.dirname(os.path.abspath(__file__))
FUSED_SHAPES = {(6, 7), (7, 7), (7, 8), (8, 8), (8, 9)}
MALL_BYTES = 256 << 20
TILE_ROUND_PLANS = 3   # split plans of the first round whose tile shapes are tried


from .build import source_hash  # noqa: E402  (one definition, compiled into the library)


def cache_path() -> str:
    return os.environ.get("NTT_TUNE_CACHE") or os.path.join(_HERE, "tune_cache.json")


def candidates(N: int) -> list[dict]:
    """Every option set the library accepts for size N (see the module docstring)."""
    logN = N.bit_length() - 1
    if N < 2 or N != 1 << logN or logN > 17:
        raise ValueError("N must be a power of two in [2, 2^17]")
    splits = []
    if logN <= 13:
        splits.append(-1)                                   # one pass
    splits += [n1 for n1 in range(4, 11) if 4 <= logN - n1 <= 13]
    out = []
    for n1 in splits:
        rows = logN if n1 < 0 else logN - n1
        tw = [dict(twiddle_mode=TWIDDLE_TABLE)]
        for stages in (1, 2):
            if rows <= stages or logN < stages + 1:
                continue
            for b in (8, 10, 12):
                if b < logN:
                    tw.append(dict(twiddle_mode=TWIDDLE_OT, ot_stages=stages, ot_log2_base=b))
        for t in tw:
            out.append(dict(log2_n1=n1, kernel_path=PATH_SPLIT, **t))
            if n1 > 0 and (n1, logN - n1) in FUSED_SHAPES:
                out.append(dict(log2_n1=n1, kernel_path=PATH_FUSED, **t))
    return out


COL_LR = 3          # log2 values per lane of the column pass (build-time constant)
ROW_THREADS = 128   # default row-pass workgroup lanes
TILE_R1 = (8, 4)
TILE_WG = (128, 64, 256)
TILE_COL = (0, 16, 32, 64, 128, 256)


def _col_width(logN: int, n1: int, col_width: int) -> int:
    """Columns per column-pass tile the library takes for a requested width (0 = its
    automatic choice): at most 1024 lanes of 2^min(3, log2 N1) values each."""
    t = (1 << n1) >> min(COL_LR, n1)
    def clip(w):
        return 1024 // t if w * t > 1024 else w
    if col_width:
        return clip(col_width)
    narrow, wide = clip(16), clip(64)
    if wide != narrow and wide * t <= 512 and (1 << (logN - n1)) >= wide:
        return wide
    return narrow


def tile_candidates(N: int, opts: dict) -> list[dict]:
    """Tile shapes for a split (or one-pass) plan with options `opts`: `opts` plus r1, wg_size
    and col_width, one per distinct kernel shape, the built-in default (no tile keys) first.
    Fused and other paths have no tile options."""
    logN = N.bit_length() - 1
    if opts.get("kernel_path", PATH_SPLIT) != PATH_SPLIT:
        return [dict(opts)]
    n1 = opts.get("log2_n1", 0)
    if n1 == 0:
        n1 = 0 if logN <= 12 else logN // 2
    n1 = max(n1, 0)
    logm = logN - n1
    out, seen = [], set()
    for r1 in TILE_R1:
        lr = r1.bit_length() - 1
        t = (1 << logm) >> min(lr, logm)
        if t > 1024:                      # a row's lanes form one workgroup of at most 1024
            continue
        for wg in TILE_WG:
            v = max(1, wg // t)
            for cw in (TILE_COL if n1 else (0,)):
                if cw and (1 << (logN - n1)) < _col_width(logN, n1, cw):
                    continue
                shape = (lr, v, _col_width(logN, n1, cw) if n1 else 0)
                if shape in seen:
                    continue
                seen.add(shape)
                o = dict(opts)
                if r1 != 8:
                    o["r1"] = r1
                if wg != ROW_THREADS:
                    o["wg_size"] = wg
                if cw:
                    o["col_width"] = cw
                out.append(o)
    return out


def _key(device: str, N: int, primes, polys: int) -> str:
    width = max(int(q).bit_length() for q in primes)
    return f"{device}|{source_hash()}|N={N}|L={len(primes)}|P={polys}|qbits={width}"


def _device_name(torch) -> str:
    """Architecture and compute-unit count: what the measured choice depends on (the
    marketing name string differs between otherwise identical boxes)."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = (getattr(p, "gcnArchName", "") or p.name).split(":")[0]
    return f"{arch}:{p.multi_processor_count}CU"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) and d.get("version") == 1 else {"version": 1, "entries": {}}
    except (OSError, ValueError):
        return {"version": 1, "entries": {}}


def flat_path(path: str | None = None) -> str:
    """The flat text copy of the cache that the C library reads (use_autotune): the JSON
    cache's path with a .txt suffix."""
    base = path or cache_path()
    return (base[:-5] if base.endswith(".json") else base) + ".txt"


def flat_lines(cache: dict) -> list[str]:
    """One line per cached shape, in the format of csrc/tune_file.hpp:
    <device> <source_hash> <N> <L> <P> <qbits> <log2_n1> <twiddle_mode> <ot_stages> <ot_log2_base> <kernel_path>
    <r1> <wg_size> <col_width>"""
    out = []
    for key, e in sorted(cache["entries"].items()):
        parts = key.split("|")
        if len(parts) != 6:
            continue
        dev, h, n, l, p, qb = parts
        o = e["opts"]
        vals = [dev, h, n.split("=")[1], l.split("=")[1], p.split("=")[1], qb.split("=")[1],
                o.get("log2_n1", 0), o.get("twiddle_mode", 0), o.get("ot_stages", 0), o.get("ot_log2_base", 0),
                o.get("kernel_path", 0), o.get("r1", 0), o.get("wg_size", 0), o.get("col_width", 0)]
        out.append(" ".join(str(v) for v in vals))
    return out


def _store(path: str, cache: dict) -> None:
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    flat = flat_path(path)
    tmp = f"{flat}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        f.write("".join(line + "\n" for line in flat_lines(cache)))
    os.replace(tmp, flat)


def _inputs(torch, N: int, primes, polys: int, rotate_bytes: int):
    """Uniform residues [polys][L][N] on the device, and enough copies to exceed the MALL."""
    L = len(primes)
    g = torch.Generator(device="cuda")
    g.manual_seed(N * 1000003 + L)
    x = torch.empty((polys, L, N), dtype=torch.int64, device="cuda")
    for l, q in enumerate(primes):
        x[:, l].random_(0, int(q), generator=g)
    per = x.numel() * 8
    R = max(2, min(64, math.ceil(rotate_bytes / per)))
    bufs = x.unsqueeze(0).repeat(R, 1, 1, 1)
    return x, bufs


def _time(torch, plan, bufs, steps: int, warmup: int, ramp_s: float = 0.01) -> float:
    R = bufs.shape[0]
    t0 = time.perf_counter()
    i = 0
    # at least `warmup` round trips and `ramp_s` seconds, so that every candidate is timed at
    # the same (risen) clock
    while i < warmup or time.perf_counter() - t0 < ramp_s:
        ntt_forward(plan, bufs[i % R])
        ntt_inverse(plan, bufs[i % R])
        i += 1
        if i % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        ntt_forward(plan, bufs[i % R])
        ntt_inverse(plan, bufs[i % R])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / steps


def _outputs(torch, plan, x, x2) -> dict:
    """Forward, inverse and negacyclic product of the tuning inputs under `plan`."""
    f = x.clone()
    ntt_forward(plan, f)
    i = x.clone()
    ntt_inverse(plan, i)
    m = torch.empty_like(x)
    ntt_polymul_negacyclic(plan, x, x2, m)
    torch.cuda.synchronize()
    return {"forward": f, "inverse": i, "product": m}


def _disagrees(torch, plan, x, x2, ref) -> str:
    """Name of the first entry point whose result under `plan` differs from the reference
    plan's, or of a failed round trip; '' when everything agrees."""
    out = _outputs(torch, plan, x, x2)
    for name in ("forward", "inverse", "product"):
        if not torch.equal(out[name], ref[name]):
            return name
    back = out["forward"]
    ntt_inverse(plan, back)
    torch.cuda.synchronize()
    if not torch.equal(back, x):
        return "inverse(forward)"
    return ""


def lookup(N: int, primes, polys: int = 1, path: str | None = None):
    """The cached entry for this shape on this device and kernel build, or None."""
    import torch
    return _load(path or cache_path())["entries"].get(_key(_device_name(torch), N, primes, polys))


def tune(N: int, primes, polys: int = 1, *, steps: int = 100, warmup: int = 3, refresh: bool = False,
         path: str | None = None, log=None) -> dict:
    """Best option set for (N, primes, polys); measured unless cached.  Returns
    {"opts": {...}, "us": forward+inverse microseconds per call, "tried": [...]}."""
    import torch
    path = path or cache_path()
    cache = _load(path)
    key = _key(_device_name(torch), N, primes, polys)
    if not refresh and key in cache["entries"]:
        return cache["entries"][key]
    x, bufs = _inputs(torch, N, primes, polys, 2 * MALL_BYTES)
    x2 = torch.flip(x, dims=[-1]).contiguous()     # a second operand for the product check
    # reference results from the default plan: every candidate computes the same exact
    # residues, so one that differs on any entry point is dropped (and reported)
    ref_plan = ntt_plan_create(N, primes)
    try:
        ref = _outputs(torch, ref_plan, x, x2)
    finally:
        ref_plan.destroy()
    tried, dropped, refused = [], [], []
    t0 = time.perf_counter()

    def measure(opts):
        try:
            plan = ntt_plan_create(N, primes, **opts)
        except NttError as e:
            refused.append({"opts": opts, "error": str(e)})
            return
        try:
            bad = _disagrees(torch, plan, x, x2, ref)
            if bad:
                dropped.append({"opts": opts, "differs": bad})
                if log:
                    log(f"  N={N} L={len(primes)} P={polys} {opts}: dropped ({bad} differs)")
                return
            us = _time(torch, plan, bufs, steps, warmup)
            info = ntt_plan_get_info(plan)
            tried.append({"opts": opts, "us": round(us, 3), "log2_n1": info["log2_n1"]})
            if log:
                log(f"  N={N} L={len(primes)} P={polys} {opts}: {us:.1f} us")
        finally:
            plan.destroy()

    for opts in candidates(N):
        measure(opts)
    # second round: the tile shapes of the fastest split plans
    split = sorted((t for t in tried if t["opts"].get("kernel_path", PATH_SPLIT) == PATH_SPLIT), key=lambda t: t["us"])
    for t in split[:TILE_ROUND_PLANS]:
        for opts in tile_candidates(N, t["opts"])[1:]:
            measure(opts)
    if not tried:
        first = refused[0]["error"] if refused else "every candidate disagreed with the first"
        raise RuntimeError(f"no plan options work for N={N}: {first}")
    best = min(tried, key=lambda t: t["us"])
    entry = {"opts": best["opts"], "us": best["us"], "tried": sorted(tried, key=lambda t: t["us"]),
             "dropped": dropped, "seconds": round(time.perf_counter() - t0, 2)}
    cache["entries"][key] = entry
    try:
        _store(path, cache)
    except OSError:
        pass                      # a read-only location still returns the measured choice
    return entry


def plan_create_tuned(N: int, primes, polys: int = 1, **kw):
    """ntt_plan_create with the tuned options for this shape."""
    return ntt_plan_create(N, primes, **tune(N, primes, polys, **kw)["opts"])
