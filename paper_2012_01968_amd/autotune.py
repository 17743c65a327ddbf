"""Per-shape choice of the plan options by measurement.

For a transform size N, a prime chain and a batch width (polynomials per call), the
tuner times forward+inverse round trips of every plan option set that the library
supports for that N:

* the split N = N1 x N2 between the column and the row pass (or one pass for N <= 2^13),
  as in the paper's choice of kernel sizes for its two-kernel NTT (Sec. IV-B, IV-D);
* stored twiddle tables, or on-the-fly twiddling on the last one or two stages with a
  digit base of 2^8, 2^10 or 2^12 (Sec. IV-E);
* the two-launch path, or the single persistent launch where that shape exists.

Tile shapes (values per lane, workgroup size) are fixed when the library is built, so
they are not part of the search.  Every candidate's output is compared bit for bit with
the first candidate's on the same input (all of them compute the same exact result), and
a candidate that differs is dropped and reported.

Results are cached in a JSON file keyed by the device, a hash of the kernel sources and
the shape, so a shape is measured once per library build.  The cache is
``$NTT_TUNE_CACHE`` if set, else ``tune_cache.json`` next to this file.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

from . import (PATH_FUSED, PATH_SPLIT, TWIDDLE_OT, TWIDDLE_TABLE, NttError, ntt_forward, ntt_inverse,
               ntt_plan_create, ntt_plan_get_info)

__all__ = ["candidates", "source_hash", "cache_path", "lookup", "tune", "plan_create_tuned"]

_HERE = os.path.dirname(os.path.abspath(__file__))
FUSED_SHAPES = {(6, 7), (7, 7), (7, 8), (8, 8), (8, 9)}
MALL_BYTES = 256 << 20


def source_hash() -> str:
    """Hash of the kernel and ABI sources the library is built from."""
    h = hashlib.sha256()
    csrc = os.path.join(_HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


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


def _store(path: str, cache: dict) -> None:
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


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
    ref = None
    tried, dropped, refused = [], [], []
    t0 = time.perf_counter()
    for opts in candidates(N):
        try:
            plan = ntt_plan_create(N, primes, **opts)
        except NttError as e:
            refused.append({"opts": opts, "error": str(e)})
            continue
        try:
            y = x.clone()
            ntt_forward(plan, y)
            torch.cuda.synchronize()
            if ref is None:
                ref = y
            elif not torch.equal(y, ref):
                dropped.append(opts)
                continue
            us = _time(torch, plan, bufs, steps, warmup)
            info = ntt_plan_get_info(plan)
            tried.append({"opts": opts, "us": round(us, 3), "log2_n1": info["log2_n1"]})
            if log:
                log(f"  N={N} L={len(primes)} P={polys} {opts}: {us:.1f} us")
        finally:
            plan.destroy()
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
