"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws numbers: SplitMix64 streams, NTT-friendly prime chains and
uniform residue arrays.  It holds none of the transform's arithmetic (no roots of
unity, no twiddles, no butterflies), so the oracle and the HIP path can both take
their inputs from here without sharing any of the method.

SplitMix64 is the generator of Steele, Lea and Flood (OOPSLA 2014): the i-th output
of the stream started at state ``s`` is ``mix(s + i*GAMMA)`` for i = 1, 2, ...,
which makes it counter-based and vectorisable.

Derivations (fixed once, documented in the design notes):

* prime chain:  candidates come from the stream ``key(seed, TAG_PRIMES, bits, n_max)``.
* data residue j of (poly p, limb l): attempt a of element j uses counter
  ``a*N + j + 1`` of the stream ``key(seed, TAG_DATA, p, l)``; the draw is masked to
  bitlen(q) bits and accepted when below q (rejection sampling, so the residues
  are exactly uniform on [0, q)).
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

TAG_PRIMES = 0x5052494D  # "PRIM"
TAG_DATA = 0x44415441    # "DATA"
TAG_MISC = 0x4D495343    # "MISC"
TAG_WIDE = 0x57494445    # "WIDE"


def mix64(z: int) -> int:
    """SplitMix64 output function on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def key(seed: int, tag: int, a: int = 0, b: int = 0) -> int:
    """Stream key for one purpose: nested mixes of (seed, tag, a, b)."""
    k = mix64(seed + GAMMA)
    k = mix64(k ^ tag)
    k = mix64(k + (a + 1) * GAMMA)
    k = mix64(k ^ ((b + 1) * M2 & MASK64))
    return k


class SplitMix64:
    """Sequential SplitMix64 stream (scalar draws)."""

    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        return mix64(self.state)


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= np.uint64(M1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(M2)
    z ^= z >> np.uint64(31)
    return z


def stream_np(k: int, counters: np.ndarray) -> np.ndarray:
    """Outputs ``mix(k + c*GAMMA)`` for an array of counters c (uint64, wrapping)."""
    with np.errstate(over="ignore"):
        s = np.uint64(k) + counters.astype(np.uint64) * np.uint64(GAMMA)
    return mix64_np(s)


# ---------------------------------------------------------------- primes (inputs)

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def _is_probable_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases.

    These bases decide primality for every n < 3.317e24 (Sorenson and Webster,
    2015), which covers all 64-bit candidates drawn here.
    """
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x == 1 or x == n - 1:
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def gen_primes(seed: int, n_max: int, bits: int, count: int) -> list[int]:
    """Draw ``count`` distinct primes q with q = 1 mod 2*n_max and 2^(bits-1) <= q < 2^bits.

    Each candidate is 2^(bits-1) + (r mod 2^(bits-1)) for a stream draw r, moved down
    to the nearest value that is 1 mod 2*n_max; it is kept when it stays in range,
    is new, and passes the primality test.
    """
    if n_max < 1 or n_max & (n_max - 1):
        raise ValueError("n_max must be a power of two")
    if not 4 <= bits <= 63:
        raise ValueError("bits out of range")
    two_n = 2 * n_max
    lo = 1 << (bits - 1)
    if lo + 1 < two_n:
        raise ValueError("bits too small for n_max")
    rng = SplitMix64(key(seed, TAG_PRIMES, bits, n_max))
    out: list[int] = []
    seen: set[int] = set()
    guard = 0
    while len(out) < count:
        guard += 1
        if guard > 10_000_000:
            raise RuntimeError("prime search did not converge")
        c = lo + (rng.next() % lo)
        c -= (c - 1) % two_n
        if c < lo or c in seen:
            continue
        if _is_probable_prime(c):
            seen.add(c)
            out.append(c)
    return out


# ---------------------------------------------------------------- residues (inputs)

def uniform_residues(seed: int, poly: int, limb: int, q: int, n: int) -> np.ndarray:
    """n residues uniform on [0, q) for (poly, limb), as uint64 (rejection sampling)."""
    k = key(seed, TAG_DATA, poly, limb)
    mask = np.uint64((1 << q.bit_length()) - 1)
    qq = np.uint64(q)
    idx = np.arange(n, dtype=np.uint64)
    vals = stream_np(k, idx + np.uint64(1)) & mask
    bad = np.nonzero(vals >= qq)[0]
    attempt = 1
    while bad.size:
        c = np.uint64(attempt) * np.uint64(n) + idx[bad] + np.uint64(1)
        vals[bad] = stream_np(k, c) & mask
        bad = bad[vals[bad] >= qq]
        attempt += 1
        if attempt > 200:
            raise RuntimeError("rejection sampling did not converge")
    return vals


def residue_batch(seed: int, primes: list[int], n: int, n_polys: int, poly_offset: int = 0) -> np.ndarray:
    """Array [n_polys][L][n] of uniform residues, limb l drawn mod primes[l]."""
    L = len(primes)
    out = np.empty((n_polys, L, n), dtype=np.uint64)
    for p in range(n_polys):
        for l, q in enumerate(primes):
            out[p, l] = uniform_residues(seed, p + poly_offset, l, q, n)
    return out


def uniform_ints(seed: int, tag_a: int, count: int, lo: int, hi: int) -> list[int]:
    """``count`` integers uniform on [lo, hi] (inclusive), by rejection, for workload mixes."""
    span = hi - lo + 1
    rng = SplitMix64(key(seed, TAG_MISC, tag_a, span))
    bound = (1 << 64) - ((1 << 64) % span)
    out = []
    while len(out) < count:
        r = rng.next()
        if r < bound:
            out.append(lo + r % span)
    return out


def uniform_unit(seed: int, tag_a: int, count: int) -> np.ndarray:
    """``count`` doubles uniform on [0, 1) (53-bit draws), for arrival processes and mixes."""
    k = key(seed, TAG_MISC, tag_a, 0)
    z = stream_np(k, np.arange(1, count + 1, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


# ---------------------------------------------------------------- wide integers (inputs)

def words_needed(bound: int) -> int:
    """64-bit words that hold every integer below ``bound``."""
    return max(1, ((bound - 1).bit_length() + 63) // 64)


def uniform_wide(seed: int, poly: int, bound: int, n: int) -> np.ndarray:
    """n integers uniform on [0, bound), as a [W][n] uint64 array of little-endian 64-bit
    words (W = words_needed(bound)).  Attempt a of element j takes word w from counter
    (a*W + w)*n + j + 1 of the stream key(seed, TAG_WIDE, poly, W), the top word masked to
    bound's bit length; a draw at or above bound is redrawn (rejection sampling)."""
    W = words_needed(bound)
    k = key(seed, TAG_WIDE, poly, W)
    top_bits = (bound - 1).bit_length() - 64 * (W - 1)
    top_mask = np.uint64((1 << top_bits) - 1) if top_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    bw = [np.uint64((bound >> (64 * w)) & 0xFFFFFFFFFFFFFFFF) for w in range(W)]
    idx = np.arange(n, dtype=np.uint64)
    out = np.empty((W, n), dtype=np.uint64)
    todo = np.arange(n)
    attempt = 0
    while todo.size:
        for w in range(W):
            c = (np.uint64(attempt * W + w) * np.uint64(n)) + idx[todo] + np.uint64(1)
            out[w, todo] = stream_np(k, c)
        out[W - 1, todo] &= top_mask
        less = np.zeros(todo.size, dtype=bool)
        eq = np.ones(todo.size, dtype=bool)
        for w in range(W - 1, -1, -1):
            v = out[w, todo]
            less |= eq & (v < bw[w])
            eq &= v == bw[w]
        if bound == 1 << (64 * W):   # every W-word draw lies below the bound
            less[:] = True
        todo = todo[~less]
        attempt += 1
        if attempt > 200:
            raise RuntimeError("rejection sampling did not converge")
    return out


def words_to_ints(words: np.ndarray) -> list[int]:
    """The integers held by a [W][n] array of little-endian 64-bit words."""
    W, n = words.shape
    out = [0] * n
    for w in range(W - 1, -1, -1):
        col = words[w].tolist()
        out = [(x << 64) | int(c) for x, c in zip(out, col)]
    return out


def ints_to_words(values, W: int) -> np.ndarray:
    """[W][n] little-endian 64-bit words of non-negative integers below 2^(64 W)."""
    vals = [int(v) for v in values]
    out = np.empty((W, len(vals)), dtype=np.uint64)
    for w in range(W):
        out[w] = [(v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for v in vals]
    if any(v >> (64 * W) for v in vals):
        raise ValueError("value does not fit in W words")
    return out
