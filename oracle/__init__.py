"""CPU oracle for the negacyclic NTT path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The library (``paper_2012_01968_amd``) never imports it, and it never
imports the library: the two share no code.  Inputs come from ``synth``, which only
draws random numbers.

Two independent implementations live here:

* ``ntt_oracle`` -- Python big integers: primality, the root convention, the O(N^2)
  definitions, Algorithm 1, the Gentleman-Sande inverse and the schoolbook
  negacyclic convolution.
* ``ntt_oracle.c`` (loaded through ctypes) -- plain C with ``__int128 %``: the same
  radix-2 transforms for full-size batches, plus single-slot evaluation of the
  definition for sampled checks at large N.

Functions whose result is pinned only by being the plain definition are pinned by
the tests in ``tests/test_oracle_pins.py``; none is left unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import ntt_oracle as py  # noqa: F401  (re-exported)
from .ntt_oracle import find_psi, is_prime  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntt_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into oracle/_build/liboracle.so."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            for name in ("oracle_forward", "oracle_inverse"):
                f = getattr(L, name)
                f.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint32, u64p, u64p, ctypes.c_uint32, ctypes.c_uint64]
                f.restype = ctypes.c_int
            for name in ("oracle_forward_at", "oracle_inverse_at"):
                f = getattr(L, name)
                f.argtypes = [u64p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
                f.restype = ctypes.c_uint64
            L.oracle_pointwise.argtypes = [u64p, u64p, u64p, ctypes.c_uint64, ctypes.c_uint32, u64p,
                                           ctypes.c_uint32, ctypes.c_uint64]
            L.oracle_pointwise.restype = None
            L.oracle_negacyclic_schoolbook.argtypes = [u64p, u64p, u64p, ctypes.c_uint32, ctypes.c_uint64]
            L.oracle_negacyclic_schoolbook.restype = None
            L.oracle_powmod.argtypes = [ctypes.c_uint64] * 3
            L.oracle_powmod.restype = ctypes.c_uint64
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def _run_vectors(fn_name: str, data: np.ndarray, primes, psis, threads: int | None) -> np.ndarray:
    data = _u64(data).copy()
    N = data.shape[-1]
    L = len(primes)
    n_vec = data.size // N
    if n_vec % L:
        raise ValueError("number of vectors must be a multiple of the number of primes")
    q = _u64(primes)
    ps = _u64(psis)
    fn = getattr(lib(), fn_name)
    threads = max(1, min(threads or 1, n_vec))
    chunks = np.array_split(np.arange(n_vec), threads)
    flat = data.reshape(n_vec, N)

    def work(idx):
        if idx.size == 0:
            return 0
        v0, v1 = int(idx[0]), int(idx[-1]) + 1
        view = flat[v0:v1]
        return fn(_ptr(view), v1 - v0, N, _ptr(q), _ptr(ps), L, v0)

    if threads == 1:
        rcs = [work(chunks[0])]
    else:
        with ThreadPoolExecutor(threads) as ex:
            rcs = list(ex.map(work, chunks))
    if any(rcs):
        raise MemoryError("oracle allocation failed")
    return data


def forward(data, primes, psis, threads: int | None = None) -> np.ndarray:
    """Algorithm 1 on every vector of a [..][L][N] uint64 array (new array, bit-reversed order)."""
    return _run_vectors("oracle_forward", data, primes, psis, threads)


def inverse(data, primes, psis, threads: int | None = None) -> np.ndarray:
    """Gentleman-Sande inverse with the 1/N scale on every vector (natural order out)."""
    return _run_vectors("oracle_inverse", data, primes, psis, threads)


def pointwise(a, b, primes) -> np.ndarray:
    a = _u64(a)
    b = _u64(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    N = a.shape[-1]
    c = np.empty_like(a)
    q = _u64(primes)
    lib().oracle_pointwise(_ptr(a), _ptr(b), _ptr(c), a.size // N, N, _ptr(q), len(primes), 0)
    return c


def polymul(a, b, primes, psis, threads: int | None = None) -> np.ndarray:
    """c = iNTT(NTT(a) * NTT(b)) per vector (negacyclic product in Z_q[X]/(X^N+1))."""
    fa = forward(a, primes, psis, threads)
    fb = forward(b, primes, psis, threads)
    return inverse(pointwise(fa, fb, primes), primes, psis, threads)


def forward_at(vec, q: int, psi: int, i: int) -> int:
    """Output slot i of the forward definition for one vector (O(N))."""
    v = _u64(vec)
    return int(lib().oracle_forward_at(_ptr(v), v.size, q, psi, i))


def inverse_at(vec, q: int, psi: int, n: int) -> int:
    """Coefficient n of the inverse definition for one vector (O(N log q))."""
    v = _u64(vec)
    return int(lib().oracle_inverse_at(_ptr(v), v.size, q, psi, n))


def schoolbook(a, b, q: int) -> np.ndarray:
    a = _u64(a)
    b = _u64(b)
    c = np.empty_like(a)
    lib().oracle_negacyclic_schoolbook(_ptr(a), _ptr(b), _ptr(c), a.size, q)
    return c


def natural_order(x) -> np.ndarray:
    """Slots of the last axis in natural order: slot k of the result is slot brv(k) of x
    (Algorithm 1's output holds A_brv(i) in slot i, so this gives A_k in slot k)."""
    x = _u64(x)
    N = x.shape[-1]
    b = N.bit_length() - 1
    idx = np.array([py.bitrev(k, b) for k in range(N)], dtype=np.int64)
    return np.ascontiguousarray(x[..., idx])


def roots(primes, N: int) -> list[int]:
    """The root convention for every prime: smallest primitive 2N-th root of unity."""
    return [find_psi(int(q), N) for q in primes]


def rns_decompose_words(words, primes) -> np.ndarray:
    """[P][W][N] little-endian 64-bit words of integers -> [P][L][N] residues (Section III-B)."""
    import synth
    words = _u64(words)
    P, W, N = words.shape
    out = np.empty((P, len(primes), N), dtype=np.uint64)
    for p in range(P):
        xs = synth.words_to_ints(words[p])
        for l, q in enumerate(primes):
            out[p, l] = [x % int(q) for x in xs]
    return out


def crt_words(primes) -> int:
    """64-bit words of Q = prod q_l: the width of a reconstructed integer."""
    Q = 1
    for q in primes:
        Q *= int(q)
    return max(1, (Q.bit_length() + 63) // 64)


def crt_reconstruct_words(res, primes) -> np.ndarray:
    """[P][L][N] residues -> [P][W][N] little-endian words of the integers in [0, Q) they
    represent (Chinese remainder theorem, one coefficient at a time)."""
    import synth
    res = _u64(res)
    P, L, N = res.shape
    W = crt_words(primes)
    out = np.empty((P, W, N), dtype=np.uint64)
    for p in range(P):
        cols = [res[p, l].tolist() for l in range(L)]
        xs = [py.crt_reconstruct([cols[l][j] for l in range(L)], primes) for j in range(N)]
        out[p] = synth.ints_to_words(xs, W)
    return out
