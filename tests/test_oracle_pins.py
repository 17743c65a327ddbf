"""Pins for the CPU oracle: checks against facts that do not come from the oracle itself.

Every pin here is one of: a hand-derived worked example (tests/golden), brute force on
tiny inputs, a closed form or special case, an invariant of the mathematics, or a
library routine (numpy's integer convolution, trial division).  The mutation tests at
the end plant plausible mistakes in copies of the oracle and check that a pin fails.
"""
import os
import random

import numpy as np
import pytest

import oracle
import synth
from oracle import ntt_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, name, N, q, psi, a, out = [x.strip() for x in line.split("|")]
        rows.append((kind, name, int(N), int(q), int(psi), a, out))
    return rows


def _ints(s):
    return [int(x) for x in s.split()]


# ----------------------------------------------------------------- primality

def _trial_division(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def test_is_prime_matches_trial_division():
    for n in range(0, 20000):
        assert O.is_prime(n) == _trial_division(n), n


def test_is_prime_known_values():
    # strong pseudoprimes to small base sets must be rejected
    for n in (2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383,
              341550071728321, 3825123056546413051):
        assert not O.is_prime(n), n
    # 2^61 - 1 (Mersenne prime) and 2^64 - 59 (largest 64-bit prime)
    assert O.is_prime((1 << 61) - 1)
    assert O.is_prime((1 << 64) - 59)
    assert not O.is_prime((1 << 61) + 1)


def test_synth_primes_properties():
    for seed, n_max, bits, count in ((1, 1 << 12, 54, 4), (2, 1 << 16, 60, 45), (4, 1 << 17, 60, 60)):
        ps = synth.gen_primes(seed, n_max, bits, count)
        assert len(ps) == count and len(set(ps)) == count
        for q in ps:
            assert (1 << (bits - 1)) <= q < (1 << bits)
            assert q % (2 * n_max) == 1
            assert O.is_prime(q)
        assert ps == synth.gen_primes(seed, n_max, bits, count)  # deterministic


def test_synth_residues():
    q = synth.gen_primes(7, 1 << 10, 60, 1)[0]
    a = synth.uniform_residues(7, 0, 0, q, 1 << 16)
    assert a.dtype == np.uint64 and int(a.max()) < q
    assert np.array_equal(a, synth.uniform_residues(7, 0, 0, q, 1 << 16))
    b = synth.uniform_residues(7, 1, 0, q, 1 << 16)
    assert not np.array_equal(a, b)
    # mean of U[0, q) is q/2: the sample mean of 65536 draws lies within 1% of it
    assert abs(float(a.astype(np.float64).mean()) / (q / 2) - 1.0) < 0.01
    # first draws of SplitMix64 from state 0 (published reference values of the generator)
    g = synth.SplitMix64(0)
    assert [g.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


# ----------------------------------------------------------------- roots

def _brute_smallest_primitive_root(q, N):
    for x in range(2, q):
        if pow(x, N, q) == q - 1:
            return x
    raise AssertionError


@pytest.mark.parametrize("q,N", [(17, 4), (17, 8), (97, 16), (193, 32), (257, 64), (257, 128),
                                 (1153, 16), (7681, 256), (12289, 1024), (40961, 4096)])
def test_psi_is_smallest_primitive_root_bruteforce(q, N):
    psi = O.find_psi(q, N)
    assert psi == _brute_smallest_primitive_root(q, N)
    assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1


def test_psi_large_primes_invariants():
    for bits, n in ((54, 1 << 12), (60, 1 << 16), (60, 1 << 17)):
        for q in synth.gen_primes(11, n, bits, 3):
            psi = O.find_psi(q, n)
            assert pow(psi, n, q) == q - 1
            assert pow(psi, 2 * n, q) == 1
            # minimality: every odd power of psi (all primitive 2n-th roots) is >= psi
            sq = psi * psi % q
            cur = psi
            for _ in range(n - 1):
                cur = cur * sq % q
                assert cur >= psi


def test_golden_psi():
    for kind, name, N, q, psi, _, _ in _golden():
        if kind in ("psi", "forward", "polymul"):
            assert O.find_psi(q, N) == psi, name


# ----------------------------------------------------------------- forward

def test_golden_forward():
    n = 0
    for kind, name, N, q, psi, a, out in _golden():
        if kind != "forward":
            continue
        a, out = _ints(a), _ints(out)
        assert O.forward_definition(a, q, psi) == out, name
        assert O.forward_radix2(a, q, psi) == out, name
        got = oracle.forward(np.array([a], dtype=np.uint64), [q], [psi])[0].tolist()
        assert got == out, name
        n += 1
    assert n == 2


def test_golden_polymul():
    for kind, name, N, q, psi, ab, out in _golden():
        if kind != "polymul":
            continue
        a, b = [_ints(s) for s in ab.split(";")]
        out = _ints(out)
        assert O.negacyclic_schoolbook(a, b, q) == out
        assert O.polymul_ntt(a, b, q, psi) == out
        assert oracle.polymul(np.array([a], dtype=np.uint64), np.array([b], dtype=np.uint64), [q], [psi])[0].tolist() == out


def test_forward_n2_closed_form():
    # N = 2: X^2 + 1 has roots psi and -psi; slot 0 is a(psi), slot 1 is a(psi^3) = a(-psi)
    for q in (5, 13, 17, 29, 37, 41):
        psi = O.find_psi(q, 2)
        for a0, a1 in ((1, 0), (0, 1), (3, 4), (q - 1, q - 2)):
            assert O.forward_radix2([a0, a1], q, psi) == [(a0 + psi * a1) % q, (a0 - psi * a1) % q]


def test_output_points_are_the_roots_of_xn_plus_1():
    for q, N in ((97, 16), (7681, 256)):
        psi = O.find_psi(q, N)
        xs = O.output_points(q, psi, N)
        assert len(set(xs)) == N
        assert all(pow(x, N, q) == q - 1 for x in xs)


def test_forward_special_inputs():
    q, N = 7681, 64
    psi = O.find_psi(q, N)
    xs = O.output_points(q, psi, N)
    e0 = [1] + [0] * (N - 1)
    assert O.forward_radix2(e0, q, psi) == [1] * N
    for k in (1, 2, 5, N - 1):
        ek = [0] * N
        ek[k] = 1
        assert O.forward_radix2(ek, q, psi) == [pow(x, k, q) for x in xs]


def test_forward_linearity():
    rnd = random.Random(3)
    q, N = 12289, 512
    psi = O.find_psi(q, N)
    a = [rnd.randrange(q) for _ in range(N)]
    b = [rnd.randrange(q) for _ in range(N)]
    al = 1234
    lhs = O.forward_radix2([(al * x + y) % q for x, y in zip(a, b)], q, psi)
    fa, fb = O.forward_radix2(a, q, psi), O.forward_radix2(b, q, psi)
    assert lhs == [(al * x + y) % q for x, y in zip(fa, fb)]


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64, 128])
def test_radix2_equals_definition(N):
    rnd = random.Random(N)
    for q in (synth.gen_primes(N, N, 30, 1)[0], synth.gen_primes(N, N, 60, 1)[0]):
        psi = O.find_psi(q, N)
        a = [rnd.randrange(q) for _ in range(N)]
        d = O.forward_definition(a, q, psi)
        assert O.forward_radix2(a, q, psi) == d
        assert O.inverse_definition(d, q, psi) == a
        assert O.inverse_gs(d, q, psi) == a


def test_inverse_special_and_roundtrip():
    q, N = 40961, 1024
    psi = O.find_psi(q, N)
    assert O.inverse_gs([1] * N, q, psi) == [1] + [0] * (N - 1)
    rnd = random.Random(5)
    y = [rnd.randrange(q) for _ in range(N)]
    assert O.forward_radix2(O.inverse_gs(y, q, psi), q, psi) == y


# ----------------------------------------------------------------- products

def _numpy_negacyclic(a, b, q):
    full = np.convolve(np.array(a, dtype=object), np.array(b, dtype=object))
    N = len(a)
    c = [int(full[k]) - (int(full[k + N]) if k + N < len(full) else 0) for k in range(N)]
    return [x % q for x in c]


def test_schoolbook_matches_numpy_convolution():
    rnd = random.Random(9)
    for N in (4, 16, 64):
        q = synth.gen_primes(N, N, 60, 1)[0]
        a = [rnd.randrange(q) for _ in range(N)]
        b = [rnd.randrange(q) for _ in range(N)]
        assert O.negacyclic_schoolbook(a, b, q) == _numpy_negacyclic(a, b, q)
        assert oracle.schoolbook(np.array(a, dtype=np.uint64), np.array(b, dtype=np.uint64), q).tolist() == \
            _numpy_negacyclic(a, b, q)


def test_polymul_small_coefficients_is_integer_convolution():
    # small inputs: the integer negacyclic convolution never wraps mod q
    rnd = random.Random(10)
    N = 256
    q = synth.gen_primes(1, N, 60, 1)[0]
    psi = O.find_psi(q, N)
    a = [rnd.randrange(-50, 51) for _ in range(N)]
    b = [rnd.randrange(-50, 51) for _ in range(N)]
    want = _numpy_negacyclic(a, b, q)
    got = O.polymul_ntt([x % q for x in a], [x % q for x in b], q, psi)
    assert got == want


def test_polymul_xn_minus_one_times_x():
    q, N = 12289, 256
    psi = O.find_psi(q, N)
    a = [0] * N
    a[N - 1] = 1
    b = [0] * N
    b[1] = 1
    assert O.polymul_ntt(a, b, q, psi) == [q - 1] + [0] * (N - 1)


# ----------------------------------------------------------------- C oracle

def test_c_oracle_matches_python_oracle():
    N = 256
    primes = synth.gen_primes(21, N, 60, 3)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(21, primes, N, 2)
    fc = oracle.forward(data, primes, psis, threads=3)
    for p in range(2):
        for l, q in enumerate(primes):
            assert fc[p, l].tolist() == O.forward_radix2(data[p, l].tolist(), q, psis[l])
    ic = oracle.inverse(fc, primes, psis)
    assert np.array_equal(ic, data)
    for l, q in enumerate(primes):
        assert ic[1, l].tolist() == O.inverse_gs(fc[1, l].tolist(), q, psis[l])


def test_c_oracle_full_size_against_definition_slots():
    N = 1 << 16
    primes = synth.gen_primes(2, N, 60, 2)
    psis = oracle.roots(primes, N)
    data = synth.residue_batch(2, primes, N, 1)
    f = oracle.forward(data, primes, psis, threads=2)
    rnd = random.Random(1)
    for l, q in enumerate(primes):
        for i in [0, 1, N - 1] + [rnd.randrange(N) for _ in range(8)]:
            assert int(f[0, l, i]) == oracle.forward_at(data[0, l], q, psis[l], i)
            assert int(f[0, l, i]) == O.forward_at(data[0, l].tolist(), q, psis[l], i)
        for n in (0, 7, N - 1):
            assert oracle.inverse_at(f[0, l], q, psis[l], n) == int(data[0, l, n])
    assert np.array_equal(oracle.inverse(f, primes, psis, threads=2), data)


# ----------------------------------------------------------------- mutations (planted on CPU)

def _mutant_forward(kind):
    def fwd(a, q, psi):
        a = [x % q for x in a]
        N = len(a)
        b = O.log2_exact(N)
        Psi = O.psi_table(q, psi, N)
        if kind == "no_bitrev":
            Psi = [pow(psi, i, q) for i in range(N)]
        if kind == "omega_not_psi":
            Psi = [pow(psi * psi % q, O.bitrev(i, b), q) for i in range(N)]
        span = N
        while span >= 2:
            half, blocks = span // 2, N // span
            for j in range(blocks):
                w = Psi[j if kind == "index_j" else blocks + j]
                for k in range(j * span, j * span + half):
                    v = a[k + half] * w % q
                    if kind == "sign":
                        a[k + half], a[k] = (a[k] + v) % q, (a[k] - v) % q
                    elif kind == "operand":
                        v = a[k] * w % q
                        a[k + half], a[k] = (a[k + half] - v) % q, (a[k + half] + v) % q
                    else:
                        a[k + half], a[k] = (a[k] - v) % q, (a[k] + v) % q
            span //= 2
        return a
    return fwd


def _pins_hold(fwd):
    for kind, name, N, q, psi, a, out in _golden():
        if kind == "forward" and fwd(_ints(a), q, psi) != _ints(out):
            return False
    q, N = 7681, 32
    psi = O.find_psi(q, N)
    xs = O.output_points(q, psi, N)
    e1 = [0, 1] + [0] * (N - 2)
    if fwd(e1, q, psi) != xs:
        return False
    rnd = random.Random(2)
    a = [rnd.randrange(q) for _ in range(N)]
    b = [rnd.randrange(q) for _ in range(N)]
    prod = [x * y % q for x, y in zip(fwd(a, q, psi), fwd(b, q, psi))]
    return prod == fwd(_numpy_negacyclic(a, b, q), q, psi)


def test_pins_accept_the_oracle():
    assert _pins_hold(O.forward_radix2)


@pytest.mark.parametrize("kind", ["no_bitrev", "omega_not_psi", "index_j", "sign", "operand"])
def test_pins_reject_planted_mistakes(kind):
    assert not _pins_hold(_mutant_forward(kind))


# ----------------------------------------------------------------- natural order (Section III-C)

def _natural_pins_hold(fwd_nat):
    """Pins of a natural-order forward transform: e_1 goes to the N roots psi^(2k+1) of
    X^N + 1 in increasing exponent order (each a root, all distinct), and the transform turns
    the negacyclic convolution (numpy's integer convolution, folded) into the slot-wise
    product."""
    q, N = 7681, 32
    psi = O.find_psi(q, N)
    e1 = [0, 1] + [0] * (N - 2)
    xs = fwd_nat(e1, q, psi)
    if len(set(xs)) != N or any(pow(x, N, q) != q - 1 for x in xs):
        return False
    if any(xs[k + 1] != xs[k] * psi * psi % q for k in range(N - 1)) or xs[0] != psi:
        return False
    rnd = random.Random(3)
    a = [rnd.randrange(q) for _ in range(N)]
    b = [rnd.randrange(q) for _ in range(N)]
    prod = [x * y % q for x, y in zip(fwd_nat(a, q, psi), fwd_nat(b, q, psi))]
    return prod == fwd_nat(_numpy_negacyclic(a, b, q), q, psi)


def test_natural_definition_pins():
    assert _natural_pins_hold(O.forward_natural_definition)


def test_natural_pins_reject_planted_mistakes():
    # the twist dropped (psi^(2k) instead of psi^(2k+1)): a cyclic transform
    def untwisted(a, q, psi):
        N = len(a)
        return [sum(a[n] * pow(psi, 2 * k * n, q) for n in range(N)) % q for k in range(N)]
    # Algorithm 1's bit-reversed order passed off as natural
    assert not _natural_pins_hold(untwisted)
    assert not _natural_pins_hold(O.forward_definition)


def test_natural_order_of_the_c_oracle():
    """natural_order() of the C oracle's (bit-reversed) forward output equals the natural
    definition, computed independently in Python."""
    q_list = synth.gen_primes(77, 64, 60, 2)
    psis = oracle.roots(q_list, 64)
    data = synth.residue_batch(77, q_list, 64, 1)
    nat = oracle.natural_order(oracle.forward(data, q_list, psis))
    for l, q in enumerate(q_list):
        assert nat[0, l].tolist() == O.forward_natural_definition(data[0, l].tolist(), q, psis[l])


# ----------------------------------------------------------------- residue number system (Section III-B)

def _crt_golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crt_examples.txt")
    out = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, name, mods, res, x = [f.strip() for f in line.split("|")]
        assert kind == "crt"
        out.append((name, _ints(mods), _ints(res), int(x)))
    return out


def _crt_pins_hold(reconstruct):
    """Pins of a reconstruction: the hand-derived cases, round trips at full width (45 primes
    of 60 bits), the ring homomorphism, and the idempotents (e_l maps to the number that is 1
    mod q_l and 0 mod every other prime)."""
    for name, mods, res, x in _crt_golden():
        if reconstruct(res, mods) != x or O.rns_decompose(x, mods) != res:
            return False
    primes = synth.gen_primes(2, 1 << 16, 60, 45)
    Q = 1
    for q in primes:
        Q *= q
    xs = synth.words_to_ints(synth.uniform_wide(11, 0, Q, 40))
    for x in xs:
        if reconstruct(O.rns_decompose(x, primes), primes) != x:
            return False
    a, b = xs[0], xs[1]
    ra, rb = O.rns_decompose(a, primes), O.rns_decompose(b, primes)
    if reconstruct([u * v % q for u, v, q in zip(ra, rb, primes)], primes) != a * b % Q:
        return False
    if reconstruct([(u + v) % q for u, v, q in zip(ra, rb, primes)], primes) != (a + b) % Q:
        return False
    for l in (0, 17, 44):
        e = reconstruct([1 if k == l else 0 for k in range(len(primes))], primes)
        if any(e % q != (1 if k == l else 0) for k, q in enumerate(primes)):
            return False
    return True


def test_crt_pins():
    assert _crt_pins_hold(O.crt_reconstruct)


def test_crt_pins_reject_planted_mistakes():
    def prod(ms):
        Q = 1
        for q in ms:
            Q *= q
        return Q

    def no_inverse(r, ms):
        Q = prod(ms)
        return sum(int(x) * (Q // q) for x, q in zip(r, ms)) % Q

    def no_final_mod(r, ms):
        Q = prod(ms)
        return sum(int(x) * (Q // q) * pow((Q // q) % q, q - 2, q) for x, q in zip(r, ms))

    def reduced_weight(r, ms):   # M_l mod q_l in place of M_l
        Q = prod(ms)
        return sum(int(x) * ((Q // q) % q) * pow((Q // q) % q, q - 2, q) for x, q in zip(r, ms)) % Q

    for bad in (no_inverse, no_final_mod, reduced_weight):
        assert not _crt_pins_hold(bad), bad.__name__


def test_wide_words_and_batch_conversions():
    """The word packing round-trips, draws stay below the bound, and the batch conversions
    of the oracle invert each other on [P][W][N] words."""
    primes = synth.gen_primes(5, 1 << 10, 60, 7)
    Q = 1
    for q in primes:
        Q *= q
    w = np.stack([synth.uniform_wide(12, p, Q, 64) for p in range(2)])
    assert w.shape == (2, oracle.crt_words(primes), 64)
    for p in range(2):
        xs = synth.words_to_ints(w[p])
        assert max(xs) < Q and np.array_equal(synth.ints_to_words(xs, w.shape[1]), w[p])
    res = oracle.rns_decompose_words(w, primes)
    assert res.shape == (2, 7, 64)
    assert np.array_equal(oracle.crt_reconstruct_words(res, primes), w)
