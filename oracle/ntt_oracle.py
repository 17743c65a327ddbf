"""Plain, slow, exact reference for the negacyclic NTT path (Python big integers).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; only the
test suite, the smoke check and the benchmark's CPU-baseline leg may call it.  It
shares no code with the HIP path: every table and root here is recomputed from
the mathematics with Python integers.

Paper: Kim, Jung, Park, Ahn, "Accelerating Number Theoretic Transformations for
Bootstrappable Homomorphic Encryption on GPUs" (arXiv 2012.01968).

What each function follows:

* ``forward_definition`` -- the merged-twist NTT of Section III-A,
  A_k = sum_n a_n psi_{2N}^{n(2k+1)}, with the output written in bit-reversed order
  as Algorithm 1 leaves it (output slot i holds A_{brv(i)}).
* ``forward_radix2`` -- Algorithm 1 (Cooley-Tukey) with the butterfly of
  Algorithm 2, every value fully reduced mod q, taken stage by stage over blocks.
* ``forward_natural_definition`` -- the same transform with A_k in slot k (the natural
  order of Section III-C), for the library's natural-order option.
* ``inverse_definition`` / ``inverse_gs`` -- the inverse with the Psi^{-1} twist
  and the 1/N scale merged in (Section III-A says the merge is possible; the
  paper prints no inverse algorithm, so the Gentleman-Sande form used here is
  the reading recorded in the design notes).
* ``negacyclic_schoolbook`` -- the convolution formula of Section III-A,
  c_k = sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}.
* ``rns_decompose`` / ``crt_reconstruct`` -- the residue number system of Section III-B:
  an integer below Q = q_0 q_1 ... q_{L-1} is held as its residues mod each q_l, and the
  Chinese remainder theorem recovers it as sum_l r_l M_l (M_l^{-1} mod q_l) mod Q with
  M_l = Q / q_l.
* ``find_psi`` -- the root convention: the smallest primitive 2N-th root of unity
  mod q (the paper does not say which root; this is the stated reading).
"""
from __future__ import annotations

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (bases 2..37, Sorenson-Webster 2015)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d = n - 1
    s = 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        composite = True
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                composite = False
                break
        if composite:
            return False
    return True


def log2_exact(n: int) -> int:
    if n < 1 or n & (n - 1):
        raise ValueError(f"{n} is not a power of two")
    return n.bit_length() - 1


def bitrev(i: int, bits: int) -> int:
    """Reverse the low ``bits`` bits of i."""
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def check_modulus(q: int, N: int) -> None:
    """The conditions Algorithm 1 requires of its prime: q prime and q = 1 mod 2N."""
    if not is_prime(q):
        raise ValueError(f"{q} is not prime")
    if (q - 1) % (2 * N):
        raise ValueError(f"{q} is not 1 mod 2N (N={N})")


def find_psi(q: int, N: int) -> int:
    """Smallest primitive 2N-th root of unity mod q.

    A 2N-th root psi is primitive exactly when psi^N = -1 (2N is a power of two).
    Step 1 finds one such root psi0 as x^((q-1)/2N) for the first x that gives one;
    step 2 takes the minimum over all primitive roots, which are the odd powers
    psi0^k, k < 2N.
    """
    check_modulus(q, N)
    e = (q - 1) // (2 * N)
    x = 2
    while True:
        y = pow(x, e, q)
        if pow(y, N, q) == q - 1:
            psi0 = y
            break
        x += 1
    best = psi0
    sq = psi0 * psi0 % q
    cur = psi0
    for _ in range(N - 1):
        cur = cur * sq % q
        if cur < best:
            best = cur
    return best


def psi_table(q: int, psi: int, N: int) -> list[int]:
    """Psi[i] = psi^{brv(i)} for i < N (the table Algorithm 1 requires)."""
    b = log2_exact(N)
    return [pow(psi, bitrev(i, b), q) for i in range(N)]


def output_points(q: int, psi: int, N: int) -> list[int]:
    """x_i = psi^{2 brv(i) + 1}: output slot i is the input polynomial evaluated at x_i."""
    b = log2_exact(N)
    return [pow(psi, 2 * bitrev(i, b) + 1, q) for i in range(N)]


# ------------------------------------------------------------------ forward

def forward_definition(a: list[int], q: int, psi: int) -> list[int]:
    """O(N^2) merged-twist NTT, bit-reversed output: out[i] = sum_n a_n psi^{n(2 brv(i)+1)}."""
    N = len(a)
    b = log2_exact(N)
    out = []
    for i in range(N):
        k = bitrev(i, b)
        w = pow(psi, 2 * k + 1, q)
        acc = 0
        wn = 1
        for n in range(N):
            acc = (acc + a[n] * wn) % q
            wn = wn * w % q
        out.append(acc)
    return out


def forward_at(a: list[int], q: int, psi: int, i: int) -> int:
    """One output slot of the definition, out[i] = a(psi^{2 brv(i)+1}) (Horner, O(N))."""
    N = len(a)
    x = pow(psi, 2 * bitrev(i, log2_exact(N)) + 1, q)
    acc = 0
    for c in reversed(a):
        acc = (acc * x + int(c)) % q
    return acc


def forward_radix2(a: list[int], q: int, psi: int) -> list[int]:
    """Algorithm 1 (radix-2 Cooley-Tukey), bit-reversed output, taken stage by stage over
    blocks: a stage cuts the vector into blocks of ``span`` slots (span = N, N/2, ..., 2);
    block b pairs each slot of its first half with the slot span/2 above it and applies the
    butterfly of Algorithm 2, (x, y) -> (x + w y, x - w y), with w = Psi[N/span + b], every
    result fully reduced mod q.
    """
    a = [int(x) % q for x in a]
    N = len(a)
    Psi = psi_table(q, psi, N)
    span = N
    while span >= 2:
        half, blocks = span // 2, N // span
        for b in range(blocks):
            w = Psi[blocks + b]
            lo = b * span
            for k in range(lo, lo + half):
                v = a[k + half] * w % q
                a[k + half] = (a[k] - v) % q
                a[k] = (a[k] + v) % q
        span //= 2
    return a


def forward_natural_definition(a: list[int], q: int, psi: int) -> list[int]:
    """O(N^2) merged-twist NTT in natural order (Section III-C's other output order):
    out[k] = A_k = sum_n a_n psi^{n(2k+1)}, the polynomial at the k-th root psi^{2k+1}."""
    N = len(a)
    out = []
    for k in range(N):
        w = pow(psi, 2 * k + 1, q)
        acc = 0
        wn = 1
        for n in range(N):
            acc = (acc + a[n] * wn) % q
            wn = wn * w % q
        out.append(acc)
    return out


# ------------------------------------------------------------------ inverse

def inverse_definition(A: list[int], q: int, psi: int) -> list[int]:
    """O(N^2) inverse of ``forward_definition``: a_n = N^{-1} sum_i A[i] psi^{-n(2 brv(i)+1)}."""
    N = len(A)
    b = log2_exact(N)
    psi_inv = pow(psi, q - 2, q)
    n_inv = pow(N, q - 2, q)
    out = []
    for n in range(N):
        acc = 0
        for i in range(N):
            acc = (acc + A[i] * pow(psi_inv, n * (2 * bitrev(i, b) + 1), q)) % q
        out.append(acc * n_inv % q)
    return out


def inverse_gs(A: list[int], q: int, psi: int) -> list[int]:
    """Gentleman-Sande inverse of Algorithm 1: bit-reversed input, natural-order output.

    The blocks of ``forward_radix2`` visited in the opposite order (span = 2, 4, ..., N);
    block b maps each pair (x, y) to (x + y, (x - y) * Psi_inv[N/span + b]) with
    Psi_inv[i] = psi^{-brv(i)}; every output is finally multiplied by N^{-1}.
    """
    a = [int(x) % q for x in A]
    N = len(a)
    psi_inv = pow(psi, q - 2, q)
    Pinv = psi_table(q, psi_inv, N)
    span = 2
    while span <= N:
        half, blocks = span // 2, N // span
        for b in range(blocks):
            w = Pinv[blocks + b]
            lo = b * span
            for k in range(lo, lo + half):
                x, y = a[k], a[k + half]
                a[k] = (x + y) % q
                a[k + half] = (x - y) * w % q
        span *= 2
    n_inv = pow(N, q - 2, q)
    return [x * n_inv % q for x in a]


# ------------------------------------------------------------------ products

def pointwise(a: list[int], b: list[int], q: int) -> list[int]:
    """Element-wise product mod q (the Hadamard product in the NTT domain)."""
    return [int(x) * int(y) % q for x, y in zip(a, b)]


def negacyclic_schoolbook(a: list[int], b: list[int], q: int) -> list[int]:
    """c_k = sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}  (mod q), O(N^2)."""
    N = len(a)
    c = []
    for k in range(N):
        s = 0
        for i in range(k + 1):
            s += int(a[i]) * int(b[k - i])
        for i in range(k + 1, N):
            s -= int(a[i]) * int(b[N + k - i])
        c.append(s % q)
    return c


def polymul_ntt(a: list[int], b: list[int], q: int, psi: int) -> list[int]:
    """c = iNTT(NTT(a) * NTT(b)) with both twists merged (Section III-A)."""
    return inverse_gs(pointwise(forward_radix2(a, q, psi), forward_radix2(b, q, psi), q), q, psi)


# ------------------------------------------------------------------ residue number system

def rns_decompose(x: int, primes) -> list[int]:
    """Residues of the integer x modulo each prime (Section III-B's RNS form)."""
    return [int(x) % int(q) for q in primes]


def crt_reconstruct(residues, primes) -> int:
    """The unique x in [0, Q) with x = r_l mod q_l for every l (Chinese remainder theorem):
    x = sum_l r_l * M_l * (M_l^{-1} mod q_l) mod Q, M_l = Q / q_l."""
    Q = 1
    for q in primes:
        Q *= int(q)
    acc = 0
    for r, q in zip(residues, primes):
        q = int(q)
        M = Q // q
        acc += int(r) * M * pow(M % q, q - 2, q)
    return acc % Q
