/*
 * Plain C reference for the negacyclic NTT path.  TEST INFRASTRUCTURE ONLY: the
 * library never links or calls this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no header, table or helper with
 * the HIP path.
 *
 * Arithmetic is the obvious kind: every product is reduced with
 * (unsigned __int128)a*b % q, every sum and difference is fully reduced, and no
 * lazy range, Shoup companion or on-the-fly twiddle is used.
 *
 * Paper: Kim, Jung, Park, Ahn, arXiv 2012.01968.
 *   forward   -- Algorithm 1 (radix-2 Cooley-Tukey over Psi[i] = psi^{brv(i)}) with
 *                the butterfly of Algorithm 2; output in bit-reversed order.
 *   inverse   -- Gentleman-Sande mirror of Algorithm 1 with Psi_inv[i] = psi^{-brv(i)}
 *                and the final 1/N scale (the merged inverse of Section III-A).
 *   forward_at-- one output slot of the definition in Section III-A:
 *                out[i] = sum_n a_n psi^{n(2 brv(i)+1)}, evaluated by Horner's rule.
 *   schoolbook-- the negacyclic convolution formula of Section III-A.
 *
 * Batch layout: n_vec vectors of N residues stored back to back; vector v of a call
 * uses prime index (vec_offset + v) mod L, which is the [poly][limb][coefficient]
 * layout when a call starts at a vector boundary.
 */
#include <stdint.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { u128 s = (u128)a + b; return (uint64_t)(s % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : (uint64_t)((u128)a + q - b); }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

static uint32_t bitrev32(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1u); x >>= 1; }
    return r;
}

static int log2u(uint32_t n) { int b = 0; while ((1u << b) < n) ++b; return b; }

/* table[i] = root^{brv(i)}, built from the plain power sequence root^0, root^1, ... */
static int build_brv_table(uint64_t* table, uint32_t N, uint64_t q, uint64_t root) {
    uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * N);
    if (!pw) return -1;
    int bits = log2u(N);
    pw[0] = 1 % q;
    for (uint32_t e = 1; e < N; ++e) pw[e] = mulmod(pw[e - 1], root, q);
    for (uint32_t i = 0; i < N; ++i) table[i] = pw[bitrev32(i, bits)];
    free(pw);
    return 0;
}

/* Algorithm 1 taken stage by stage over blocks: a stage cuts the vector into blocks of
 * `span` slots (span = N, N/2, ..., 2).  Block b, starting at slot b*span, pairs each slot
 * of its first half with the slot span/2 above it and uses the twiddle Psi[N/span + b]:
 * the Cooley-Tukey butterfly of Algorithm 2, (x, y) -> (x + w y, x - w y), fully reduced. */
static void forward_one(uint64_t* a, uint32_t N, uint64_t q, const uint64_t* Psi) {
    for (uint32_t span = N; span >= 2; span /= 2) {
        const uint32_t half = span / 2, blocks = N / span;
        for (uint32_t b = 0; b < blocks; ++b) {
            const uint64_t w = Psi[blocks + b];
            uint64_t* lo = a + (uint64_t)b * span;
            uint64_t* hi = lo + half;
            for (uint32_t k = 0; k < half; ++k) {
                const uint64_t v = mulmod(hi[k], w, q);
                hi[k] = submod(lo[k], v, q);
                lo[k] = addmod(lo[k], v, q);
            }
        }
    }
}

/* The Gentleman-Sande inverse: the same blocks visited from span 2 up to span N, each
 * butterfly (x, y) -> (x + y, (x - y) w) with w = Psi_inv[N/span + b], then every slot times
 * N^{-1}. */
static void inverse_one(uint64_t* a, uint32_t N, uint64_t q, const uint64_t* Pinv, uint64_t n_inv) {
    for (uint32_t span = 2; span <= N; span *= 2) {
        const uint32_t half = span / 2, blocks = N / span;
        for (uint32_t b = 0; b < blocks; ++b) {
            const uint64_t w = Pinv[blocks + b];
            uint64_t* lo = a + (uint64_t)b * span;
            uint64_t* hi = lo + half;
            for (uint32_t k = 0; k < half; ++k) {
                const uint64_t x = lo[k], y = hi[k];
                lo[k] = addmod(x, y, q);
                hi[k] = mulmod(submod(x, y, q), w, q);
            }
        }
    }
    for (uint32_t i = 0; i < N; ++i) a[i] = mulmod(a[i], n_inv, q);
}

/* In-place forward transform of n_vec vectors.  Returns 0, or -1 on allocation failure. */
int oracle_forward(uint64_t* data, uint64_t n_vec, uint32_t N, const uint64_t* q, const uint64_t* psi,
                   uint32_t L, uint64_t vec_offset) {
    uint64_t* Psi = (uint64_t*)malloc(sizeof(uint64_t) * N);
    if (!Psi) return -1;
    int64_t last = -1;
    for (uint64_t v = 0; v < n_vec; ++v) {
        uint32_t l = (uint32_t)((vec_offset + v) % L);
        if ((int64_t)l != last) {
            if (build_brv_table(Psi, N, q[l], psi[l])) { free(Psi); return -1; }
            last = l;
        }
        forward_one(data + v * (uint64_t)N, N, q[l], Psi);
    }
    free(Psi);
    return 0;
}

int oracle_inverse(uint64_t* data, uint64_t n_vec, uint32_t N, const uint64_t* q, const uint64_t* psi,
                   uint32_t L, uint64_t vec_offset) {
    uint64_t* Pinv = (uint64_t*)malloc(sizeof(uint64_t) * N);
    if (!Pinv) return -1;
    int64_t last = -1;
    uint64_t n_inv = 0;
    for (uint64_t v = 0; v < n_vec; ++v) {
        uint32_t l = (uint32_t)((vec_offset + v) % L);
        if ((int64_t)l != last) {
            uint64_t psi_inv = powmod(psi[l], q[l] - 2, q[l]);
            if (build_brv_table(Pinv, N, q[l], psi_inv)) { free(Pinv); return -1; }
            n_inv = powmod(N % q[l], q[l] - 2, q[l]);
            last = l;
        }
        inverse_one(data + v * (uint64_t)N, N, q[l], Pinv, n_inv);
    }
    free(Pinv);
    return 0;
}

/* out[i] of the definition for one vector: a evaluated at psi^{2 brv(i) + 1}. */
uint64_t oracle_forward_at(const uint64_t* a, uint32_t N, uint64_t q, uint64_t psi, uint32_t i) {
    uint64_t x = powmod(psi, 2 * (uint64_t)bitrev32(i, log2u(N)) + 1, q);
    uint64_t acc = 0;
    for (int64_t n = (int64_t)N - 1; n >= 0; --n) acc = addmod(mulmod(acc, x, q), a[n] % q, q);
    return acc;
}

/* Coefficient n of the inverse definition: N^{-1} sum_i A[i] psi^{-n(2 brv(i)+1)}. */
uint64_t oracle_inverse_at(const uint64_t* A, uint32_t N, uint64_t q, uint64_t psi, uint32_t n) {
    uint64_t psi_inv = powmod(psi, q - 2, q);
    int bits = log2u(N);
    uint64_t acc = 0;
    for (uint32_t i = 0; i < N; ++i) {
        uint64_t e = ((uint64_t)n * (2 * (uint64_t)bitrev32(i, bits) + 1)) % (2 * (uint64_t)N);
        acc = addmod(acc, mulmod(A[i] % q, powmod(psi_inv, e, q), q), q);
    }
    return mulmod(acc, powmod(N % q, q - 2, q), q);
}

void oracle_pointwise(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n_vec, uint32_t N,
                      const uint64_t* q, uint32_t L, uint64_t vec_offset) {
    for (uint64_t v = 0; v < n_vec; ++v) {
        uint64_t qq = q[(vec_offset + v) % L];
        for (uint32_t i = 0; i < N; ++i) {
            uint64_t k = v * (uint64_t)N + i;
            c[k] = mulmod(a[k] % qq, b[k] % qq, qq);
        }
    }
}

/* c_k = sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}  (mod q), one vector. */
void oracle_negacyclic_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q) {
    for (uint32_t k = 0; k < N; ++k) {
        uint64_t s = 0;
        for (uint32_t i = 0; i <= k; ++i) s = addmod(s, mulmod(a[i] % q, b[k - i] % q, q), q);
        for (uint32_t i = k + 1; i < N; ++i) s = submod(s, mulmod(a[i] % q, b[N + k - i] % q, q), q);
        c[k] = s;
    }
}

uint64_t oracle_powmod(uint64_t b, uint64_t e, uint64_t q) { return powmod(b, e, q); }
