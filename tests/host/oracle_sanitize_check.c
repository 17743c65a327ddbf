/* Host sanitizer run of the C oracle (compiled together with oracle/ntt_oracle.c under
 * -fsanitize=address,undefined by the test suite): every entry point on small sizes, with
 * results checked against each other (forward at a slot = the full forward's slot, inverse
 * undoes forward, the NTT-based product equals the schoolbook one).  Primes q = 1 mod 2N are
 * found by trial division and psi by search, so nothing here comes from the GPU library. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_forward(uint64_t* data, uint64_t n_vec, uint32_t N, const uint64_t* q, const uint64_t* psi, uint32_t L,
                   uint64_t vec_offset);
int oracle_inverse(uint64_t* data, uint64_t n_vec, uint32_t N, const uint64_t* q, const uint64_t* psi, uint32_t L,
                   uint64_t vec_offset);
uint64_t oracle_forward_at(const uint64_t* a, uint32_t N, uint64_t q, uint64_t psi, uint32_t i);
uint64_t oracle_inverse_at(const uint64_t* A, uint32_t N, uint64_t q, uint64_t psi, uint32_t n);
void oracle_pointwise(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n_vec, uint32_t N,
                      const uint64_t* q, uint32_t L, uint64_t vec_offset);
void oracle_negacyclic_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q);
uint64_t oracle_powmod(uint64_t b, uint64_t e, uint64_t q);

static long failures = 0;
static void check(int ok, const char* what, uint32_t N) {
    if (!ok && failures++ < 20) printf("FAIL %s (N=%u)\n", what, N);
}

static int is_prime_td(uint64_t n) {
    if (n < 2) return 0;
    for (uint64_t d = 2; d * d <= n; ++d)
        if (n % d == 0) return 0;
    return 1;
}

/* a primitive 2N-th root of unity: x^((q-1)/2N) whose N-th power is q - 1 */
static uint64_t find_root(uint64_t q, uint32_t N) {
    for (uint64_t x = 2; x < q; ++x) {
        uint64_t y = oracle_powmod(x, (q - 1) / (2 * (uint64_t)N), q);
        if (oracle_powmod(y, N, q) == q - 1) return y;
    }
    return 0;
}

static uint64_t rng = 0x243F6A8885A308D3ull;
static uint64_t next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

int main(void) {
    for (uint32_t N = 2; N <= 256; N *= 2) {
        const uint32_t L = 2;
        uint64_t q[2], psi[2];
        uint64_t c = ((1ull << 40) / (2 * N)) * 2 * N + 1;
        for (uint32_t l = 0; l < L; c += 2 * N) {
            if (!is_prime_td(c)) continue;
            q[l] = c;
            psi[l] = find_root(c, N);
            ++l;
        }
        const uint64_t n_vec = 2 * L;
        const size_t n = (size_t)n_vec * N;
        uint64_t *a = malloc(n * 8), *b = malloc(n * 8), *f = malloc(n * 8), *g = malloc(n * 8), *m = malloc(n * 8),
                 *s = malloc(n * 8);
        for (size_t k = 0; k < n; ++k) {
            a[k] = next() % q[(k / N) % L];
            b[k] = next() % q[(k / N) % L];
        }
        memcpy(f, a, n * 8);
        check(oracle_forward(f, n_vec, N, q, psi, L, 0) == 0, "forward", N);
        for (uint64_t v = 0; v < n_vec; ++v)
            for (uint32_t i = 0; i < N; i += (N > 16 ? 7 : 1))
                check(oracle_forward_at(a + v * N, N, q[v % L], psi[v % L], i) == f[v * N + i], "forward_at", N);
        memcpy(g, f, n * 8);
        check(oracle_inverse(g, n_vec, N, q, psi, L, 0) == 0, "inverse", N);
        check(memcmp(g, a, n * 8) == 0, "inverse(forward)", N);
        for (uint32_t i = 0; i < N; i += (N > 16 ? 5 : 1))
            check(oracle_inverse_at(f, N, q[0], psi[0], i) == a[i], "inverse_at", N);
        memcpy(g, b, n * 8);
        oracle_forward(g, n_vec, N, q, psi, L, 0);
        oracle_pointwise(f, g, m, n_vec, N, q, L, 0);
        oracle_inverse(m, n_vec, N, q, psi, L, 0);
        for (uint64_t v = 0; v < n_vec; ++v) {
            oracle_negacyclic_schoolbook(a + v * N, b + v * N, s + v * N, N, q[v % L]);
            check(memcmp(s + v * N, m + v * N, (size_t)N * 8) == 0, "product = schoolbook", N);
        }
        free(a); free(b); free(f); free(g); free(m); free(s);
    }
    printf("%ld failures\n", failures);
    return failures != 0;
}
