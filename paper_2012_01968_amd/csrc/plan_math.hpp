// Host-side number theory for building a plan: primality, the root convention and the
// twiddle tables with their Shoup companions.  Written independently of any test code.
#pragma once
#include <stdint.h>
#include <vector>

namespace nttp {

using u128 = unsigned __int128;

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }

inline uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit n: the first twelve primes as bases decide
// primality for all n < 3.3e24 (Sorenson and Webster, 2015).
inline bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        witness = false;
        break;
      }
    }
    if (witness) return false;
  }
  return true;
}

// Shoup companion floor(w * 2^64 / q) of a fixed multiplicand w < q (Algorithm 4).
inline uint64_t shoup_companion(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) {
    r = (r << 1) | (x & 1u);
    x >>= 1;
  }
  return r;
}

// Smallest primitive 2N-th root of unity mod q (q prime, q = 1 mod 2N).  A generator
// g of the multiplicative group gives one primitive root g^((q-1)/2N); its odd powers
// are all of them.  Returns 0 if no generator candidate below 2^20 works (cannot
// happen for a prime q = 1 mod 2N, but keeps the search bounded).
inline uint64_t smallest_primitive_root(uint64_t q, uint64_t N) {
  const uint64_t e = (q - 1) / (2 * N);
  uint64_t r0 = 0;
  for (uint64_t g = 2; g < (1u << 20); ++g) {
    const uint64_t y = powmod(g, e, q);
    if (powmod(y, N, q) == q - 1) {
      r0 = y;
      break;
    }
  }
  if (!r0) return 0;
  const uint64_t r2 = mulmod(r0, r0, q);
  uint64_t best = r0, cur = r0;
  for (uint64_t k = 1; k < N; ++k) {
    cur = mulmod(cur, r2, q);
    if (cur < best) best = cur;
  }
  return best;
}

}  // namespace nttp
