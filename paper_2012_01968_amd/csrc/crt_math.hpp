// Tables of the RNS <-> integer conversion (Section III-B), computed on the host with plain
// multi-precision arithmetic over little-endian 64-bit words.  Host only: no device code,
// so the host test suite compiles it with g++.
//
// For primes q_0 .. q_{L-1} with product Q (W words):
//   pow2[l][w] = 2^(64 w) mod q_l            (w < kCrtMaxInWords)  integer -> residues
//   inv[l]     = (Q / q_l)^-1 mod q_l                              residues -> integer
//   M[l]       = Q / q_l, W words
//   kQ[k]      = k * Q, W + 1 words, k = 0 .. L
// Reconstruction forms x' = sum_l y_l M_l with y_l = r_l inv[l] mod q_l (so x' < L Q and
// x' = x mod Q), finds the largest k with kQ <= x' and subtracts it.
#pragma once
#include <cstdint>
#include <vector>

namespace nttc {

typedef unsigned __int128 u128;
constexpr uint32_t kCrtMaxInWords = 64;   // widest integer ntt_rns_decompose accepts

// a *= m (a grows by a word when needed)
inline void mp_mul_small(std::vector<uint64_t>& a, uint64_t m) {
  uint64_t carry = 0;
  for (uint64_t& w : a) {
    const u128 t = (u128)w * m + carry;
    w = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
  if (carry) a.push_back(carry);
}

// quotient of a / d (same length as a), remainder returned
inline uint64_t mp_divmod_small(const std::vector<uint64_t>& a, uint64_t d, std::vector<uint64_t>& quot) {
  quot.assign(a.size(), 0);
  u128 rem = 0;
  for (size_t i = a.size(); i-- > 0;) {
    const u128 cur = (rem << 64) | a[i];
    quot[i] = (uint64_t)(cur / d);
    rem = cur % d;
  }
  return (uint64_t)rem;
}

inline uint64_t mulmod_u128(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

inline uint64_t powmod_u128(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod_u128(r, b, q);
    b = mulmod_u128(b, b, q);
    e >>= 1;
  }
  return r;
}

struct CrtTables {
  uint32_t L = 0, W = 0;                 // primes, words of Q
  std::vector<uint64_t> Q;               // W words
  std::vector<uint64_t> pow2;            // [L][kCrtMaxInWords]
  std::vector<uint64_t> inv;             // [L]
  std::vector<uint64_t> M;               // [L][W]
  std::vector<uint64_t> kQ;              // [L + 1][W + 1]
};

inline CrtTables crt_tables(const std::vector<uint64_t>& primes) {
  CrtTables t;
  t.L = (uint32_t)primes.size();
  t.Q = {1};
  for (uint64_t q : primes) mp_mul_small(t.Q, q);
  while (t.Q.size() > 1 && t.Q.back() == 0) t.Q.pop_back();
  t.W = (uint32_t)t.Q.size();
  t.pow2.assign((size_t)t.L * kCrtMaxInWords, 0);
  t.inv.assign(t.L, 0);
  t.M.assign((size_t)t.L * t.W, 0);
  t.kQ.assign((size_t)(t.L + 1) * (t.W + 1), 0);
  std::vector<uint64_t> quot;
  for (uint32_t l = 0; l < t.L; ++l) {
    const uint64_t q = primes[l];
    const uint64_t two64 = (uint64_t)(((u128)1 << 64) % q);
    uint64_t c = 1 % q;
    for (uint32_t w = 0; w < kCrtMaxInWords; ++w) {
      t.pow2[(size_t)l * kCrtMaxInWords + w] = c;
      c = mulmod_u128(c, two64, q);
    }
    const uint64_t rem = mp_divmod_small(t.Q, q, quot);
    (void)rem;   // zero: q divides Q
    for (uint32_t w = 0; w < t.W; ++w) t.M[(size_t)l * t.W + w] = quot[w];
    std::vector<uint64_t> tmp;
    const uint64_t m_mod_q = mp_divmod_small(quot, q, tmp);
    t.inv[l] = powmod_u128(m_mod_q, q - 2, q);
  }
  for (uint32_t k = 0; k <= t.L; ++k) {
    std::vector<uint64_t> kq = t.Q;
    mp_mul_small(kq, k);
    for (uint32_t w = 0; w < t.W + 1 && w < kq.size(); ++w) t.kQ[(size_t)k * (t.W + 1) + w] = kq[w];
  }
  return t;
}

}  // namespace nttc
