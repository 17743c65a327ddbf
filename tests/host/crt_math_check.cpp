// Host check of the RNS conversion tables (compiled with g++ by the test suite), for random
// sets of 2..64 primes of 30 to 62 bits (odd numbers suffice: only coprimality and the
// table identities matter here, and distinct primes are drawn):
//   * Q is the product of the primes, with no leading zero word;
//   * M_l * q_l = Q and inv_l * (M_l mod q_l) = 1 mod q_l;
//   * kQ[k] = k * Q for k = 0..L;
//   * pow2[l][w] = 2^(64 w) mod q_l, by repeated doubling with __int128.
#include <cstdio>
#include <random>
#include <set>

#include "crt_math.hpp"

using namespace nttc;

static long failures = 0;
static void check(bool ok, const char* what) {
  if (!ok && failures++ < 20) std::printf("FAIL %s\n", what);
}

static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    uint64_t x = powmod_u128(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = mulmod_u128(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static bool equal_words(const std::vector<uint64_t>& a, const uint64_t* b, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if ((i < a.size() ? a[i] : 0) != b[i]) return false;
  for (size_t i = n; i < a.size(); ++i)
    if (a[i]) return false;
  return true;
}

int main() {
  std::mt19937_64 g(2012);
  for (int trial = 0; trial < 200; ++trial) {
    const int L = 2 + (int)(g() % 63);
    std::set<uint64_t> ps;
    while ((int)ps.size() < L) {
      const int bits = 30 + (int)(g() % 33);
      uint64_t c = (g() >> (64 - bits)) | (1ull << (bits - 1)) | 1;
      if (is_prime(c)) ps.insert(c);
    }
    const std::vector<uint64_t> primes(ps.begin(), ps.end());
    const CrtTables t = crt_tables(primes);
    std::vector<uint64_t> Q = {1};
    for (uint64_t q : primes) mp_mul_small(Q, q);
    check(equal_words(Q, t.Q.data(), t.W), "Q is the product");
    check(t.Q.back() != 0 || t.W == 1, "no leading zero word");
    for (uint32_t l = 0; l < t.L; ++l) {
      const uint64_t q = primes[l];
      std::vector<uint64_t> m(t.M.begin() + (size_t)l * t.W, t.M.begin() + (size_t)(l + 1) * t.W);
      mp_mul_small(m, q);
      check(equal_words(m, t.Q.data(), t.W), "M_l * q_l = Q");
      std::vector<uint64_t> tmp;
      const uint64_t mm = mp_divmod_small(std::vector<uint64_t>(t.M.begin() + (size_t)l * t.W,
                                                                 t.M.begin() + (size_t)(l + 1) * t.W),
                                          q, tmp);
      check(mulmod_u128(mm, t.inv[l], q) == 1, "inverse of M_l mod q_l");
      uint64_t c = 1 % q;
      for (uint32_t w = 0; w < kCrtMaxInWords; ++w) {
        check(t.pow2[(size_t)l * kCrtMaxInWords + w] == c, "2^(64w) mod q");
        for (int b = 0; b < 64; ++b) c = (uint64_t)(((u128)c * 2) % q);
      }
    }
    for (uint32_t k = 0; k <= t.L; ++k) {
      std::vector<uint64_t> kq = Q;
      mp_mul_small(kq, k);
      check(equal_words(kq, &t.kQ[(size_t)k * (t.W + 1)], t.W + 1), "kQ = k * Q");
    }
  }
  std::printf("%ld failures\n", failures);
  return failures != 0;
}
