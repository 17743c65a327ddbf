// Range claims of the fast arithmetic policy (primes below 2^60), checked on the host with
// unsigned __int128 as the reference.  The product below restates the kernels' formula: the
// Shoup quotient estimated from the three high 32x32 partial products of b * wb, and the
// remainder b*w - qh*q taken modulo 2^64.
//   1. for any b < 2^64 the remainder lies in [0, 4q) and is congruent to b*w mod q;
//   2. Cooley-Tukey butterflies that reduce X by 8q only in even stages keep values below 16q,
//      and every conditional subtraction has |x - m| < 2^63 (the sign test is valid);
//   3. the forward final reduction (8q, 4q, 2q, q) maps [0, 16q) onto [0, q);
//   4. so does the quotient-estimate form: k = floor(x / q) estimated in integers as
//      ((x >> (s - 3)) * floor(2^(s+6) / q)) >> 9 with s = bitlen(q) (a product below 2^14,
//      one 24-bit multiply on the GPU), then x - k*q (in [0, 2q) when the estimate is k or
//      k - 1) and one subtraction of q.  QSHIFT, QEXTRA and QROUNDUP plant mistakes in it
//      (a shift of s - 2, a multiplier scaled by 2^7 instead of 2^6 with the same final
//      shift, a multiplier rounded up); each must make this check fail;
//   5. Gentleman-Sande register steps (8 values, up to 3 stages) with per-register bounds:
//      inputs below IN_B q, a sum reduced by 8q only when its inputs' bound is above 4q, the
//      difference offset by the inputs' bound, products below 4q; every value stays below 8q,
//      and a chain of steps ending in the scaled stage and the final reduction is canonical
//      and congruent to the exact transform's arithmetic.
#include <cstdint>
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

static uint64_t fast_mul(uint64_t b, uint64_t w, uint64_t wb, uint64_t q) {
  const uint64_t b0 = (uint32_t)b, b1 = b >> 32, s0 = (uint32_t)wb, s1 = wb >> 32;
  const uint64_t h1 = (b0 * s1) >> 32, h2 = (b1 * s0) >> 32;
  const uint64_t qh = b1 * s1 + h1 + h2;   // < 2^64: it is at most floor(b * wb / 2^64)
  return b * w - qh * q;                   // modulo 2^64
}

static long failures = 0;
static void fail(const char* what, uint64_t q, uint64_t a, uint64_t b) {
  if (failures++ < 10) std::printf("FAIL %s q=%llu a=%llu b=%llu\n", what, (unsigned long long)q,
                                   (unsigned long long)a, (unsigned long long)b);
}

// conditional subtraction by the sign of x - m; records whether the sign test was valid
static uint64_t csub(uint64_t x, uint64_t m, uint64_t q) {
  const u128 diff = x >= m ? (u128)(x - m) : (u128)(m - x);
  if (diff >= ((u128)1 << 63)) fail("|x - m| >= 2^63", q, x, m);
  const uint64_t d = x - m;
  return (int64_t)d < 0 ? x : d;
}

#ifndef QSHIFT
#define QSHIFT 3
#endif
#ifndef QEXTRA
#define QEXTRA 6
#endif
#ifndef QROUNDUP
#define QROUNDUP 0
#endif

static uint64_t quotient_final(uint64_t x, uint64_t q) {
  uint32_t s = 0;
  while (s < 64 && (q >> s)) ++s;
  const u128 num = (u128)1 << (s + QEXTRA);
  const uint64_t m = (uint64_t)(num / q + (QROUNDUP && num % q ? 1 : 0));
  const uint64_t t = x >> (s - QSHIFT);
  if (t >= 128 || m > 128) fail("quotient estimate operands exceed 2^7", q, x, m);
  const uint32_t k = (uint32_t)((t * m) >> 9);
  if (k > 15) fail("quotient estimate above 15", q, x, k);
  const uint64_t r = x - (uint64_t)k * q;        // modulo 2^64
  if (r >= 2 * q) fail("x - k*q outside [0, 2q)", q, x, k);
  return csub(r, q, q);
}

static void check_quotient_final(uint64_t q, uint64_t x) {
  const uint64_t v = quotient_final(x, q);
  if (v >= q || v != x % q) fail("quotient final reduction", q, x, v);
}

// bound (in q) of register u before local stage i of a step whose inputs lie below in_b q
static int gs_before(int in_b, int i, int u) {
  int b = in_b;
  for (int j = 0; j < i; ++j) b = (u >> j) & 1 ? 4 : (2 * b > 8 ? 8 : 2 * b);
  return b;
}

// one step of nb stages on x[8] (values) and r[8] (their exact residues)
static void gs_register_step(uint64_t* x, uint64_t* r, int in_b, int nb, uint64_t q, std::mt19937_64& g) {
  for (int i = 0; i < nb; ++i) {
    const uint64_t w = g() % q, wb = (uint64_t)(((u128)w << 64) / q);
    for (int u = 0; u < 8; ++u) {
      if (u & (1 << i)) continue;
      const int v = u | (1 << i);
      const int b = gs_before(in_b, i, u);
      if (x[u] >= (uint64_t)b * q || x[v] >= (uint64_t)b * q) fail("GS input above its bound", q, x[u], x[v]);
      const uint64_t sum = x[u] + x[v];
      const uint64_t s = 2 * b > 8 ? csub(sum, 8 * q, q) : sum;
      const uint64_t d = x[u] + (uint64_t)b * q - x[v];
      const uint64_t p = fast_mul(d, w, wb, q);
      if (s >= 8 * q) fail("GS sum >= 8q", q, x[u], x[v]);
      if (p >= 4 * q) fail("GS product >= 4q", q, d, w);
      const uint64_t rs = (r[u] + r[v]) % q, rp = mulmod((r[u] + q - r[v]) % q, w, q);
      if (s % q != rs || p % q != rp) fail("GS not congruent", q, s, p);
      x[u] = s; r[u] = rs; x[v] = p; r[v] = rp;
    }
  }
}

int main() {
  std::mt19937_64 g(2012);
  // claim 5: chains of Gentleman-Sande register steps, inputs pushed to the top of their bounds
  for (int trial = 0; trial < 100000; ++trial) {
    const int bits = 40 + (int)(g() % 21);
    uint64_t q = (g() >> (64 - bits)) | (1ull << (bits - 1)) | 1;
    if (q >= (1ull << 60)) q = (1ull << 60) - 1;
    uint64_t x[8], r[8];
    for (int u = 0; u < 8; ++u) {   // canonical input, half of it at q - 1
      x[u] = (g() & 1) ? q - 1 - (g() & 3) : g() % q;
      r[u] = x[u];
    }
    const int steps = 1 + (int)(g() % 4);
    for (int k = 0; k < steps; ++k) {
      gs_register_step(x, r, k == 0 ? 1 : 8, 1 + (int)(g() % 3), q, g);
      // between steps the values are permuted across registers (the LDS exchange); push some
      // to the top of the next step's input range, keeping them congruent
      for (int u = 7; u > 0; --u) {
        const int v = (int)(g() % (u + 1));
        std::swap(x[u], x[v]);
        std::swap(r[u], r[v]);
      }
      for (int u = 0; u < 8; ++u)
        if (g() % 4 == 0) x[u] = r[u] + q * ((8 * q - 1 - r[u]) / q);   // largest value below 8q
    }
    // the scaled last stage and the final reduction
    const uint64_t n = g() % q, nb = (uint64_t)(((u128)n << 64) / q);
    const uint64_t wn = g() % q, wnb = (uint64_t)(((u128)wn << 64) / q);
    for (int u = 0; u < 8; u += 2) {
      const uint64_t s = x[u] + x[u + 1], d = x[u] + 8 * q - x[u + 1];
      const uint64_t a = fast_mul(s, n, nb, q), b = fast_mul(d, wn, wnb, q);
      if (a >= 4 * q || b >= 4 * q) fail("scaled stage output >= 4q", q, a, b);
      const uint64_t ca = csub(csub(a, 2 * q, q), q, q), cb = csub(csub(b, 2 * q, q), q, q);
      const uint64_t ra = mulmod((r[u] + r[u + 1]) % q, n, q), rb = mulmod((r[u] + q - r[u + 1]) % q, wn, q);
      if (ca != ra || cb != rb) fail("scaled stage / final reduction", q, ca, cb);
    }
  }
  // claim 4 at every multiple of q below 16q (and just around it), for random and extreme q
  {
    // moduli of at least 3 bits: an NTT prime is 1 mod 2N with N >= 2, so q >= 5
    std::vector<uint64_t> qs = {5, 7, (1ull << 31) - 1, (1ull << 32) + 15, (1ull << 59) + 1,
                                (1ull << 59) + 55, (1ull << 60) - 93, (1ull << 60) - 1};
    for (int i = 0; i < 20000; ++i) {
      const int bits = 3 + (int)(g() % 58);   // 3..60-bit odd moduli
      uint64_t q = (g() >> (64 - bits)) | (1ull << (bits - 1)) | 1;
      if (q >= (1ull << 60)) q = (1ull << 60) - 1;
      if (q > 2) qs.push_back(q);
    }
    for (const uint64_t q : qs) {
      for (uint64_t k = 0; k <= 16; ++k) {
        for (int64_t d = -3; d <= 3; ++d) {
          const __int128 x = (__int128)k * q + d;
          if (x >= 0 && x < (__int128)16 * q) check_quotient_final(q, (uint64_t)x);
        }
      }
      for (int j = 0; j < 16; ++j) check_quotient_final(q, g() % (16 * q));
    }
  }
  for (int trial = 0; trial < 300000; ++trial) {
    const int bits = 30 + (int)(g() % 31);   // 30..60-bit odd moduli (primality is irrelevant here)
    uint64_t q = (g() >> (64 - bits)) | (1ull << (bits - 1)) | 1;
    if (q >= (1ull << 60)) q = (1ull << 60) - 1;
    const uint64_t w = g() % q, wb = (uint64_t)(((u128)w << 64) / q);
    uint64_t b;
    switch (trial % 5) {
      case 0: b = g(); break;
      case 1: b = g() % (16 * q); break;
      case 2: b = ~0ull - (g() & 0xffff); break;
      case 3: b = 16 * q - 1 - (g() & 7); break;
      default: b = g() & 0xff;
    }
    const uint64_t r = fast_mul(b, w, wb, q);
    if (r >= 4 * q) fail("product >= 4q", q, b, w);
    if (r % q != mulmod(b % q, w % q, q)) fail("product not congruent", q, b, w);
  }
  // butterfly ranges: run random stage sequences with values pushed to the top of each range
  for (int trial = 0; trial < 20000; ++trial) {
    const int bits = 40 + (int)(g() % 21);
    uint64_t q = (g() >> (64 - bits)) | (1ull << (bits - 1)) | 1;
    if (q >= (1ull << 60)) q = (1ull << 60) - 1;
    uint64_t X = g() % q, Y = g() % q;   // canonical input
    const uint64_t X0 = X, Y0 = Y;
    uint64_t xr = X0 % q, yr = Y0 % q;   // reference residues of the same two values
    const int stages = 1 + (int)(g() % 17);
    for (int s = 0; s < stages; ++s) {
      const uint64_t w = g() % q, wb = (uint64_t)(((u128)w << 64) / q);
      const uint64_t x = (s % 2 == 0) ? csub(X, 8 * q, q) : X;
      const uint64_t t = fast_mul(Y, w, wb, q);
      const uint64_t nx = x + t, ny = x + 4 * q - t;
      if (nx >= 16 * q || ny >= 16 * q) fail("butterfly output >= 16q", q, nx, ny);
      const uint64_t rt = mulmod(yr, w, q);
      const uint64_t rx = (xr + rt) % q, ry = (xr + q - rt) % q;
      if (nx % q != rx || ny % q != ry) fail("butterfly not congruent", q, nx, ny);
      // keep the larger output on the X side so the worst case propagates
      if (g() & 1) { X = nx; Y = ny; xr = rx; yr = ry; } else { X = ny; Y = nx; xr = ry; yr = rx; }
    }
    uint64_t v = X;
    v = csub(v, 8 * q, q); v = csub(v, 4 * q, q); v = csub(v, 2 * q, q); v = csub(v, q, q);
    if (v >= q || v != xr) fail("final reduction", q, X, v);
    if (quotient_final(X, q) != xr) fail("quotient final reduction", q, X, xr);
  }
  std::printf("%ld failures\n", failures);
  return failures != 0;
}
