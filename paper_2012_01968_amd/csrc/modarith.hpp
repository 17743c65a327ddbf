// Device modular arithmetic for 64-bit NTT-friendly primes on gfx950.
//
// Shoup's modular multiplication (Algorithm 4 of the paper): with the companion
// wb = floor(w * 2^64 / q) precomputed for a fixed operand w < q, the quotient
// estimate qh = floor(b * wb / 2^64) is within one of floor(b * w / q) for any
// b < 2^64, so r = b*w - qh*q lies in [0, 2q) and only the low 64 bits of the two
// products are needed.  The paper's listing writes the quotient step with a garbled
// shift and tests `r > p`; the reading here is the high half of the 128-bit product
// and a lazy result (the final reduction to [0, q) happens once, at the end of a
// transform).  Butterflies keep their values in lazy ranges in the manner of Harvey,
// whom the paper cites for Algorithm 2's [0, 4p) input bound.
//
// Two arithmetic policies, chosen per plan from the largest prime:
//
//  Arith<false>  any q < 2^62.  Exact quotient; Cooley-Tukey values in [0, 4q),
//                Gentleman-Sande values in [0, 2q) (Harvey's bounds).
//  Arith<true>   q < 2^60.  The quotient is estimated from the three high partial
//                products only, b1*wb1 + hi(b0*wb1) + hi(b1*wb0): the dropped terms sum
//                to less than 3 * 2^64, so the estimate undershoots the exact one by at
//                most 2 and r lies in [0, 4q).  The low half is formed as
//                b*w + qh*(2^64 - q) mod 2^64 with the four cross products folded into
//                the high word.  Gentleman-Sande values live in [0, 4q).  Cooley-Tukey
//                values live in [0, 16q) (16q < 2^64): X is reduced by 8q only in every
//                other stage, so a reducing stage maps inputs below 16q to outputs below
//                12q and the plain stage after it maps those to outputs below 16q.  Every
//                conditional subtraction has |x - m| < 8q < 2^63, so it can test the
//                sign of x - m instead of comparing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

struct Tw {  // a twiddle and its Shoup companion, stored as one 16-byte entry
  uint64_t w, wb;
};

// Integer estimate of k = floor(x / q) for x < 16q (the forward final reduction), with
// s = bitlen(q) >= 3: t = floor(x / 2^(s-3)) < 2^7 and m = floor(2^(s+6) / q) <= 2^7, so
// t * m < 2^14 fits a 24-bit multiply, and est = floor(t * m / 2^9) is k or k - 1.
//   est <= t 2^(s-3) / q <= x / q, so est <= k;
//   x/q - est < (x - t 2^(s-3))/q + t (2^(s-3)/q - m/2^9) + 1 < 1/4 + 1/4 + 1, so est >= k - 1.
// The two per-prime constants are packed as m | (s - 3) << 32.
__host__ inline uint64_t quot_estimate_consts(uint64_t q) {
  uint32_t s = 0;
  while (s < 64 && (q >> s)) ++s;
  const uint64_t m = (uint64_t)(((unsigned __int128)1 << (s + 6)) / q);
  return m | ((uint64_t)(s - 3) << 32);
}

struct Mod {  // per-prime constants
  uint64_t q, q2, q4, q8, nq, nq2, nq4, nq8;  // q, 2q, 4q, 8q, and the negatives mod 2^64 of q, 2q, 4q, 8q
  uint32_t qm, qsh;                       // quotient-estimate multiplier and shift (quot_estimate_consts)
  Mod() = default;
  // From a per-prime constant row {q, 2q, 4q, -q, -2q, -4q, -8q, c} (negatives mod 2^64), c
  // = quot_estimate_consts(q).
  template <typename Ptr>
  static __device__ __forceinline__ Mod load(Ptr c) {
    Mod m;
    m.q = c[0];
    m.q2 = c[1];
    m.q4 = c[2];
    m.q8 = m.q4 + m.q4;
    m.nq = c[3];
    m.nq2 = c[4];
    m.nq4 = c[5];
    m.nq8 = c[6];
    const uint64_t f = c[7];
    m.qm = (uint32_t)f;
    m.qsh = (uint32_t)(f >> 32);
    return m;
  }
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

__device__ __forceinline__ uint64_t make_u64(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(uint64_t, (uint2{lo, hi}));
}

// a + b on 32 bits.  Written as one instruction so that the compiler keeps the high word
// of a 64-bit result as a separate 32-bit add instead of widening it into a 64-bit add
// (which costs a register move to zero-extend the operand).
__device__ __forceinline__ uint32_t add_u32(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// x - m when x >= m, else x; needs |x - m| < 2^63 (negm = 2^64 - m), so the sign of x - m
// decides.  Written as a plain conditional: a 64-bit sign test and two conditional moves, as
// many instructions as the mask-and-bit-field-select form (v_bfi_b32) it replaces.  With that
// form (issued from inline asm, or kept by an empty asm statement on the mask) the key-product
// row pass of 128-point rows with 4 values per lane and one OT stage computed wrong products
// at N1 >= 256; with this one it is exact, like every other kernel.
__device__ __forceinline__ uint64_t csub_sign(uint64_t x, uint64_t negm) {
  const uint64_t d = x + negm;
  return (int64_t)d < 0 ? x : d;
}

template <bool FAST>
struct Arith;

template <>
struct Arith<false> {
  // b * w mod q in [0, 2q), any b < 2^64.
  static __device__ __forceinline__ uint64_t mul(uint64_t b, const Tw& t, const Mod& m) {
    const uint64_t qh = mulhi64(b, t.wb);
    return b * t.w - qh * m.q;
  }
  // Cooley-Tukey: X, Y in [0, 4q) -> X + WY, X - WY in [0, 4q).
  static __device__ __forceinline__ void ct(uint64_t& X, uint64_t& Y, const Tw& t, const Mod& m) {
    const uint64_t x = csub(X, m.q2);
    const uint64_t v = mul(Y, t, m);
    X = x + v;
    Y = x - v + m.q2;
  }
  // Same with the twiddle applied as two factors (on-the-fly twiddling, Section VII).
  static __device__ __forceinline__ void ct2(uint64_t& X, uint64_t& Y, const Tw& a, const Tw& b, const Mod& m) {
    const uint64_t x = csub(X, m.q2);
    const uint64_t v = mul(mul(Y, a, m), b, m);
    X = x + v;
    Y = x - v + m.q2;
  }
  // Gentleman-Sande: X, Y in [0, 2q) -> X + Y, (X - Y) W in [0, 2q).
  static __device__ __forceinline__ void gs(uint64_t& X, uint64_t& Y, const Tw& t, const Mod& m) {
    const uint64_t s = csub(X + Y, m.q2);
    const uint64_t d = X - Y + m.q2;
    X = s;
    Y = mul(d, t, m);
  }
  static __device__ __forceinline__ void gs2(uint64_t& X, uint64_t& Y, const Tw& a, const Tw& b, const Mod& m) {
    const uint64_t s = csub(X + Y, m.q2);
    const uint64_t d = X - Y + m.q2;
    X = s;
    Y = mul(mul(d, a, m), b, m);
  }
  // Last inverse stage with the 1/N scale: X' = (X + Y)/N, Y' = (X - Y) W/N, in [0, 2q).
  static __device__ __forceinline__ void gs_scaled(uint64_t& X, uint64_t& Y, const Tw& wn, const Tw& n,
                                                   const Mod& m) {
    const uint64_t s = X + Y;
    const uint64_t d = X - Y + m.q2;
    X = mul(s, n, m);
    Y = mul(d, wn, m);
  }
  static __device__ __forceinline__ uint64_t fwd_final(uint64_t x, const Mod& m) { return csub(csub(x, m.q2), m.q); }
  static __device__ __forceinline__ uint64_t inv_final(uint64_t x, const Mod& m) { return csub(x, m.q); }
  template <int NB>
  static __device__ __forceinline__ void mul_n(uint64_t (&r)[NB], const uint64_t (&b)[NB], const Tw (&t)[NB],
                                               const Mod& m) {
#pragma unroll
    for (int k = 0; k < NB; ++k) r[k] = mul(b[k], t[k], m);
  }
};

template <>
struct Arith<true> {
  // b * w mod q in [0, 4q), any b < 2^64 (q < 2^60).
  static __device__ __forceinline__ uint64_t mul(uint64_t b, const Tw& t, const Mod& m) {
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint32_t w0 = (uint32_t)t.w, w1 = (uint32_t)(t.w >> 32);
    const uint32_t s0 = (uint32_t)t.wb, s1 = (uint32_t)(t.wb >> 32);
    const uint32_t n0 = (uint32_t)m.nq, n1 = (uint32_t)(m.nq >> 32);
    const uint32_t h1 = __umulhi(b0, s1), h2 = __umulhi(b1, s0);
    const uint64_t qh = (uint64_t)b1 * s1 + ((uint64_t)h1 + h2);
    const uint32_t c0 = (uint32_t)qh, c1 = (uint32_t)(qh >> 32);
    const uint64_t lo = (uint64_t)b0 * w0 + (uint64_t)c0 * n0;
    const uint32_t cross = b0 * w1 + b1 * w0 + c0 * n1 + c1 * n0;
    return make_u64((uint32_t)lo, add_u32((uint32_t)(lo >> 32), cross));
  }

  // NB independent products b[k] * t[k] mod q, written phase by phase so that the
  // multiply chains of different butterflies sit next to each other for the scheduler.
  template <int NB>
  static __device__ __forceinline__ void mul_n(uint64_t (&r)[NB], const uint64_t (&b)[NB], const Tw (&t)[NB],
                                               const Mod& m) {
    const uint32_t n0 = (uint32_t)m.nq, n1 = (uint32_t)(m.nq >> 32);
    uint32_t h1[NB], h2[NB];
    uint64_t qh[NB], lo[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) h1[k] = __umulhi((uint32_t)b[k], (uint32_t)(t[k].wb >> 32));
#pragma unroll
    for (int k = 0; k < NB; ++k) h2[k] = __umulhi((uint32_t)(b[k] >> 32), (uint32_t)t[k].wb);
#pragma unroll
    for (int k = 0; k < NB; ++k)
      qh[k] = (uint64_t)(uint32_t)(b[k] >> 32) * (uint32_t)(t[k].wb >> 32) + ((uint64_t)h1[k] + h2[k]);
#pragma unroll
    for (int k = 0; k < NB; ++k) lo[k] = (uint64_t)(uint32_t)b[k] * (uint32_t)t[k].w + (uint64_t)(uint32_t)qh[k] * n0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const uint32_t b0 = (uint32_t)b[k], b1 = (uint32_t)(b[k] >> 32);
      const uint32_t cross = b0 * (uint32_t)(t[k].w >> 32) + b1 * (uint32_t)t[k].w + (uint32_t)qh[k] * n1 +
                             (uint32_t)(qh[k] >> 32) * n0;
      r[k] = make_u64((uint32_t)lo[k], add_u32((uint32_t)(lo[k] >> 32), cross));
    }
  }
  // The kernels run this policy's butterflies stage by stage over all R/2 pairs of a lane
  // (ct_step, gs_step in passes.hpp, on top of mul_n); the single-butterfly forms below
  // keep the same ranges.
  // Cooley-Tukey: X, Y in [0, 16q) -> X + WY, X - WY in [0, 12q).
  static __device__ __forceinline__ void ct(uint64_t& X, uint64_t& Y, const Tw& t, const Mod& m) {
    const uint64_t x = csub_sign(X, m.nq8);
    const uint64_t v = mul(Y, t, m);
    X = x + v;
    Y = x + m.q4 - v;
  }
  static __device__ __forceinline__ void ct2(uint64_t& X, uint64_t& Y, const Tw& a, const Tw& b, const Mod& m) {
    const uint64_t x = csub_sign(X, m.nq8);
    const uint64_t v = mul(mul(Y, a, m), b, m);
    X = x + v;
    Y = x + m.q4 - v;
  }
  // Gentleman-Sande: X, Y in [0, 8q) -> X + Y in [0, 8q), (X - Y) W in [0, 4q).  (gs_step
  // tracks tighter bounds per register and skips reductions these forms always make.)
  static __device__ __forceinline__ void gs(uint64_t& X, uint64_t& Y, const Tw& t, const Mod& m) {
    const uint64_t s = csub_sign(X + Y, m.nq8);
    const uint64_t d = X + m.q8 - Y;
    X = s;
    Y = mul(d, t, m);
  }
  static __device__ __forceinline__ void gs2(uint64_t& X, uint64_t& Y, const Tw& a, const Tw& b, const Mod& m) {
    const uint64_t s = csub_sign(X + Y, m.nq8);
    const uint64_t d = X + m.q8 - Y;
    X = s;
    Y = mul(mul(d, a, m), b, m);
  }
  // Stage 0 of the whole inverse, with the 1/N scale: X, Y in [0, 8q) -> [0, 4q).
  static __device__ __forceinline__ void gs_scaled(uint64_t& X, uint64_t& Y, const Tw& wn, const Tw& n,
                                                   const Mod& m) {
    const uint64_t s = X + Y;
    const uint64_t d = X + m.q8 - Y;
    X = mul(s, n, m);
    Y = mul(d, wn, m);
  }
  // [0, 16q) -> [0, q).  k = floor(x / q) < 16 is estimated from the top bits of x and the
  // per-prime multiplier (quot_estimate_consts): the estimate is k or k - 1, so x - est * q
  // lies in [0, 2q) and one conditional subtraction finishes (four before).
  static __device__ __forceinline__ uint64_t fwd_final(uint64_t x, const Mod& m) {
    const uint32_t t = (uint32_t)(x >> m.qsh);
    const uint32_t k = __umul24(t, m.qm) >> 9;
    return csub_sign(x + (uint64_t)k * m.nq, m.nq);
  }
  static __device__ __forceinline__ uint64_t inv_final(uint64_t x, const Mod& m) {
    return csub_sign(csub_sign(x, m.nq2), m.nq);
  }
};

// General a * b mod q for a, b < q < 2^62 (no precomputed companion): Barrett
// reduction with s = bitlen(q), mu = floor(2^(2s) / q) < 2^(s+1).
// x = a*b < 2^(2s); x1 = floor(x / 2^(s-1)); qh = floor(x1 * mu / 2^(s+1)) undershoots
// floor(x / q) by at most 2, so r = x - qh*q < 3q and two conditional subtractions
// finish the reduction.
__device__ __forceinline__ uint64_t mulmod_barrett(uint64_t a, uint64_t b, uint64_t q, uint64_t mu, uint32_t s) {
  const uint64_t lo = a * b;
  const uint64_t hi = mulhi64(a, b);
  const uint64_t x1 = (lo >> (s - 1)) | (hi << (65 - s));   // s >= 2; s - 1 >= 1 so both shifts are < 64
  const uint64_t plo = x1 * mu;
  const uint64_t phi = mulhi64(x1, mu);
  const uint64_t qh = (plo >> (s + 1)) | (phi << (63 - s));  // s <= 62: 63 - s >= 1
  uint64_t r = lo - qh * q;
  r = csub(r, q);
  r = csub(r, q);
  return r;
}

}  // namespace nttk
