// Device modular arithmetic for 64-bit NTT-friendly primes q < 2^62 on gfx950.
//
// Shoup's modular multiplication (Algorithm 4 of the paper): with the companion
// wb = floor(w * 2^64 / q) precomputed for a fixed operand w < q, the quotient
// estimate qh = floor(b * wb / 2^64) is within one of floor(b * w / q) for any
// b < 2^64, so r = b*w - qh*q lies in [0, 2q) and only the low 64 bits of the two
// products are needed.  The paper's listing writes the quotient step with a garbled
// shift and tests `r > p`; the reading here is the high half of the 128-bit product
// and a lazy result in [0, 2q) (the final canonicalisation happens once, at the end
// of a transform).
//
// Butterflies follow Harvey's lazy form (the paper's Algorithm 2 takes inputs in
// [0, 4q) and cites Harvey for the bound): the Cooley-Tukey butterfly keeps values in
// [0, 4q), the Gentleman-Sande butterfly in [0, 2q).  Both need 4q < 2^64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

struct Tw {  // a twiddle and its Shoup companion, stored as one 16-byte entry
  uint64_t w, wb;
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// b * w mod q in [0, 2q), any b < 2^64.
__device__ __forceinline__ uint64_t shoup(uint64_t b, uint64_t w, uint64_t wb, uint64_t q) {
  const uint64_t qh = mulhi64(b, wb);
  return b * w - qh * q;
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// Cooley-Tukey butterfly: X, Y in [0, 4q) -> X + WY, X - WY, both in [0, 4q).
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wb, uint64_t q,
                                        uint64_t q2) {
  const uint64_t x = csub(X, q2);
  const uint64_t t = shoup(Y, w, wb, q);
  X = x + t;
  Y = x - t + q2;
}

// Same, with the twiddle applied as two Shoup products (on-the-fly twiddling:
// w = w1 * w2 mod q is never formed, Section VII).
__device__ __forceinline__ void ct_bfly_ot(uint64_t& X, uint64_t& Y, Tw a, Tw b, uint64_t q, uint64_t q2) {
  const uint64_t x = csub(X, q2);
  const uint64_t t = shoup(shoup(Y, a.w, a.wb, q), b.w, b.wb, q);
  X = x + t;
  Y = x - t + q2;
}

// Gentleman-Sande butterfly: X, Y in [0, 2q) -> X + Y, (X - Y) W, both in [0, 2q).
__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wb, uint64_t q,
                                        uint64_t q2) {
  const uint64_t s = csub(X + Y, q2);
  const uint64_t d = X - Y + q2;
  X = s;
  Y = shoup(d, w, wb, q);
}

__device__ __forceinline__ void gs_bfly_ot(uint64_t& X, uint64_t& Y, Tw a, Tw b, uint64_t q, uint64_t q2) {
  const uint64_t s = csub(X + Y, q2);
  const uint64_t d = X - Y + q2;
  X = s;
  Y = shoup(shoup(d, a.w, a.wb, q), b.w, b.wb, q);
}

// Last inverse stage with the 1/N scale folded in: X' = (X + Y)/N, Y' = (X - Y) W/N,
// both in [0, 2q); `n` holds 1/N and `wn` holds W/N, each with its companion.
__device__ __forceinline__ void gs_bfly_scaled(uint64_t& X, uint64_t& Y, Tw wn, Tw n, uint64_t q, uint64_t q2) {
  const uint64_t s = X + Y;
  const uint64_t d = X - Y + q2;
  X = shoup(s, n.w, n.wb, q);
  Y = shoup(d, wn.w, wn.wb, q);
}

// [0, 4q) -> [0, q)
__device__ __forceinline__ uint64_t canon4(uint64_t x, uint64_t q, uint64_t q2) { return csub(csub(x, q2), q); }
// [0, 2q) -> [0, q)
__device__ __forceinline__ uint64_t canon2(uint64_t x, uint64_t q) { return csub(x, q); }

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
