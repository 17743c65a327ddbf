// Queue order of the fused transform (see fused.hpp), shared by the kernel and a host test.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define NTTK_HD __host__ __device__
#else
#define NTTK_HD
#endif

namespace nttk {

// Queue geometry of one XCD.
struct Queue {
  uint32_t n;      // vectors on this XCD
  uint32_t D;      // lag (<= n)
  uint32_t total;  // tiles
};

NTTK_HD inline Queue queue_of(uint32_t x, uint32_t L, uint32_t P, uint32_t lag, uint32_t Tc,
                                          uint32_t Tr) {
  Queue qq;
  const uint32_t nl = L > x ? (L - x + 7) / 8 : 0;
  qq.n = nl * P;
  qq.D = lag < qq.n ? lag : qq.n;
  qq.total = qq.n * (Tc + Tr);
  return qq;
}

// Position p of the queue -> (first pass?, queue vector j, tile).  `A` tiles are those of the
// pass that runs first (columns forward, rows inverse), `B` tiles those that wait.
NTTK_HD inline void decode(const Queue& qq, uint32_t p, uint32_t TA, uint32_t TB, bool& first,
                                       uint32_t& j, uint32_t& tile) {
  const uint32_t P0 = qq.D * TA;
  const uint32_t P1 = (qq.n - qq.D) * (TA + TB);
  if (p < P0) {
    first = true;
    j = p / TA;
    tile = p % TA;
  } else if (p < P0 + P1) {
    const uint32_t pp = p - P0, w = TA + TB;
    const uint32_t t = qq.D + pp / w, off = pp % w;
    if (off < TA) {
      first = true;
      j = t;
      tile = off;
    } else {
      first = false;
      j = t - qq.D;
      tile = off - TA;
    }
  } else {
    const uint32_t pp = p - P0 - P1;
    first = false;
    j = qq.n - qq.D + pp / TB;
    tile = pp % TB;
  }
}

// Queue vector j of XCD x -> batch vector index (limb x + 8 i, polynomial p).
NTTK_HD inline uint32_t vector_of(uint32_t x, uint32_t j, uint32_t L, uint32_t P) {
  const uint32_t i = j / P, p = j % P;
  return p * L + x + 8 * i;
}

}  // namespace nttk
