// Host check of the fused transform's queue order (compiled with g++ by the test suite).
// Every (pass, vector, tile) of every XCD queue appears exactly once, every batch vector
// lands on the XCD of its limb, and each vector's first-pass tiles all precede its
// second-pass tiles in the queue, which is what makes every wait in the kernel end.
#include <algorithm>
#include <cstdio>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

#include "fused_queue.hpp"

using namespace nttk;

int main() {
  int bad = 0, cases = 0;
  const std::vector<std::pair<uint32_t, uint32_t>> tiles = {{16, 16}, {2, 2}, {4, 4}, {8, 8}, {32, 32}, {16, 8}, {8, 16}};
  for (uint32_t L : {1u, 3u, 7u, 8u, 9u, 45u, 60u})
    for (uint32_t P : {1u, 2u, 3u, 4u})
      for (uint32_t lag : {1u, 2u, 4u, 6u, 100u})
        for (auto [TA, TB] : tiles) {
          std::set<uint32_t> vecs;
          for (uint32_t x = 0; x < 8; ++x) {
            const Queue q = queue_of(x, L, P, lag, TA, TB);
            std::set<std::tuple<bool, uint32_t, uint32_t>> seen;
            std::vector<long> lastA(q.n, -1), firstB(q.n, 1L << 40);
            for (uint32_t p = 0; p < q.total; ++p) {
              bool f;
              uint32_t j, t;
              decode(q, p, TA, TB, f, j, t);
              if (j >= q.n || t >= (f ? TA : TB)) { ++bad; continue; }
              if (!seen.insert({f, j, t}).second) ++bad;
              if (f) lastA[j] = std::max<long>(lastA[j], p);
              else firstB[j] = std::min<long>(firstB[j], p);
              const uint32_t v = vector_of(x, j, L, P);
              if (v >= L * P || (v % L) % 8 != x) ++bad;
              vecs.insert(v);
            }
            if (seen.size() != (size_t)q.n * (TA + TB)) ++bad;
            for (uint32_t j = 0; j < q.n; ++j)
              if (!(lastA[j] < firstB[j])) ++bad;
            ++cases;
          }
          if (vecs.size() != (size_t)L * P) ++bad;
        }
  std::printf("%d queue cases, %d failures\n", cases, bad);
  return bad != 0;
}
