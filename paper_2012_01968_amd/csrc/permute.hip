// Natural-order option (Section III-C): the forward transform leaves A_brv(i) in slot i
// (Algorithm 1's output order); a plan created with NTT_ORDER_NATURAL moves every slot i to
// slot brv(i) after the forward transform, and back before the inverse.  The bit-reversal
// permutation is an involution, so one kernel serves both directions.
//
// The permutation runs in place as swaps of tile pairs.  Write a slot index of log2 N bits as
// (h, m, l): h the top t bits, m the middle log2 N - 2t bits, l the low t bits.  Then
// brv(h, m, l) = (brv_t(l), brv(m), brv_t(h)), so the 2^t x 2^t tile of middle index m (rows
// h, each row 2^t consecutive slots) maps onto the tile of middle index brv(m), with row and
// column swapped and each bit-reversed.  A workgroup loads the tiles of m and brv(m) (one tile
// when they coincide) into LDS and writes each into the other's place, so global reads and
// writes go by rows of 2^t consecutive slots.
#include "kernels.hpp"
#include "passes.hpp"

namespace nttk {

constexpr int kPermThreads = 256;

template <int TB>   // t = TB: tiles of 2^TB x 2^TB slots
__global__ __launch_bounds__(kPermThreads) void brv_permute_kernel(PassArgs a) {
  constexpr uint32_t T = 1u << TB, E = T * T, PITCH = T + 1;   // one pad slot per LDS row
  __shared__ uint64_t tile[2][T * PITCH];
  const uint32_t mb = a.logN - 2 * TB;                 // middle bits
  const uint64_t vec = blockIdx.x >> mb;
  const uint32_t m = blockIdx.x & ((1u << mb) - 1u);
  const uint32_t mr = mb ? __brev(m) >> (32 - mb) : 0u;
  if (vec >= a.n_vec || m > mr) return;                // each pair once (uniform per workgroup)
  gu64* base = vec_ref(a, vec).base;
  const uint32_t hs = a.logN - TB;                     // shift of h in a slot index
  auto slot = [&](uint32_t h, uint32_t mm, uint32_t l) { return ((size_t)h << hs) | ((size_t)mm << TB) | l; };
  const int n_tiles = m == mr ? 1 : 2;
  for (int k = 0; k < n_tiles; ++k) {
    const uint32_t mm = k ? mr : m;
    for (uint32_t j = threadIdx.x; j < E; j += kPermThreads) {
      const uint32_t h = j >> TB, l = j & (T - 1);
      tile[k][h * PITCH + l] = base[slot(h, mm, l)];
    }
  }
  __syncthreads();
  // the tile of m goes to brv(m) and the tile of brv(m) to m: destination row h', column l'
  // takes source row brv_t(l'), column brv_t(h')
  for (int k = 0; k < n_tiles; ++k) {
    const uint32_t dst_m = k ? m : mr;
    for (uint32_t j = threadIdx.x; j < E; j += kPermThreads) {
      const uint32_t h2 = j >> TB, l2 = j & (T - 1);
      const uint32_t hs_ = TB ? __brev(l2) >> (32 - TB) : 0u, ls_ = TB ? __brev(h2) >> (32 - TB) : 0u;
      base[slot(h2, dst_m, l2)] = tile[k][hs_ * PITCH + ls_];
    }
  }
}

template <int TB>
static hipError_t go_permute(const PassArgs& a, hipStream_t st) {
  const uint32_t mb = a.logN - 2 * TB;
  const uint64_t blocks = a.n_vec << mb;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(brv_permute_kernel<TB>, dim3((uint32_t)blocks), dim3(kPermThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_brv_permute(const PassArgs& a, hipStream_t st) {
  if (a.logN < 1 || a.logN > 17) return hipErrorInvalidValue;
  const uint32_t t = a.logN / 2 < 5 ? a.logN / 2 : 5;   // 32 x 32 tiles from N = 2^10 up
  switch (t) {
    case 0: return go_permute<0>(a, st);
    case 1: return go_permute<1>(a, st);
    case 2: return go_permute<2>(a, st);
    case 3: return go_permute<3>(a, st);
    case 4: return go_permute<4>(a, st);
    default: return go_permute<5>(a, st);
  }
}

}  // namespace nttk
