// The paper's ablation ladder (Section VI-A, VI-B, Table II): transforms that keep the data
// in global memory between launches.
//
//  * radix-2 (NTT_PATH_RADIX2): one launch per stage of Algorithm 1, one butterfly per lane,
//    twiddles read from the table;
//  * register-only high radix (NTT_PATH_REGISTER): one launch per group of k consecutive
//    stages, each lane loading the 2^k elements one group of butterflies needs, running the
//    k stages in registers and writing them back (radix 2^k; ceil(log2 N / k) launches).
//
// Why a lane's elements form a sub-transform: global stage s of Algorithm 1 pairs slots that
// differ in bit log2 N - 1 - s and gives slot i the twiddle Psi[2^s + (i >> (log2 N - s))].
// The group of stages s0 .. s0 + k - 1 touches bits lo .. lo + k - 1, lo = log2 N - s0 - k.
// Write a slot as (H, u, w): H the bits above the group, u the k group bits, w the lo bits
// below.  In local stage i (s = s0 + i) the twiddle index is 2^(s0+i) + (H << i) + (u >> (k-i))
// = ((2^s0 + H) << i) + (u >> (k - i)): the k-point sub-transform of passes.hpp with row base
// 2^s0 + H.  So the register steps of the two-pass kernels (ct_step, gs_step) do the work.
#include "kernels.hpp"
#include "passes.hpp"

namespace nttk {

constexpr int kStageThreads = 256;

// Group of K stages starting at global stage s0 (forward) on every vector.  FINAL: this group
// ends the transform (reduce to [0, q)).  Inverse (INV): stages run in Gentleman-Sande order;
// CANON_IN: the group sees the caller's canonical input; SCALE0: the group holds global
// stage 0 (1/N scale and final reduction).
template <bool FAST, int K, bool INV, bool FINAL, bool CANON_IN, bool SCALE0>
__global__ __launch_bounds__(kStageThreads) void stage_group_kernel(PassArgs a, uint32_t s0) {
  using A = Arith<FAST>;
  constexpr int R = 1 << K;
  const uint32_t lo = a.logN - s0 - K;
  const uint64_t per_vec = (uint64_t)1 << (a.logN - K);      // lanes per vector
  const uint64_t g = (uint64_t)blockIdx.x * kStageThreads + threadIdx.x;
  const uint64_t vec = g >> (a.logN - K);
  if (vec >= a.n_vec) return;
  const uint64_t r = g & (per_vec - 1);                        // (H, w) of this lane, w fastest
  const uint32_t w = (uint32_t)(r & ((1ull << lo) - 1)), H = (uint32_t)(r >> lo);
  const VecRef vr = vec_ref(a, vec);
  const Mod md = Mod::load((const uint64_t*)a.mc + 8 * (size_t)vr.limb);
  const Tw* tab = a.tw + ((size_t)vr.limb << a.logN);
  gu64* p = vr.base + (((size_t)H << (lo + K)) | w);
  const uint32_t base = (1u << s0) + H;
  auto tabfn = [&](uint32_t ix) { return tab[ix]; };
  OtTables ot{};
  uint64_t x[R];
#pragma unroll
  for (int u = 0; u < R; ++u) x[u] = p[(size_t)u << lo];
  if constexpr (!INV) {
    ct_step<FAST, K, K, 0, 0>(x, 0u, base, tabfn, ot, md);
    if constexpr (FINAL) {
#pragma unroll
      for (int u = 0; u < R; ++u) x[u] = A::fwd_final(x[u], md);
    }
  } else {
    Tw sc0{}, sc1{};
    if constexpr (SCALE0) {
      sc0 = a.scale[2 * vr.limb];
      sc1 = a.scale[2 * vr.limb + 1];
    }
    gs_step<FAST, K, K, 0, 0, SCALE0, CANON_IN ? 1 : 8>(x, 0u, base, tabfn, ot, md, sc0, sc1);
    if constexpr (SCALE0) {
#pragma unroll
      for (int u = 0; u < R; ++u) x[u] = A::inv_final(x[u], md);
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) p[(size_t)u << lo] = x[u];
}

template <bool FAST, int K, bool INV, bool F1, bool F2, bool F3>
static hipError_t go_group(const PassArgs& a, uint32_t s0, hipStream_t st) {
  const uint64_t lanes = a.n_vec << (a.logN - K);
  const uint64_t blocks = (lanes + kStageThreads - 1) / kStageThreads;
  hipLaunchKernelGGL((stage_group_kernel<FAST, K, INV, F1, F2, F3>), dim3((uint32_t)blocks), dim3(kStageThreads), 0,
                     st, a, s0);
  return hipGetLastError();
}

template <bool FAST, int K>
static hipError_t group_k(const PassArgs& a, uint32_t s0, bool inverse, hipStream_t st) {
  const bool last = s0 + K == a.logN;   // forward: the group that ends the transform
  if (!inverse) return last ? go_group<FAST, K, false, true, false, false>(a, s0, st)
                            : go_group<FAST, K, false, false, false, false>(a, s0, st);
  // the inverse runs the groups from the last stages down: the top group sees canonical
  // input, the group of stage 0 applies the scale
  const bool first = s0 + K == a.logN, scale = s0 == 0;
  if (first && scale) return go_group<FAST, K, true, false, true, true>(a, s0, st);
  if (first) return go_group<FAST, K, true, false, true, false>(a, s0, st);
  if (scale) return go_group<FAST, K, true, false, false, true>(a, s0, st);
  return go_group<FAST, K, true, false, false, false>(a, s0, st);
}

template <bool FAST>
static hipError_t group_any(const PassArgs& a, int k, uint32_t s0, bool inverse, hipStream_t st) {
  switch (k) {
    case 1: return group_k<FAST, 1>(a, s0, inverse, st);
    case 2: return group_k<FAST, 2>(a, s0, inverse, st);
    case 3: return group_k<FAST, 3>(a, s0, inverse, st);
    case 4: return group_k<FAST, 4>(a, s0, inverse, st);
    case 5: return group_k<FAST, 5>(a, s0, inverse, st);
  }
  return hipErrorInvalidValue;
}

uint32_t stage_group_count(uint32_t logN, int log2_radix) {
  return (logN + (uint32_t)log2_radix - 1) / (uint32_t)log2_radix;
}

// Group g of a transform: forward groups start at stage 0 and go up, each of log2_radix
// stages except a shorter last one; the inverse runs the same groups in the opposite order.
hipError_t launch_stage_group(const PassArgs& a, int log2_radix, bool inverse, uint32_t g, hipStream_t st) {
  if (log2_radix < 1 || log2_radix > 5 || a.logN < 1 || a.logN > 17) return hipErrorInvalidValue;
  const uint32_t n = stage_group_count(a.logN, log2_radix);
  if (g >= n) return hipErrorInvalidValue;
  const uint32_t fg = inverse ? n - 1 - g : g;                 // the group in forward order
  const uint32_t s0 = fg * (uint32_t)log2_radix;
  const int k = (int)(a.logN - s0 < (uint32_t)log2_radix ? a.logN - s0 : (uint32_t)log2_radix);
  return a.fast ? group_any<true>(a, k, s0, inverse, st) : group_any<false>(a, k, s0, inverse, st);
}

hipError_t launch_stage_groups(const PassArgs& a, int log2_radix, bool inverse, hipStream_t st) {
  const uint32_t n = stage_group_count(a.logN, log2_radix);
  for (uint32_t g = 0; g < n; ++g) {
    const hipError_t e = launch_stage_group(a, log2_radix, inverse, g, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace nttk
