// One persistent launch per transform direction, both passes fused (Section VI-C's
// Kernel-1 and Kernel-2 in a single grid).
//
// Work is cut into tiles: a column tile is C adjacent columns of one limb-vector (the
// first log2 N1 stages), a row tile is V rows of one limb-vector (the remaining stages).
// A limb-vector's row tiles may start only after all its column tiles are done (the
// other way round for the inverse), so each vector carries a completion counter.
//
// Every vector is bound to one XCD (limb l -> XCD l mod 8, all polynomials of that limb
// together so they share its twiddles) and each XCD drains its own queue: a workgroup
// reads its XCD from the hardware register HW_REG_XCC_ID and takes the next position of
// that XCD's queue.  Both passes of a vector therefore run on CUs that share one L2, and
// the pass-1 output is read back by pass 2 from that L2 instead of HBM.  Within an XCD
// the L2 is the point of coherence: a producer waits for its stores to complete before
// bumping the vector's counter, and a consumer invalidates its CU's L1 after seeing the
// counter complete, before loading.
//
// Queue order of an XCD with n vectors, lag D: C(0) .. C(D-1), then C(t), R(t-D) for
// t = D .. n-1, then R(n-D) .. R(n-1), where C(j) / R(j) are the tiles of pass 1 / pass 2
// of its j-th vector.  A row tile only ever waits for column tiles taken earlier from the
// same queue by running workgroups, and column tiles never wait, so the wait always ends.
//
// The last workgroup to leave (one counter over the grid) drains any queue whose XCD got
// no workgroup at all, then zeroes every counter for the next launch on the stream.
#pragma once
#include "fused_args.hpp"
#include "fused_queue.hpp"
#include "kernels_impl.hpp"

namespace nttk {

constexpr uint32_t kFusedThreads = 256;
constexpr int kFusedLR = 4;         // 16 values per lane in both sub-transforms
constexpr uint32_t kCtrDone = 16;   // counters: [0..7] queue heads, [8] exit count, [16 + v] vector done

__device__ __forceinline__ uint32_t xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;   // HW_REG_XCC_ID, bits [3:0]
}

template <int LOGM1, int LOGM2>
struct FusedShape {
  using SC = Steps<LOGM1, kFusedLR>;         // column sub-transform
  static constexpr int M1 = 1 << LOGM1;      // column length N1
  static constexpr int C = 4096 / M1;        // columns per column tile
  static constexpr int TC = M1 / SC::R;      // lanes per column
  using RC = RowCfg<LOGM2, (int)kFusedThreads, kFusedLR>;   // row tile: V rows of M2
  static constexpr int M2 = 1 << LOGM2;
  static constexpr int Tc = M2 / C;          // column tiles per vector
  static constexpr int Tr = M1 / RC::V;      // row tiles per vector
  static constexpr int LDS_WORDS = (M1 * C > RC::V * RC::PITCH) ? M1 * C : RC::V * RC::PITCH;
  static_assert(C * TC == (int)kFusedThreads, "column tile must fill the workgroup");
  static_assert(RC::NT == (int)kFusedThreads, "row tile must fill the workgroup");
  static_assert(Tc >= 1 && Tr >= 1, "N too small for the fused shape");
};

__device__ __forceinline__ void signal_done(uint32_t* ctr, uint32_t v) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this lane's stores have reached L2
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(&ctr[kCtrDone + v], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_done(const uint32_t* ctr, uint32_t v, uint32_t need) {
  if (threadIdx.x == 0) {
    while (__hip_atomic_load(&ctr[kCtrDone + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need)
      __builtin_amdgcn_s_sleep(2);
  }
  __syncthreads();
  asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");   // drop stale L1 lines of this CU
}

// ---------------------------------------------------------------- tiles (forward)

template <bool FAST, int LOGM1, int LOGM2>
__device__ __forceinline__ void fwd_col_tile(const PassArgs& a, uint32_t v, uint32_t cg, uint64_t* lds, Tw* twl) {
  using F = FusedShape<LOGM1, LOGM2>;
  using S = typename F::SC;
  const uint32_t tid = threadIdx.x, c = tid % F::C, t = tid / F::C;
  const uint32_t limb = v % a.L;
  const Mod md = Mod::load(a.mc + 8 * (size_t)limb);
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  for (uint32_t i = tid; i < (uint32_t)F::M1; i += kFusedThreads) twl[i] = tab[i];
  uint64_t* colp = a.data + ((uint64_t)v << a.logN) + cg * F::C + c;
  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = colp[(size_t)S::template idx<0>(t, u) << LOGM2];
  __syncthreads();
  auto tabfn = [&](uint32_t ix) { return twl[ix]; };
  OtTables ot{};
  static_for<0, S::K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k > 0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) lds[S::template idx<k - 1>(t, u) * F::C + c] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = lds[S::template idx<k>(t, u) * F::C + c];
    }
    ct_step<FAST, LOGM1, kFusedLR, k, 0>(x, t, 1u, tabfn, ot, md);
  });
#pragma unroll
  for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<S::K - 1>(t, u) << LOGM2] = x[u];
}

template <bool FAST, int LOGM1, int LOGM2, int OTS>
__device__ __forceinline__ void fwd_row_tile(const PassArgs& a, uint32_t v, uint32_t rt, uint64_t* lds) {
  using F = FusedShape<LOGM1, LOGM2>;
  using RC = typename F::RC;
  using S = typename RC::S;
  using A = Arith<FAST>;
  const uint32_t tid = threadIdx.x, vr = tid / RC::T, t = tid % RC::T;
  const uint32_t limb = v % a.L;
  const Mod md = Mod::load(a.mc + 8 * (size_t)limb);
  const uint32_t row = rt * RC::V + vr;
  const uint32_t base = (uint32_t)F::M1 + row;
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  OtTables ot{};
  if constexpr (OTS > 0) {
    ot.lo = a.ot_lo + ((size_t)limb << a.ot_log2_base);
    ot.hi = a.ot_hi + ((size_t)limb << (a.logN - a.ot_log2_base));
    ot.logN = a.logN;
    ot.b = a.ot_log2_base;
  }
  auto tabfn = [&](uint32_t ix) { return tab[ix]; };
  uint64_t* rowp = a.data + ((uint64_t)v << a.logN) + (size_t)row * RC::M;
  uint64_t* l = lds + vr * RC::PITCH;
  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = rowp[S::template idx<0>(t, u)];
  static_for<0, S::K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k > 0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[RC::at(S::template idx<k - 1>(t, u))] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[RC::at(S::template idx<k>(t, u))];
    }
    ct_step<FAST, LOGM2, kFusedLR, k, OTS>(x, t, base, tabfn, ot, md);
  });
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = A::fwd_final(x[u], md);
  if constexpr (S::K > 1) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) l[RC::at(S::template idx<S::K - 1>(t, u))] = x[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = l[RC::at(S::template idx<0>(t, u))];
  }
#pragma unroll
  for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
}

// ---------------------------------------------------------------- tiles (inverse)

template <bool FAST, int LOGM1, int LOGM2, int OTS>
__device__ __forceinline__ void inv_row_tile(const PassArgs& a, uint32_t v, uint32_t rt, uint64_t* lds) {
  using F = FusedShape<LOGM1, LOGM2>;
  using RC = typename F::RC;
  using S = typename RC::S;
  const uint32_t tid = threadIdx.x, vr = tid / RC::T, t = tid % RC::T;
  const uint32_t limb = v % a.L;
  const Mod md = Mod::load(a.mc + 8 * (size_t)limb);
  const uint32_t row = rt * RC::V + vr;
  const uint32_t base = (uint32_t)F::M1 + row;
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  OtTables ot{};
  if constexpr (OTS > 0) {
    ot.lo = a.ot_lo + ((size_t)limb << a.ot_log2_base);
    ot.hi = a.ot_hi + ((size_t)limb << (a.logN - a.ot_log2_base));
    ot.logN = a.logN;
    ot.b = a.ot_log2_base;
  }
  const Tw sc{};
  auto tabfn = [&](uint32_t ix) { return tab[ix]; };
  uint64_t* rowp = a.data + ((uint64_t)v << a.logN) + (size_t)row * RC::M;
  uint64_t* l = lds + vr * RC::PITCH;
  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = rowp[S::template idx<0>(t, u)];
  if constexpr (S::K > 1) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) l[RC::at(S::template idx<0>(t, u))] = x[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = l[RC::at(S::template idx<S::K - 1>(t, u))];
  }
  static_for_down<S::K, 0>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k < S::K - 1) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[RC::at(S::template idx<k + 1>(t, u))] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[RC::at(S::template idx<k>(t, u))];
    }
    gs_step<FAST, LOGM2, kFusedLR, k, OTS, false>(x, t, base, tabfn, ot, md, sc, sc);
  });
#pragma unroll
  for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
}

template <bool FAST, int LOGM1, int LOGM2>
__device__ __forceinline__ void inv_col_tile(const PassArgs& a, uint32_t v, uint32_t cg, uint64_t* lds, Tw* twl) {
  using F = FusedShape<LOGM1, LOGM2>;
  using S = typename F::SC;
  using A = Arith<FAST>;
  const uint32_t tid = threadIdx.x, c = tid % F::C, t = tid / F::C;
  const uint32_t limb = v % a.L;
  const Mod md = Mod::load(a.mc + 8 * (size_t)limb);
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  for (uint32_t i = tid; i < (uint32_t)F::M1; i += kFusedThreads) twl[i] = tab[i];
  const Tw sc0 = a.scale[2 * limb], sc1 = a.scale[2 * limb + 1];
  uint64_t* colp = a.data + ((uint64_t)v << a.logN) + cg * F::C + c;
  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = colp[(size_t)S::template idx<S::K - 1>(t, u) << LOGM2];
  __syncthreads();
  auto tabfn = [&](uint32_t ix) { return twl[ix]; };
  OtTables ot{};
  static_for_down<S::K, 0>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k < S::K - 1) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) lds[S::template idx<k + 1>(t, u) * F::C + c] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = lds[S::template idx<k>(t, u) * F::C + c];
    }
    gs_step<FAST, LOGM1, kFusedLR, k, 0, true>(x, t, 1u, tabfn, ot, md, sc0, sc1);
  });
#pragma unroll
  for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<0>(t, u) << LOGM2] = A::inv_final(x[u], md);
}

// ---------------------------------------------------------------- persistent kernel

template <bool FAST, int LOGM1, int LOGM2, int OTS, bool INV>
__device__ __forceinline__ void run_item(const FusedArgs& f, uint32_t x, uint32_t p, const Queue& qq,
                                         uint64_t* lds, Tw* twl) {
  using F = FusedShape<LOGM1, LOGM2>;
  constexpr uint32_t TA = INV ? F::Tr : F::Tc;   // tiles of the pass that runs first
  constexpr uint32_t TB = INV ? F::Tc : F::Tr;
  bool first;
  uint32_t j, tile;
  decode(qq, p, TA, TB, first, j, tile);
  const uint32_t v = vector_of(x, j, f.a.L, f.P);
  __syncthreads();   // the previous tile is done with LDS
  if (first) {
    if constexpr (INV) inv_row_tile<FAST, LOGM1, LOGM2, OTS>(f.a, v, tile, lds);
    else fwd_col_tile<FAST, LOGM1, LOGM2>(f.a, v, tile, lds, twl);
    signal_done(f.ctr, v);
  } else {
    wait_done(f.ctr, v, TA);
    if constexpr (INV) inv_col_tile<FAST, LOGM1, LOGM2>(f.a, v, tile, lds, twl);
    else fwd_row_tile<FAST, LOGM1, LOGM2, OTS>(f.a, v, tile, lds);
  }
}

template <bool FAST, int LOGM1, int LOGM2, int OTS, bool INV>
__global__ __launch_bounds__(kFusedThreads) void fused_kernel(FusedArgs f) {
  using F = FusedShape<LOGM1, LOGM2>;
  __shared__ uint64_t lds[F::LDS_WORDS];
  __shared__ Tw twl[F::M1];
  __shared__ uint32_t s_pos;
  const uint32_t x = xcc_id();
  const Queue qq = queue_of(x, f.a.L, f.P, f.lag, F::Tc, F::Tr);
  for (;;) {
    if (threadIdx.x == 0) s_pos = __hip_atomic_fetch_add(&f.ctr[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t p = s_pos;
    if (p >= qq.total) break;
    run_item<FAST, LOGM1, LOGM2, OTS, INV>(f, x, p, qq, lds, twl);
    __syncthreads();   // every lane has read s_pos before lane 0 overwrites it
  }
  // Exit protocol: the last workgroup out drains queues nobody served, then resets.
  __syncthreads();
  if (threadIdx.x == 0) s_pos = __hip_atomic_fetch_add(&f.ctr[8], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (s_pos != gridDim.x - 1) return;
  for (uint32_t y = 0; y < 8; ++y) {
    const Queue qy = queue_of(y, f.a.L, f.P, f.lag, F::Tc, F::Tr);
    const uint32_t h = __hip_atomic_load(&f.ctr[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t p = h; p < qy.total; ++p) run_item<FAST, LOGM1, LOGM2, OTS, INV>(f, y, p, qy, lds, twl);
  }
  __syncthreads();
  const uint64_t nv = f.a.n_vec;
  for (uint64_t i = threadIdx.x; i < kCtrDone + nv; i += kFusedThreads) f.ctr[i] = 0;
}

template <bool FAST, int LOGM1, int LOGM2, int OTS, bool INV>
hipError_t go_fused(const FusedArgs& f, uint32_t max_grid, hipStream_t st) {
  using F = FusedShape<LOGM1, LOGM2>;
  const uint64_t tiles = f.a.n_vec * (uint64_t)(F::Tc + F::Tr);
  uint64_t grid = tiles < max_grid ? tiles : max_grid;
  if (max_grid >= 8) grid = (grid + 7) & ~7ull;   // one workgroup per XCD at least (smaller only on request)
  hipLaunchKernelGGL((fused_kernel<FAST, LOGM1, LOGM2, OTS, INV>), dim3((uint32_t)grid), dim3(kFusedThreads), 0, st,
                     f);
  return hipGetLastError();
}

// Fused shapes built: (log2 N1, log2 N2) for N = 2^13 .. 2^17 with the default split.
#define NTTK_FUSED_SHAPES(X) X(6, 7) X(7, 7) X(7, 8) X(8, 8) X(8, 9)

template <bool INV>
hipError_t fused_dispatch(const FusedArgs& f, int ots, uint32_t max_grid, hipStream_t st) {
  const uint32_t n1 = f.a.logN1, n2 = f.a.logN - f.a.logN1;
#define X(A, B)                                                                   \
  if (n1 == A && n2 == B) {                                                       \
    if (ots == 0) return go_fused<true, A, B, 0, INV>(f, max_grid, st);           \
    if (ots == 1) return go_fused<true, A, B, 1, INV>(f, max_grid, st);           \
    if (ots == 2) return go_fused<true, A, B, 2, INV>(f, max_grid, st);           \
  }
  NTTK_FUSED_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace nttk
