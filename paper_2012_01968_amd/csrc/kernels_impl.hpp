// NTT kernel templates for gfx950: the LDS-staged column pass and row pass of Section
// VI-C in both directions, and their launchers.  Each translation unit kernels_*.hip
// instantiates one direction for one arithmetic policy.  See passes.hpp for the split.
#pragma once
#include "kernels.hpp"
#include "passes.hpp"

namespace nttk {

#ifndef NTTK_LR
#define NTTK_LR 3
#endif
#ifndef NTTK_ROW_LR
#define NTTK_ROW_LR 0
#endif
constexpr int kLR = NTTK_LR;    // 2^kLR values per lane per register step (column pass)
// Row pass: NTTK_ROW_LR if set, else kLR; policy 9 takes 16 values per lane for rows of at
// least 2^10 points and kLR below.
constexpr int row_lr(int logm) {
  return NTTK_ROW_LR == 9 ? (logm >= 10 ? 4 : kLR) : (NTTK_ROW_LR > 0 ? NTTK_ROW_LR : kLR);
}
inline int row_lr_default(uint32_t logm) { return row_lr((int)logm); }
#ifndef NTTK_COL_WIDTH
#define NTTK_COL_WIDTH 16
#endif
#ifndef NTTK_ROW_THREADS
#define NTTK_ROW_THREADS 128
#endif
#ifndef NTTK_ROW_PRELOAD
#define NTTK_ROW_PRELOAD 1
#endif
constexpr int kColWidth = NTTK_COL_WIDTH;     // columns per column-pass tile (any N2 >= 16)
#ifndef NTTK_COL_WIDTH_WIDE
#define NTTK_COL_WIDTH_WIDE 64
#endif
constexpr int kColWidthWide = NTTK_COL_WIDTH_WIDE;   // columns per tile when N2 allows it
constexpr bool kRowPreload = NTTK_ROW_PRELOAD != 0;   // row pass: a step's twiddles loaded up front

template <int R>
struct PreTw {   // twiddles of one register step (see load_step_twiddles)
  Tw w[R];
  Tw w2[R];
};
constexpr int kRowThreads = NTTK_ROW_THREADS; // lanes per row-pass workgroup

// Tile of this workgroup.  Workgroups are dispatched to the eight XCDs round-robin (block
// b runs on XCD b mod 8), so XCD x gets the contiguous tile range [x*per, (x+1)*per):
// neighbouring tiles, which share cache lines (column tiles) or twiddles (row tiles of
// the polynomials of one limb), then meet in one L2.  The grid is 8*per workgroups;
// tiles past the end are padding.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t n_tiles, uint32_t debug) {
  const uint32_t per = (n_tiles + 7) / 8;
  const uint32_t t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  // debug mode: the tiles in reverse order (a different workgroup -> tile mapping must give
  // the same bits, since no tile depends on another)
  return (debug & kDebugReverseTiles) && t < n_tiles ? n_tiles - 1 - t : t;
}

// Debug mode: fill a workgroup's LDS with a poison pattern before use, so that a read of a
// slot that the exchange did not write shows up in the results.  Every lane of the workgroup
// takes part (call it where the whole workgroup is present).
template <int WORDS>
__device__ __forceinline__ void poison_lds(uint64_t* lds, uint32_t debug, uint32_t tid, uint32_t nt) {
  if (debug & kDebugPoisonLds) {
    for (uint32_t i = tid; i < (uint32_t)WORDS; i += nt) lds[i] = 0xBAD0BAD0BAD0BAD0ull;
    __syncthreads();
  }
}

// Limb-major order of the vectors of a [P][L] batch: position lp = l*P + p holds vector
// p*L + l, so the polynomials of one limb (one prime, one twiddle table) are adjacent.
__device__ __forceinline__ uint64_t limb_major_vec(uint64_t lp, uint32_t L, uint32_t P) {
  return (lp % P) * L + lp / P;
}

__device__ __forceinline__ uint32_t lds_pad(uint32_t r) { return r + (r >> 4); }

#ifndef NTTK_WAVE_SYNC
#define NTTK_WAVE_SYNC 1
#endif
// Ordering between the LDS writes and reads of one exchange among the T lanes of a row.  A
// row of at most 64 lanes lies in one wave (rows start at multiples of T in the workgroup),
// whose LDS instructions execute in program order, so a compiler-level fence at wavefront
// scope orders the exchange without a workgroup barrier.  Each exchange writes only the
// slots its lane read in the previous one, so no lane overwrites a slot another lane has
// yet to read (see fwd_row_kernel).
template <int T>
__device__ __forceinline__ void row_sync() {
  if constexpr (NTTK_WAVE_SYNC != 0 && T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int LOGM, int NTH = kRowThreads, int LR_ = row_lr(LOGM)>
struct RowCfg {
  using S = Steps<LOGM, LR_>;
  static constexpr int LR = LR_;
  static constexpr int M = 1 << LOGM;
  static constexpr int T = M / S::R;                    // lanes per row
  static constexpr int V = T >= NTH ? 1 : NTH / T;      // rows per workgroup
  static constexpr int NT = V * T;
  static constexpr int PITCH = M >= 16 ? M + M / 16 : M;
  // LDS slot of element r of a row: one pad slot per 16 elements.
  static __device__ __forceinline__ uint32_t at(uint32_t r) { return lds_pad(r); }
};

// ----------------------------------------------------------------------------- row pass
// Rows of length M = N / N1, V rows per workgroup; row g of the batch starts at
// data + g*M, belongs to vector g / N1 and is row g mod N1 of that vector's matrix.

// Read-only lookups that are the same for the whole workgroup (vector lists, primes) go
// through the constant address space so that the compiler can use scalar loads.
typedef const __attribute__((address_space(4))) VecDesc cVecDesc;
typedef const __attribute__((address_space(4))) uint64_t cu64;

struct RowRef {
  gu64* rowp;       // start of this lane's row
  const gu64* srcp; // where the row's input is read (rowp unless the launch is out of place)
  const gu64* keyp; // the row of the key vector at the same position (key-product launches)
  uint32_t limb;    // its prime
  uint32_t base;    // N1 + (row within its vector): the row's twiddle base
  bool valid;       // false for padding rows
};

// Row v of this workgroup's tile.  When V divides N1 (every split launch with at least V
// rows per vector) the tile's rows are consecutive rows of one vector, so the vector is
// looked up once per workgroup; otherwise each row finds its own vector.
template <typename C>
__device__ __forceinline__ RowRef row_ref(const PassArgs& a, uint32_t v) {
  const uint64_t rows = a.n_vec << a.logN1;
  const uint32_t n_tiles = (uint32_t)((rows + C::V - 1) / C::V);
  const uint32_t tile = __builtin_amdgcn_readfirstlane(xcd_tile(n_tiles, a.debug));
  const uint32_t N1 = 1u << a.logN1;
  if ((uint32_t)C::V <= N1) {
    const bool valid = tile < n_tiles;
    const uint32_t tl = valid ? tile : 0;
    gu64* vb;
    const gu64* sb;
    const gu64* kb = nullptr;
    uint32_t limb, r0;
    if (a.vecs) {
      const uint64_t h0 = (uint64_t)tl * C::V;   // list order
      const cVecDesc* d = (const cVecDesc*)a.vecs + (h0 >> a.logN1);
      vb = (gu64*)d->ptr;
      sb = vb;
      kb = (const gu64*)d->key;
      limb = d->limb;
      r0 = (uint32_t)(h0 & (N1 - 1));
    } else {
      // tile order (limb, row group, polynomial): the polynomials of one limb take the same
      // rows back to back, so a row's twiddles are fetched once into L2 for all of them
      const uint32_t log_groups = a.logN1 - (uint32_t)__builtin_ctz((uint32_t)C::V);
      const uint32_t p = tl % a.P, rest = tl / a.P;
      const uint32_t l = rest >> log_groups;
      r0 = (rest & ((1u << log_groups) - 1u)) * C::V;
      const uint64_t vec = (uint64_t)p * a.L + l;
      vb = (gu64*)(a.data + (vec << a.logN));
      sb = a.src ? (const gu64*)(a.src + (vec << a.logN)) : vb;
      if (a.key) kb = (const gu64*)(a.key + (vec << a.logN));
      limb = l;
    }
    const uint32_t r = r0 + v;
    const size_t off = (size_t)r * C::M;
    return RowRef{vb + off, sb + off, kb ? kb + off : nullptr, limb, N1 + r, valid};
  }
  const uint64_t h = (uint64_t)tile * C::V + v;
  const bool valid = tile < n_tiles && h < rows;
  uint64_t g = 0;   // row index in [vector][row] order
  if (valid) {
    const uint64_t lp = h >> a.logN1;
    g = ((a.vecs || !a.logN1 ? lp : limb_major_vec(lp, a.L, a.P)) << a.logN1) | (h & (N1 - 1));
  }
  const uint64_t vec = g >> a.logN1;
  const VecRef vr = vec_ref(a, vec);
  const uint32_t r = (uint32_t)(g & (N1 - 1));
  const size_t off = (size_t)r * C::M;
  const gu64* sb = (!a.vecs && a.src) ? (const gu64*)(a.src + (vec << a.logN)) : vr.base;
  const gu64* kb = a.vecs ? (const gu64*)a.vecs[vec].key : (a.key ? (const gu64*)(a.key + (vec << a.logN)) : nullptr);
  return RowRef{vr.base + off, sb + off, kb ? kb + off : nullptr, vr.limb, N1 + r, valid};
}

template <bool FAST, int LOGM, int OTS, int NTH, int LRR>
__global__ __launch_bounds__((RowCfg<LOGM, NTH, LRR>::NT)) void fwd_row_kernel(PassArgs a) {
  using A = Arith<FAST>;
  using C = RowCfg<LOGM, NTH, LRR>;
  using S = typename C::S;
  __shared__ uint64_t lds[C::V * C::PITCH];
  const uint32_t tid = threadIdx.x, v = tid / C::T, t = tid % C::T;
  poison_lds<C::V * C::PITCH>(lds, a.debug, tid, C::NT);
  const RowRef rr = row_ref<C>(a, v);
  const bool valid = rr.valid;
  const uint32_t limb = rr.limb;
  const Mod md = Mod::load((cu64*)a.mc + 8 * (size_t)limb);
  const uint32_t base = rr.base;
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  OtTables ot{};
  if constexpr (OTS > 0) {
    ot.lo = a.ot_lo + ((size_t)limb << a.ot_log2_base);
    ot.hi = a.ot_hi + ((size_t)limb << (a.logN - a.ot_log2_base));
    ot.logN = a.logN;
    ot.b = a.ot_log2_base;
  }
  auto tabfn = [&](uint32_t ix) { return tab[ix]; };
  // the first register step's twiddles are the same for every lane of a row: with one row per
  // wave (or fewer) they come through scalar loads
  auto tabu = [&](uint32_t ix) {
    const cu64* p = (const cu64*)tab + 2 * (size_t)ix;
    Tw w;
    w.w = p[0];
    w.wb = p[1];
    return w;
  };
  gu64* rowp = rr.rowp;
  uint64_t* l = lds + v * C::PITCH;

  uint64_t x[S::R];
  if (valid) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = rr.srcp[S::template idx<0>(t, u)];
  } else {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = 0;
  }

  static_for<0, S::K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    PreTw<S::R> pre;   // issued before the exchange so the loads overlap the barrier
    if constexpr (kRowPreload) {
      // (step 0's twiddle index does not depend on the lane: its bits all lie below the step;
      // with one row per wave the row base is the same in every lane of the wave)
      if constexpr (k == 0 && C::T >= 64)
        load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, 0u, __builtin_amdgcn_readfirstlane(base), tabu, ot);
      else load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, t, base, tabfn, ot);
    }
    if constexpr (k > 0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k - 1>(t, u))] = x[u];
      row_sync<C::T>();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
    }
    if constexpr (kRowPreload) ct_step<FAST, LOGM, C::LR, k, OTS>(x, t, base, tabfn, ot, md, pre);
    else ct_step<FAST, LOGM, C::LR, k, OTS>(x, t, base, tabfn, ot, md);
  });

#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = A::fwd_final(x[u], md);
  // back to natural positions through LDS, so that each store instruction writes whole lines
  // (storing each lane's 8 consecutive elements directly measured 7% slower: partial lines)
  if constexpr (S::K > 1 && C::T >= 64 && C::LR == 3) {
    // A wave holds 512 consecutive elements of its row (8 per lane), so it transposes them
    // through its own part of the row's LDS slots and needs no barrier: since the last
    // exchange's barrier every wave only touches its own part.
    const uint32_t wbase = (t & ~63u) * 8u, lane = t & 63u;
#pragma unroll
    for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<S::K - 1>(t, u))] = x[u];
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = l[C::at(wbase + 64u * u + lane)];
    if (valid) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) rowp[wbase + 64u * u + lane] = x[u];
    }
  } else {
    if constexpr (S::K > 1) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<S::K - 1>(t, u))] = x[u];
      row_sync<C::T>();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<0>(t, u))];
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
    }
  }
}

// SCALE0: single-pass inverse (N1 = 1), so this pass ends with global stage 0 and
// applies the 1/N scale and the final reduction.
template <bool FAST, int LOGM, int OTS, bool SCALE0, int NTH, int LRR>
__global__ __launch_bounds__((RowCfg<LOGM, NTH, LRR>::NT)) void inv_row_kernel(PassArgs a) {
  using A = Arith<FAST>;
  using C = RowCfg<LOGM, NTH, LRR>;
  using S = typename C::S;
  __shared__ uint64_t lds[C::V * C::PITCH];
  const uint32_t tid = threadIdx.x, v = tid / C::T, t = tid % C::T;
  poison_lds<C::V * C::PITCH>(lds, a.debug, tid, C::NT);
  const RowRef rr = row_ref<C>(a, v);
  const bool valid = rr.valid;
  const uint32_t limb = rr.limb;
  const Mod md = Mod::load((cu64*)a.mc + 8 * (size_t)limb);
  const uint32_t base = rr.base;
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  OtTables ot{};
  if constexpr (OTS > 0) {
    ot.lo = a.ot_lo + ((size_t)limb << a.ot_log2_base);
    ot.hi = a.ot_hi + ((size_t)limb << (a.logN - a.ot_log2_base));
    ot.logN = a.logN;
    ot.b = a.ot_log2_base;
  }
  Tw sc0{}, sc1{};
  if constexpr (SCALE0) {
    sc0 = a.scale[2 * limb];
    sc1 = a.scale[2 * limb + 1];
  }
  auto tabfn = [&](uint32_t ix) { return tab[ix]; };
  // the first register step's twiddles are the same for every lane of a row: with one row per
  // wave (or fewer) they come through scalar loads
  auto tabu = [&](uint32_t ix) {
    const cu64* p = (const cu64*)tab + 2 * (size_t)ix;
    Tw w;
    w.w = p[0];
    w.wb = p[1];
    return w;
  };
  gu64* rowp = rr.rowp;
  uint64_t* l = lds + v * C::PITCH;

  // loaded straight into the first step's positions (8 consecutive elements per lane): the
  // wave's loads still cover whole lines across its 4 instructions, and no LDS exchange
  // precedes the first step
  uint64_t x[S::R];
  if (valid) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = rowp[S::template idx<S::K - 1>(t, u)];
  } else {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = 0;
  }

  static_for_down<S::K, 0>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    PreTw<S::R> pre;   // issued before the exchange so the loads overlap the barrier
    if constexpr (kRowPreload) {
      // (step 0's twiddle index does not depend on the lane: its bits all lie below the step;
      // with one row per wave the row base is the same in every lane of the wave)
      if constexpr (k == 0 && C::T >= 64)
        load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, 0u, __builtin_amdgcn_readfirstlane(base), tabu, ot);
      else load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, t, base, tabfn, ot);
    }
    if constexpr (k < S::K - 1) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k + 1>(t, u))] = x[u];
      row_sync<C::T>();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
    }
    // the first register step sees the caller's canonical input
    constexpr int IN_B = k == S::K - 1 ? 1 : 8;
    if constexpr (kRowPreload) gs_step<FAST, LOGM, C::LR, k, OTS, SCALE0, IN_B>(x, t, base, tabfn, ot, md, sc0, sc1, pre);
    else gs_step<FAST, LOGM, C::LR, k, OTS, SCALE0, IN_B>(x, t, base, tabfn, ot, md, sc0, sc1);
  });

  if constexpr (SCALE0) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = A::inv_final(x[u], md);
  }
  if (valid) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
  }
}

// ----------------------------------------------------------------- row pass with a key product
// The NTT-based product of Section III-A on the rows of an N1 x N2 split: the forward row
// stages, the final reduction, the element-wise product with the key (already in the NTT
// domain, same bit-reversed positions) and the inverse row stages, on registers, in one
// launch.  The forward row pass leaves each lane holding the positions of its last register
// step, which are the positions the inverse row pass starts from, so no exchange separates
// the two halves, and the key is read at those positions (R consecutive elements per lane).
// af carries the data, the keys and the forward tables; ai the inverse tables and 1/N.
// SCALE0: single-pass transform (N1 = 1): the whole product happens here.
template <bool FAST, int LOGM, int OTS, bool SCALE0, int NTH, int LRR>
__global__ __launch_bounds__((RowCfg<LOGM, NTH, LRR>::NT)) void mul_row_kernel(PassArgs af, PassArgs ai) {
  using A = Arith<FAST>;
  using C = RowCfg<LOGM, NTH, LRR>;
  using S = typename C::S;
  __shared__ uint64_t lds[C::V * C::PITCH];
  const uint32_t tid = threadIdx.x, v = tid / C::T, t = tid % C::T;
  poison_lds<C::V * C::PITCH>(lds, af.debug, tid, C::NT);
  const RowRef rr = row_ref<C>(af, v);
  const bool valid = rr.valid;
  const uint32_t limb = rr.limb;
  const Mod md = Mod::load((cu64*)af.mc + 8 * (size_t)limb);
  const uint32_t base = rr.base;
  const Tw* tabf = af.tw + ((size_t)limb << af.logN);
  const Tw* tabi = ai.tw + ((size_t)limb << af.logN);
  OtTables otf{}, oti{};
  if constexpr (OTS > 0) {
    otf.lo = af.ot_lo + ((size_t)limb << af.ot_log2_base);
    otf.hi = af.ot_hi + ((size_t)limb << (af.logN - af.ot_log2_base));
    oti.lo = ai.ot_lo + ((size_t)limb << af.ot_log2_base);
    oti.hi = ai.ot_hi + ((size_t)limb << (af.logN - af.ot_log2_base));
    otf.logN = oti.logN = af.logN;
    otf.b = oti.b = af.ot_log2_base;
  }
  Tw sc0{}, sc1{};
  if constexpr (SCALE0) {
    sc0 = ai.scale[2 * limb];
    sc1 = ai.scale[2 * limb + 1];
  }
  auto tabfnf = [&](uint32_t ix) { return tabf[ix]; };
  auto tabfni = [&](uint32_t ix) { return tabi[ix]; };
  // step 0's twiddles through scalar loads when a wave holds one row (see fwd_row_kernel)
  auto scalar_tw = [](const Tw* tab, uint32_t ix) {
    const cu64* p = (const cu64*)tab + 2 * (size_t)ix;
    Tw w;
    w.w = p[0];
    w.wb = p[1];
    return w;
  };
  auto tabuf = [&](uint32_t ix) { return scalar_tw(tabf, ix); };
  auto tabui = [&](uint32_t ix) { return scalar_tw(tabi, ix); };
  uint64_t* l = lds + v * C::PITCH;

  uint64_t x[S::R];
  if (valid) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = rr.srcp[S::template idx<0>(t, u)];
  } else {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = 0;
  }
  static_for<0, S::K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    PreTw<S::R> pre;
    if constexpr (k == 0 && C::T >= 64)
      load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, 0u, __builtin_amdgcn_readfirstlane(base), tabuf, otf);
    else
      load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, t, base, tabfnf, otf);
    if constexpr (k > 0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k - 1>(t, u))] = x[u];
      row_sync<C::T>();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
    }
    ct_step<FAST, LOGM, C::LR, k, OTS>(x, t, base, tabfnf, otf, md, pre);
  });
  // canonical NTT-domain values times the key at the same positions
  if (valid) {
    const uint64_t mu = ((cu64*)af.mu)[limb];
    const uint32_t bits = ((const __attribute__((address_space(4))) uint32_t*)af.bits)[limb];
#pragma unroll
    for (int u = 0; u < S::R; ++u)
      x[u] = mulmod_barrett(A::fwd_final(x[u], md), rr.keyp[S::template idx<S::K - 1>(t, u)], md.q, mu, bits);
  }
  static_for_down<S::K, 0>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    PreTw<S::R> pre;
    if constexpr (k == 0 && C::T >= 64)
      load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, 0u, __builtin_amdgcn_readfirstlane(base), tabui, oti);
    else
      load_step_twiddles<LOGM, C::LR, k, OTS>(pre.w, pre.w2, t, base, tabfni, oti);
    if constexpr (k < S::K - 1) {
      // the first of these writes goes to the slots this lane read in the forward half's
      // last exchange, which no other lane reads, so it needs no barrier before it
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k + 1>(t, u))] = x[u];
      row_sync<C::T>();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
    }
    // the key product leaves canonical values (padding rows skip it, but are never stored)
    gs_step<FAST, LOGM, C::LR, k, OTS, SCALE0, k == S::K - 1 ? 1 : 8>(x, t, base, tabfni, oti, md, sc0, sc1, pre);
  });
  if constexpr (SCALE0) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = A::inv_final(x[u], md);
  }
  if (valid) {
#pragma unroll
    for (int u = 0; u < S::R; ++u) rr.rowp[S::template idx<0>(t, u)] = x[u];
  }
}

// -------------------------------------------------------------------------- column pass
// W adjacent columns of one vector per workgroup (the coalesced Kernel-1 of Section VI-C:
// lanes of a wave cover adjacent columns, so every row segment is one run of W * 8 bytes).
// Longer runs stream better from HBM: the launcher takes kColWidthWide columns when N2 has
// that many and the workgroup stays at 512 lanes or fewer, and kColWidth otherwise.  The first N1 twiddles are staged in LDS before use.

template <int LOGM, int WREQ = kColWidth>
struct ColCfg {
  using S = Steps<LOGM, kLR>;
  static constexpr int M = 1 << LOGM;
  static constexpr int T = M / S::R;      // lanes per column
  static constexpr int W = WREQ * T > 1024 ? 1024 / T : WREQ;   // at most 1024 lanes
  static constexpr int NT = W * T;
  static constexpr int PITCH = W;         // LDS elements per matrix row
  static __device__ __forceinline__ uint32_t at(uint32_t r) { return r * PITCH; }   // LDS offset of row r
};

template <bool FAST, int LOGM, int WREQ>
__global__ __launch_bounds__((ColCfg<LOGM, WREQ>::NT)) void fwd_col_kernel(PassArgs a) {
  using C = ColCfg<LOGM, WREQ>;
  using S = typename C::S;
  __shared__ uint64_t lds[C::M * C::PITCH];
  __shared__ Tw twl[C::M];
  const uint32_t tid = threadIdx.x, c = tid % C::W, t = tid / C::W;
  const uint32_t logN2 = a.logN - LOGM;
  const uint32_t groups = (1u << logN2) / C::W;
  const uint32_t n_tiles = (uint32_t)(a.n_vec * groups);
  const uint32_t tile = xcd_tile(n_tiles, a.debug);
  if (tile >= n_tiles) return;   // padding workgroup (uniform: no barrier is skipped by part of it)
  poison_lds<C::M * C::PITCH>(lds, a.debug, tid, C::NT);
  const uint64_t vec = a.vecs ? tile / groups : limb_major_vec(tile / groups, a.L, a.P);
  const uint32_t cg = tile % groups;
  const VecRef vr = vec_ref(a, vec);
  const uint32_t limb = vr.limb;
  const Mod md = Mod::load((cu64*)a.mc + 8 * (size_t)limb);
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  gu64* colp = vr.base + cg * C::W + c;
  const gu64* colsrc = (!a.vecs && a.src) ? (const gu64*)(a.src + (vec << a.logN)) + cg * C::W + c : colp;

  // the column loads go out first, so that the twiddle staging waits on both at once
  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = colsrc[(size_t)S::template idx<0>(t, u) << logN2];
  for (uint32_t i = tid; i < (uint32_t)C::M; i += C::NT) twl[i] = tab[i];
  __syncthreads();
  auto tabfn = [&](uint32_t ix) { return twl[ix]; };
  OtTables ot{};

  static_for<0, S::K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k > 0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) lds[C::at(S::template idx<k - 1>(t, u)) + c] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = lds[C::at(S::template idx<k>(t, u)) + c];
    }
    ct_step<FAST, LOGM, kLR, k, 0>(x, t, 1u, tabfn, ot, md);
  });

#pragma unroll
  for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<S::K - 1>(t, u) << logN2] = x[u];
}

template <bool FAST, int LOGM, int WREQ>
__global__ __launch_bounds__((ColCfg<LOGM, WREQ>::NT)) void inv_col_kernel(PassArgs a) {
  using A = Arith<FAST>;
  using C = ColCfg<LOGM, WREQ>;
  using S = typename C::S;
  __shared__ uint64_t lds[C::M * C::PITCH];
  __shared__ Tw twl[C::M];
  const uint32_t tid = threadIdx.x, c = tid % C::W, t = tid / C::W;
  const uint32_t logN2 = a.logN - LOGM;
  const uint32_t groups = (1u << logN2) / C::W;
  const uint32_t n_tiles = (uint32_t)(a.n_vec * groups);
  const uint32_t tile = xcd_tile(n_tiles, a.debug);
  if (tile >= n_tiles) return;   // padding workgroup (uniform: no barrier is skipped by part of it)
  poison_lds<C::M * C::PITCH>(lds, a.debug, tid, C::NT);
  const uint64_t vec = a.vecs ? tile / groups : limb_major_vec(tile / groups, a.L, a.P);
  const uint32_t cg = tile % groups;
  const VecRef vr = vec_ref(a, vec);
  const uint32_t limb = vr.limb;
  const Mod md = Mod::load((cu64*)a.mc + 8 * (size_t)limb);
  const Tw* tab = a.tw + ((size_t)limb << a.logN);
  const Tw sc0 = a.scale[2 * limb], sc1 = a.scale[2 * limb + 1];
  gu64* colp = vr.base + cg * C::W + c;

  uint64_t x[S::R];
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = colp[(size_t)S::template idx<S::K - 1>(t, u) << logN2];
  for (uint32_t i = tid; i < (uint32_t)C::M; i += C::NT) twl[i] = tab[i];
  __syncthreads();
  auto tabfn = [&](uint32_t ix) { return twl[ix]; };
  OtTables ot{};

  static_for_down<S::K, 0>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k < S::K - 1) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) lds[C::at(S::template idx<k + 1>(t, u)) + c] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = lds[C::at(S::template idx<k>(t, u)) + c];
    }
    gs_step<FAST, LOGM, kLR, k, 0, true>(x, t, 1u, tabfn, ot, md, sc0, sc1);
  });

#pragma unroll
  for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<0>(t, u) << logN2] = A::inv_final(x[u], md);
}

// ------------------------------------------------------------------------------ launchers

// Row-pass tile shapes a plan may ask for (PassArgs::row_lr, row_nth): 2^LR values per lane
// and a workgroup of NTH lanes (V = NTH / T rows of T lanes each, or one row when a row
// alone needs NTH lanes or more).  Shapes that give the same (LR, V) are one kernel: the
// workgroup size is canonicalised to max(T, NTH).
constexpr int row_t(int logm, int lr) { return (1 << logm) >> (lr < logm ? lr : logm); }
constexpr int row_nth_canon(int logm, int lr, int nth) { return row_t(logm, lr) >= nth ? row_t(logm, lr) : nth; }

template <int LOGM, typename F>
__host__ hipError_t with_row_shape(const PassArgs& a, F&& f) {
  const int lr = a.row_lr ? (int)a.row_lr : row_lr(LOGM);
  const int nth = a.row_nth ? (int)a.row_nth : kRowThreads;
#define NTTK_SHAPE(LR_, NTH_)                                                                             \
  if (lr == LR_ && nth == NTH_)                                                                           \
    return f(std::integral_constant<int, row_nth_canon(LOGM, LR_, NTH_)>{}, std::integral_constant<int, LR_>{});
  NTTK_SHAPE(3, 128) NTTK_SHAPE(3, 64) NTTK_SHAPE(3, 256)
  NTTK_SHAPE(2, 128) NTTK_SHAPE(2, 64) NTTK_SHAPE(2, 256)
#undef NTTK_SHAPE
  return hipErrorInvalidValue;
}

template <bool FAST, int LOGM, int OTS, int NTH, int LRR>
hipError_t go_fwd_row(const PassArgs& a, hipStream_t st) {
  using C = RowCfg<LOGM, NTH, LRR>;
  const uint64_t rows = a.n_vec << a.logN1;
  const uint64_t blocks = ((rows + C::V - 1) / C::V + 7) / 8 * 8;
  hipLaunchKernelGGL((fwd_row_kernel<FAST, LOGM, OTS, NTH, LRR>), dim3((uint32_t)blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <bool FAST, int LOGM, int OTS, bool SCALE0, int NTH, int LRR>
hipError_t go_inv_row(const PassArgs& a, hipStream_t st) {
  using C = RowCfg<LOGM, NTH, LRR>;
  const uint64_t rows = a.n_vec << a.logN1;
  const uint64_t blocks = ((rows + C::V - 1) / C::V + 7) / 8 * 8;
  hipLaunchKernelGGL((inv_row_kernel<FAST, LOGM, OTS, SCALE0, NTH, LRR>), dim3((uint32_t)blocks), dim3(C::NT), 0, st,
                     a);
  return hipGetLastError();
}

template <bool FAST, int LOGM, int WREQ>
hipError_t launch_fwd_col(const PassArgs& a, hipStream_t st) {
  using C = ColCfg<LOGM, WREQ>;
  const uint64_t blocks = (a.n_vec * ((1u << (a.logN - LOGM)) / C::W) + 7) / 8 * 8;
  hipLaunchKernelGGL((fwd_col_kernel<FAST, LOGM, WREQ>), dim3((uint32_t)blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <bool FAST, int LOGM, int WREQ>
hipError_t launch_inv_col(const PassArgs& a, hipStream_t st) {
  using C = ColCfg<LOGM, WREQ>;
  const uint64_t blocks = (a.n_vec * ((1u << (a.logN - LOGM)) / C::W) + 7) / 8 * 8;
  hipLaunchKernelGGL((inv_col_kernel<FAST, LOGM, WREQ>), dim3((uint32_t)blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

// The wide tile where N2 = N / N1 holds that many columns, for columns of at most 64 points:
// the wide tile of longer columns is a 1024-lane workgroup with over 64 KB of LDS, which
// measured slower than the narrow one.
template <int LOGM>
constexpr bool col_wide_differs() {
  return ColCfg<LOGM, kColWidthWide>::W != ColCfg<LOGM, kColWidth>::W && ColCfg<LOGM, kColWidthWide>::NT <= 512;
}

// Column tile of a launch: the plan's requested width (PassArgs::col_w: 16 to 256 adjacent
// columns, fewer when the column is long enough to reach 1024 lanes), else the wide tile
// where N2 holds it and the narrow one otherwise.  A requested width must fit N2 (checked
// when the plan is created, see tiles_supported).
template <int LOGM, typename F>
__host__ hipError_t with_col_width(const PassArgs& a, F&& f) {
  if (a.col_w == 16) return f(std::integral_constant<int, 16>{});
  if (a.col_w == 32) return f(std::integral_constant<int, 32>{});
  if (a.col_w == 64) return f(std::integral_constant<int, 64>{});
  if (a.col_w == 128) return f(std::integral_constant<int, 128>{});
  if (a.col_w == 256) return f(std::integral_constant<int, 256>{});
  if (a.col_w != 0) return hipErrorInvalidValue;
  if constexpr (col_wide_differs<LOGM>())
    if ((1u << (a.logN - LOGM)) >= (uint32_t)ColCfg<LOGM, kColWidthWide>::W)
      return f(std::integral_constant<int, kColWidthWide>{});
  return f(std::integral_constant<int, kColWidth>{});
}

template <bool FAST, int LOGM>
hipError_t go_fwd_col(const PassArgs& a, hipStream_t st) {
  return with_col_width<LOGM>(a, [&](auto w) { return launch_fwd_col<FAST, LOGM, decltype(w)::value>(a, st); });
}

template <bool FAST, int LOGM>
hipError_t go_inv_col(const PassArgs& a, hipStream_t st) {
  return with_col_width<LOGM>(a, [&](auto w) { return launch_inv_col<FAST, LOGM, decltype(w)::value>(a, st); });
}

#define NTTK_ROW_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)
#define NTTK_COL_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

template <bool FAST, int LM>
hipError_t fwd_row_lm(const PassArgs& a, int ots, hipStream_t st) {
  return with_row_shape<LM>(a, [&](auto nth, auto lr) {
    constexpr int NTH = decltype(nth)::value, LRR = decltype(lr)::value;
    if (ots == 0) return go_fwd_row<FAST, LM, 0, NTH, LRR>(a, st);
    if (ots == 1) return go_fwd_row<FAST, LM, 1, NTH, LRR>(a, st);
    if (ots == 2) return go_fwd_row<FAST, LM, 2, NTH, LRR>(a, st);
    return hipErrorInvalidValue;
  });
}

template <bool FAST>
hipError_t fwd_row(const PassArgs& a, int logm, int ots, hipStream_t st) {
  switch (logm) {
#define X(LM) \
  case LM:    \
    return fwd_row_lm<FAST, LM>(a, ots, st);
    NTTK_ROW_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <bool FAST, int LM>
hipError_t inv_row_lm(const PassArgs& a, int ots, bool scale0, hipStream_t st) {
  return with_row_shape<LM>(a, [&](auto nth, auto lr) {
    constexpr int NTH = decltype(nth)::value, LRR = decltype(lr)::value;
    if (scale0) {
      if (ots == 0) return go_inv_row<FAST, LM, 0, true, NTH, LRR>(a, st);
      if constexpr (LM >= 2) if (ots == 1) return go_inv_row<FAST, LM, 1, true, NTH, LRR>(a, st);
      if constexpr (LM >= 3) if (ots == 2) return go_inv_row<FAST, LM, 2, true, NTH, LRR>(a, st);
    } else {
      if (ots == 0) return go_inv_row<FAST, LM, 0, false, NTH, LRR>(a, st);
      if (ots == 1) return go_inv_row<FAST, LM, 1, false, NTH, LRR>(a, st);
      if (ots == 2) return go_inv_row<FAST, LM, 2, false, NTH, LRR>(a, st);
    }
    return hipErrorInvalidValue;
  });
}

template <bool FAST>
hipError_t inv_row(const PassArgs& a, int logm, int ots, bool scale0, hipStream_t st) {
  switch (logm) {
#define X(LM) \
  case LM:    \
    return inv_row_lm<FAST, LM>(a, ots, scale0, st);
    NTTK_ROW_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <bool FAST>
hipError_t fwd_col(const PassArgs& a, int logm, hipStream_t st) {
  switch (logm) {
#define X(LM) \
  case LM:    \
    return go_fwd_col<FAST, LM>(a, st);
    NTTK_COL_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <bool FAST>
hipError_t inv_col(const PassArgs& a, int logm, hipStream_t st) {
  switch (logm) {
#define X(LM) \
  case LM:    \
    return go_inv_col<FAST, LM>(a, st);
    NTTK_COL_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <bool FAST, int LOGM, int OTS, bool SCALE0, int NTH, int LRR>
hipError_t go_mul_row(const PassArgs& af, const PassArgs& ai, hipStream_t st) {
  using C = RowCfg<LOGM, NTH, LRR>;
  const uint64_t rows = af.n_vec << af.logN1;
  const uint64_t blocks = ((rows + C::V - 1) / C::V + 7) / 8 * 8;
  hipLaunchKernelGGL((mul_row_kernel<FAST, LOGM, OTS, SCALE0, NTH, LRR>), dim3((uint32_t)blocks), dim3(C::NT), 0, st,
                     af, ai);
  return hipGetLastError();
}

template <bool FAST, int LM>
hipError_t mul_rows_lm(const PassArgs& af, const PassArgs& ai, int ots, bool scale0, hipStream_t st) {
  return with_row_shape<LM>(af, [&](auto nth, auto lr) {
    constexpr int NTH = decltype(nth)::value, LRR = decltype(lr)::value;
    if (scale0) {
      if (ots == 0) return go_mul_row<FAST, LM, 0, true, NTH, LRR>(af, ai, st);
      if constexpr (LM >= 2) if (ots == 1) return go_mul_row<FAST, LM, 1, true, NTH, LRR>(af, ai, st);
      if constexpr (LM >= 3) if (ots == 2) return go_mul_row<FAST, LM, 2, true, NTH, LRR>(af, ai, st);
    } else {
      if (ots == 0) return go_mul_row<FAST, LM, 0, false, NTH, LRR>(af, ai, st);
      if (ots == 1) return go_mul_row<FAST, LM, 1, false, NTH, LRR>(af, ai, st);
      if (ots == 2) return go_mul_row<FAST, LM, 2, false, NTH, LRR>(af, ai, st);
    }
    return hipErrorInvalidValue;
  });
}

// Row passes with the key product in between (see mul_row_kernel): the whole product when
// logN1 = 0, else the part between the forward and the inverse column pass.
template <bool FAST>
hipError_t mul_rows(const PassArgs& af, const PassArgs& ai, int ots, hipStream_t st) {
  const int logm = (int)(af.logN - af.logN1);
  const bool scale0 = af.logN1 == 0;
  switch (logm) {
#define X(LM) \
  case LM:    \
    return mul_rows_lm<FAST, LM>(af, ai, ots, scale0, st);
    NTTK_ROW_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// Row-pass instances by row length.  The row kernels dominate the build, so the build spreads
// them over translation units: a dispatch unit (kernels_{fwd,inv,mul}_*.hip) declares every
// row length extern, and kernels_rows.hip, compiled once per direction, policy and range of
// row lengths, instantiates them.
#define NTTK_FWD_ROWS(PREFIX, FAST, LM) PREFIX template hipError_t fwd_row_lm<FAST, LM>(const PassArgs&, int, hipStream_t);
#define NTTK_INV_ROWS(PREFIX, FAST, LM) \
  PREFIX template hipError_t inv_row_lm<FAST, LM>(const PassArgs&, int, bool, hipStream_t);
#define NTTK_MUL_ROWS(PREFIX, FAST, LM) \
  PREFIX template hipError_t mul_rows_lm<FAST, LM>(const PassArgs&, const PassArgs&, int, bool, hipStream_t);

template <bool FAST>
hipError_t forward_pass(const PassArgs& a, int ots, int pass, hipStream_t st) {
  if (a.logN1 == 0) return pass == 0 ? fwd_row<FAST>(a, (int)a.logN, ots, st) : hipErrorInvalidValue;
  if (pass == 0) return fwd_col<FAST>(a, (int)a.logN1, st);
  if (pass == 1) return fwd_row<FAST>(a, (int)(a.logN - a.logN1), ots, st);
  return hipErrorInvalidValue;
}

template <bool FAST>
hipError_t inverse_pass(const PassArgs& a, int ots, int pass, hipStream_t st) {
  if (a.logN1 == 0) return pass == 0 ? inv_row<FAST>(a, (int)a.logN, ots, true, st) : hipErrorInvalidValue;
  if (pass == 0) return inv_row<FAST>(a, (int)(a.logN - a.logN1), ots, false, st);
  if (pass == 1) return inv_col<FAST>(a, (int)a.logN1, st);
  return hipErrorInvalidValue;
}

}  // namespace nttk
