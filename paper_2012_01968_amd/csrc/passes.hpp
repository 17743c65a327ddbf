// LDS-staged NTT passes for gfx950.
//
// An N-point transform (Algorithm 1: stages m = 1, 2, ..., N/2, twiddle Psi[m + j] for
// block j) is split as N = N1 * N2 (Section VI-C).  View a limb as an N1 x N2 row-major
// matrix.  The first log2(N1) stages only pair elements of the same column (stride N2);
// the remaining log2(N2) stages only pair elements of the same row.  For both passes
// the twiddle of local stage s and local block j is Psi[(base << s) + j], with
// base = 1 for a column and base = N1 + row for a row, so one sub-transform routine
// serves the column pass (Kernel-1 in the paper), the row pass (Kernel-2) and, with
// N1 = 1, the single-pass kernel used when a whole limb fits in one workgroup.
//
// Inside a workgroup each lane holds R = 2^LR values and runs up to LR consecutive
// stages in registers (the per-thread NTT of Section VI-C); between register steps the
// values are exchanged through LDS with one barrier.  Register step k of an M-point
// sub-transform covers the index bits [blo(k), blo(k) + nb(k)) and holds the "window"
// bits [blo(k), blo(k) + LR); the lane index supplies the remaining bits.  Steps run
// from the top bit down for the forward transform and in the opposite order for the
// inverse.
#pragma once
#include <type_traits>
#include "modarith.hpp"

namespace nttk {

// One limb-vector of a vector-list launch: its residues and the plan limb (prime) it uses.
struct VecDesc {
  uint64_t* ptr;
  const uint64_t* key;   // key-product launches: the key vector this vector is multiplied by
  uint32_t limb;
  uint32_t pad;
};

struct PassArgs {
  uint64_t* data;        // batch base, [n_vec][N] (dense launches)
  const VecDesc* vecs;   // vector list (list launches) or null
  const Tw* tw;          // [L][N] twiddles of this direction (Psi or Psi_inv)
  const Tw* ot_lo;       // [L][B]     psi^{+-k},     k < B       (OT only)
  const Tw* ot_hi;       // [L][N/B]   psi^{+-B*h},   h < N/B     (OT only)
  const uint64_t* q;     // [L]
  const Tw* scale;       // [L][2]: {1/N}, {Psi_inv[1]/N}        (inverse only)
  uint64_t n_vec;        // vectors in the batch (n_polys * L)
  uint32_t P;            // polynomials in the batch
  uint32_t L;
  uint32_t logN;
  uint32_t logN1;        // log2 of the column-pass size (0: single pass)
  uint32_t ot_log2_base; // log2 B
  uint32_t fast;         // every prime below 2^60: the Arith<true> policy applies
  // Dense launches only: the first pass of a forward transform may read its input from
  // `src` (same [n_vec][N] layout) instead of `data` (out of place); null = in place.
  const uint64_t* src;
  // Key-product launches (mul_row): the key vector of vector v is key + v*N (dense) or the
  // list's key pointer, multiplied in with Barrett constants mu[l], bits[l].
  const uint64_t* key;
  const uint64_t* mu;
  const uint32_t* bits;
  // [L][8] per-prime constants {q, 2q, 4q, -q, -2q, -4q, -8q, quotient-estimate constants}
  // (Mod::load).
  // Loaded rather than derived from q in the kernel, so that the compiler adds them as
  // 64-bit operands instead of re-deriving them from q's halves.
  const uint64_t* mc;
  // Tile shape of the split passes (0 = the built-in default): row pass values per lane as
  // log2 (2 or 3) and workgroup lanes (64, 128 or 256); column pass width in adjacent
  // columns (16, 32, 64, 128 or 256).
  uint32_t row_lr;
  uint32_t row_nth;
  uint32_t col_w;
  // Debug modes of the split passes (kDebug* bits, 0 in normal use).
  uint32_t debug;
};

constexpr uint32_t kDebugPoisonLds = 1;      // poison LDS before use
constexpr uint32_t kDebugReverseTiles = 2;   // reverse the workgroup -> tile mapping

// Base address and limb of vector `vec` of a launch: dense [P][L][N] batches place vector
// p*L + l at data + (p*L + l)*N with prime l; list launches read both from the list.
// Residue arrays live in device global memory; addressing them through this type lets
// the compiler emit global (not flat) loads and stores.
typedef __attribute__((address_space(1))) uint64_t gu64;

struct VecRef {
  gu64* base;
  uint32_t limb;
};

__device__ __forceinline__ VecRef vec_ref(const PassArgs& a, uint64_t vec) {
  if (a.vecs) {
    const VecDesc d = a.vecs[vec];
    return VecRef{(gu64*)d.ptr, d.limb};
  }
  return VecRef{(gu64*)(a.data + (vec << a.logN)), (uint32_t)(vec % a.L)};
}

template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    static_for<Begin + 1, End>(f);
  }
}

template <int Begin, int End, typename F>  // counts down: Begin-1, ..., End
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (Begin > End) {
    f(std::integral_constant<int, Begin - 1>{});
    static_for_down<Begin - 1, End>(f);
  }
}

template <int LOGM, int LR_>
struct Steps {
  static constexpr int LR = LR_ < LOGM ? LR_ : LOGM;   // values per lane = 2^LR
  static constexpr int R = 1 << LR;
  static constexpr int K = (LOGM + LR - 1) / LR;       // register steps
  static constexpr int nb(int k) { return k < K - 1 ? LR : LOGM - (K - 1) * LR; }
  static constexpr int blo(int k) { return k < K - 1 ? LOGM - (k + 1) * LR : 0; }
  // element index held by lane t in register u during step k
  template <int k>
  __device__ static __forceinline__ uint32_t idx(uint32_t t, uint32_t u) {
    constexpr int lo = blo(k);
    return ((t >> lo) << (lo + LR)) | (u << lo) | (t & ((1u << lo) - 1u));
  }
};

// On-the-fly twiddling (Section VII): Psi[ix] = psi^{e}, e = brv_logN(ix), is split into
// base-B digits e = e_lo + B * e_hi and applied as two Shoup products with the stored
// factors psi^{e_lo} and psi^{B * e_hi}.
struct OtTables {
  const Tw* lo;
  const Tw* hi;
  uint32_t logN;
  uint32_t b;
  __device__ __forceinline__ void get(uint32_t ix, Tw& a, Tw& c) const {
    const uint32_t e = __brev(ix) >> (32 - logN);
    a = lo[e & ((1u << b) - 1u)];
    c = hi[e >> b];
  }
};

// The twiddles of one register step, loaded into registers before the step runs.
// In stage bit (local index i = bit - blo) the twiddle of a butterfly depends only on the
// lane's window bits above bit i, so the stage needs R >> (i + 1) distinct twiddles and
// the whole step at most R - 1.  Slot of stage i, butterfly k (k-th index with bit i
// clear): off(i) + (k >> i).  Loading them all up front costs one memory round trip per
// step instead of one per stage.
template <int LOGM, int LR, int K_STEP>
struct StepSlots {
  using S = Steps<LOGM, LR>;
  static constexpr int lo = S::blo(K_STEP);
  static constexpr int nb = S::nb(K_STEP);
  static constexpr int R = S::R;
  static constexpr int count(int i) { return R >> (i + 1); }
  static constexpr int off(int i) { return R - (R >> i); }
};

struct NoTw {};   // stand-in for "no preloaded twiddles": gather them stage by stage

template <int LOGM, int LR, int K_STEP, int OTS, int NR, typename TabFn>
__device__ __forceinline__ void load_step_twiddles(Tw (&w)[NR], Tw (&w2)[NR], uint32_t t, uint32_t base,
                                                   TabFn&& tab, const OtTables& ot) {
  using SS = StepSlots<LOGM, LR, K_STEP>;
  using S = typename SS::S;
  static_assert(NR == S::R, "register array size");
  static_for<SS::lo, SS::lo + SS::nb>([&](auto bit_c) {
    constexpr int bit = decltype(bit_c)::value;
    constexpr int s = LOGM - 1 - bit;
    constexpr int i = bit - SS::lo;
#pragma unroll
    for (int j = 0; j < SS::count(i); ++j) {
      const uint32_t r = S::template idx<K_STEP>(t, (uint32_t)(j << (i + 1)));
      const uint32_t ix = (base << s) + (r >> (bit + 1));
      if constexpr (OTS > 0 && s >= LOGM - OTS) ot.get(ix, w[SS::off(i) + j], w2[SS::off(i) + j]);
      else w[SS::off(i) + j] = tab(ix);
    }
  });
}

// Forward (Cooley-Tukey) register step K_STEP on the R values of one lane.
// TabFn(ix) returns the table twiddle Psi[ix]; the last OTS stages of this
// sub-transform take their twiddles from `ot` instead.
// Pre: NoTw, or a struct with arrays w[R], w2[R] filled by load_step_twiddles.
template <bool FAST, int LOGM, int LR, int K_STEP, int OTS, int NR, typename TabFn, typename Pre = NoTw>
__device__ __forceinline__ void ct_step(uint64_t (&x)[NR], uint32_t t, uint32_t base,
                                        TabFn&& tab, const OtTables& ot, const Mod& md, const Pre& pre = Pre{}) {
  constexpr bool PRE = !std::is_same<Pre, NoTw>::value;
  using A = Arith<FAST>;
  using S = Steps<LOGM, LR>;
  static_assert(NR == S::R, "register array size");
  constexpr int lo = S::blo(K_STEP);
  constexpr int nb = S::nb(K_STEP);
  static_for_down<lo + nb, lo>([&](auto bit_c) {
    constexpr int bit = decltype(bit_c)::value;
    constexpr int s = LOGM - 1 - bit;
    constexpr int i = bit - lo;
    if constexpr (FAST) {
      // all R/2 butterflies of the stage at once: twiddles, X reductions, products, outputs
      constexpr int H = S::R / 2;
      Tw w[H], w2[H];
      uint64_t xs[H], ys[H], v[H];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));   // k-th index with bit i clear
        if constexpr (PRE) {
          constexpr int o = StepSlots<LOGM, LR, K_STEP>::off(i);
          w[k] = pre.w[o + (k >> i)];
          if constexpr (OTS > 0 && s >= LOGM - OTS) w2[k] = pre.w2[o + (k >> i)];
        } else {
          const uint32_t r = S::template idx<K_STEP>(t, (uint32_t)u);
          const uint32_t ix = (base << s) + (r >> (bit + 1));
          if constexpr (OTS > 0 && s >= LOGM - OTS) ot.get(ix, w[k], w2[k]);
          else w[k] = tab(ix);
        }
        ys[k] = x[u | (1 << i)];
      }
      // X is reduced by 8q in even stages only: values stay below 16q (see modarith.hpp)
      constexpr bool reduce = (s % 2) == 0;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));
        xs[k] = reduce ? csub_sign(x[u], md.nq8) : x[u];
      }
      A::template mul_n<H>(v, ys, w, md);
      if constexpr (OTS > 0 && s >= LOGM - OTS) A::template mul_n<H>(v, v, w2, md);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));
        x[u] = xs[k] + v[k];
        x[u | (1 << i)] = xs[k] + md.q4 - v[k];
      }
    } else {
#pragma unroll
      for (int u = 0; u < S::R; ++u) {
        if (u & (1 << i)) continue;
        if constexpr (PRE) {
          constexpr int o = StepSlots<LOGM, LR, K_STEP>::off(i);
          if constexpr (OTS > 0 && s >= LOGM - OTS) A::ct2(x[u], x[u | (1 << i)], pre.w[o + (u >> (i + 1))],
                                                           pre.w2[o + (u >> (i + 1))], md);
          else A::ct(x[u], x[u | (1 << i)], pre.w[o + (u >> (i + 1))], md);
          continue;
        }
        const uint32_t r = S::template idx<K_STEP>(t, (uint32_t)u);
        const uint32_t ix = (base << s) + (r >> (bit + 1));
        if constexpr (OTS > 0 && s >= LOGM - OTS) {
          Tw a, c;
          ot.get(ix, a, c);
          A::ct2(x[u], x[u | (1 << i)], a, c, md);
        } else {
          const Tw w = tab(ix);
          A::ct(x[u], x[u | (1 << i)], w, md);
        }
      }
    }
  });
}

// Inverse (Gentleman-Sande) register step K_STEP: stages from the low bit up.
// Value bounds of the fast Gentleman-Sande stages, in multiples of q.  The register step's
// inputs lie below IN_B q (IN_B <= 8).  In the local stage i of a step, register u (bit i
// clear) pairs with u | 2^i; both played the same part in the stage before (bit i-1 of u),
// so they share a bound.  A product is below 4q whatever it multiplied; a sum doubles the
// bound and is reduced by 8q only when that would pass 8q.  So a sum of two products needs
// no reduction, and everything stays below 8q.
template <int IN_B>
struct GsRange {
  static_assert(IN_B >= 1 && IN_B <= 8, "Gentleman-Sande inputs must lie below 8q");
  // bound of register u before local stage i
  static constexpr int before(int i, int u) {
    int b = IN_B;
    for (int j = 0; j < i; ++j) b = (u >> j) & 1 ? 4 : (2 * b > 8 ? 8 : 2 * b);
    return b;
  }
  static constexpr bool reduce(int i, int u) { return 2 * before(i, u) > 8; }
};

// SCALE0: this sub-transform holds stage 0 of the whole transform, whose butterfly
// also applies the 1/N scale (sc0 = 1/N, sc1 = Psi_inv[1]/N).
// IN_B: the step's inputs lie below IN_B q (fast policy; 1 for canonical inputs).
template <bool FAST, int LOGM, int LR, int K_STEP, int OTS, bool SCALE0, int IN_B = 8, int NR, typename TabFn,
          typename Pre = NoTw>
__device__ __forceinline__ void gs_step(uint64_t (&x)[NR], uint32_t t, uint32_t base,
                                        TabFn&& tab, const OtTables& ot, const Mod& md,
                                        const Tw& sc0, const Tw& sc1, const Pre& pre = Pre{}) {
  constexpr bool PRE = !std::is_same<Pre, NoTw>::value;
  using A = Arith<FAST>;
  using S = Steps<LOGM, LR>;
  static_assert(NR == S::R, "register array size");
  constexpr int lo = S::blo(K_STEP);
  constexpr int nb = S::nb(K_STEP);
  static_for<lo, lo + nb>([&](auto bit_c) {
    constexpr int bit = decltype(bit_c)::value;
    constexpr int s = LOGM - 1 - bit;
    constexpr int i = bit - lo;
    if constexpr (FAST && !(SCALE0 && s == 0)) {
      constexpr int H = S::R / 2;
      Tw w[H], w2[H];
      uint64_t ds[H], v[H];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));
        if constexpr (PRE) {
          constexpr int o = StepSlots<LOGM, LR, K_STEP>::off(i);
          w[k] = pre.w[o + (k >> i)];
          if constexpr (OTS > 0 && s >= LOGM - OTS) w2[k] = pre.w2[o + (k >> i)];
        } else {
          const uint32_t r = S::template idx<K_STEP>(t, (uint32_t)u);
          const uint32_t ix = (base << s) + (r >> (bit + 1));
          if constexpr (OTS > 0 && s >= LOGM - OTS) ot.get(ix, w[k], w2[k]);
          else w[k] = tab(ix);
        }
      }
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));
        const uint64_t X = x[u], Y = x[u | (1 << i)];
        const int b = GsRange<IN_B>::before(i, u);   // folded: i and (after unrolling) u are constants
        ds[k] = X + (b == 1 ? md.q : b == 2 ? md.q2 : b == 4 ? md.q4 : md.q8) - Y;
        x[u] = GsRange<IN_B>::reduce(i, u) ? csub_sign(X + Y, md.nq8) : X + Y;
      }
      A::template mul_n<H>(v, ds, w, md);
      if constexpr (OTS > 0 && s >= LOGM - OTS) A::template mul_n<H>(v, v, w2, md);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int u = ((k >> i) << (i + 1)) | (k & ((1 << i) - 1));
        x[u | (1 << i)] = v[k];
      }
    } else {
#pragma unroll
    for (int u = 0; u < S::R; ++u) {
      if (u & (1 << i)) continue;
      if constexpr (SCALE0 && s == 0) {
        A::gs_scaled(x[u], x[u | (1 << i)], sc1, sc0, md);
      } else if constexpr (PRE) {
        constexpr int o = StepSlots<LOGM, LR, K_STEP>::off(i);
        if constexpr (OTS > 0 && s >= LOGM - OTS) A::gs2(x[u], x[u | (1 << i)], pre.w[o + (u >> (i + 1))],
                                                         pre.w2[o + (u >> (i + 1))], md);
        else A::gs(x[u], x[u | (1 << i)], pre.w[o + (u >> (i + 1))], md);
      } else {
        const uint32_t r = S::template idx<K_STEP>(t, (uint32_t)u);
        const uint32_t ix = (base << s) + (r >> (bit + 1));
        if constexpr (OTS > 0 && s >= LOGM - OTS) {
          Tw a, c;
          ot.get(ix, a, c);
          A::gs2(x[u], x[u | (1 << i)], a, c, md);
        } else {
          const Tw w = tab(ix);
          A::gs(x[u], x[u | (1 << i)], w, md);
        }
      }
    }
    }
  });
}

}  // namespace nttk
