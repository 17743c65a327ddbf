// 32-bit words (Section IV's word-size choice taken the other way): primes below 2^30, so
// four times a prime fits a 32-bit word and Harvey's lazy ranges apply to 32-bit values.
// Shoup's product (Algorithm 4) on 32-bit words takes one high and two low 32x32 products:
// qh = hi(b * wb), r = b*w - qh*q mod 2^32, r in [0, 2q) for any b < 2^32.  The same
// modulus budget takes twice the limbs of the 64-bit path, at half the bytes per residue and
// about a third of the integer multiplies per butterfly.
//
// Same two-pass structure as the 64-bit kernels (Section VI-C): a column pass over the first
// log2 N1 stages and a row pass over the rest, each lane running up to LR stages in
// registers between LDS exchanges; N <= 2^12 runs in one row pass.  Data [n_vec][N] uint32,
// vector v reduced mod prime v mod L; tables Tw32 [L][N] (twiddle, companion).
#include "kernels.hpp"
#include "passes.hpp"

namespace nttk {

struct Tw32 {
  uint32_t w, wb;
};

struct Args32 {
  uint32_t* data;
  const Tw32* tw;       // [L][N] of this direction
  const Tw32* scale;    // [L][2]: {1/N}, {Psi_inv[1]/N}
  const uint32_t* q;    // [L]
  uint64_t n_vec;
  uint32_t L, logN, logN1;
};

__device__ __forceinline__ uint32_t mul32(uint32_t b, Tw32 t, uint32_t q) {
  return b * t.w - __umulhi(b, t.wb) * q;   // [0, 2q)
}
__device__ __forceinline__ uint32_t csub32(uint32_t x, uint32_t m) { return x >= m ? x - m : x; }

typedef __attribute__((address_space(1))) uint32_t gu32;

// Forward register step K of an M-point sub-transform (twiddle Psi[(base << s) + j] for local
// stage s, local block j, as in passes.hpp): values in [0, 4q).
template <int LOGM, int LR, int K, int R>
__device__ __forceinline__ void ct32_step(uint32_t (&x)[R], uint32_t t, uint32_t base, const Tw32* tab, uint32_t q) {
  using S = Steps<LOGM, LR>;
  constexpr int lo = S::blo(K), nb = S::nb(K);
  const uint32_t q2 = 2 * q;
  static_for_down<lo + nb, lo>([&](auto bit_c) {
    constexpr int bit = decltype(bit_c)::value;
    constexpr int s = LOGM - 1 - bit;
    constexpr int i = bit - lo;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (u & (1 << i)) continue;
      const uint32_t r = S::template idx<K>(t, (uint32_t)u);
      const Tw32 w = tab[(base << s) + (r >> (bit + 1))];
      const uint32_t X = csub32(x[u], q2);
      const uint32_t v = mul32(x[u | (1 << i)], w, q);
      x[u] = X + v;
      x[u | (1 << i)] = X - v + q2;
    }
  });
}

// Inverse (Gentleman-Sande) register step K: values in [0, 2q); SCALE0: the step holds
// stage 0 of the whole transform, whose butterfly also applies 1/N.
template <int LOGM, int LR, int K, bool SCALE0, int R>
__device__ __forceinline__ void gs32_step(uint32_t (&x)[R], uint32_t t, uint32_t base, const Tw32* tab, uint32_t q,
                                          Tw32 sc0, Tw32 sc1) {
  using S = Steps<LOGM, LR>;
  constexpr int lo = S::blo(K), nb = S::nb(K);
  const uint32_t q2 = 2 * q;
  static_for<lo, lo + nb>([&](auto bit_c) {
    constexpr int bit = decltype(bit_c)::value;
    constexpr int s = LOGM - 1 - bit;
    constexpr int i = bit - lo;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (u & (1 << i)) continue;
      const uint32_t X = x[u], Y = x[u | (1 << i)];
      if constexpr (SCALE0 && s == 0) {
        x[u] = mul32(X + Y, sc0, q);
        x[u | (1 << i)] = mul32(X - Y + q2, sc1, q);
      } else {
        const uint32_t r = S::template idx<K>(t, (uint32_t)u);
        const Tw32 w = tab[(base << s) + (r >> (bit + 1))];
        x[u] = csub32(X + Y, q2);
        x[u | (1 << i)] = mul32(X - Y + q2, w, q);
      }
    }
  });
}

constexpr int kLR32 = 4;          // 16 values per lane: 16 VGPRs of data
constexpr int kRowThreads32 = 128;
constexpr int kColWidth32 = 32;   // 32 adjacent columns: 128-byte row segments

template <int LOGM>
struct Row32 {
  using S = Steps<LOGM, kLR32>;
  static constexpr int M = 1 << LOGM;
  static constexpr int T = M / S::R;
  static constexpr int V = T >= kRowThreads32 ? 1 : kRowThreads32 / T;
  static constexpr int NT = V * T;
  static constexpr int PITCH = M + M / 32;
  static __device__ __forceinline__ uint32_t at(uint32_t r) { return r + (r >> 5); }
};

// Row pass: rows of M = N / N1 contiguous points, V rows per workgroup (SCALE0 / FINAL: the
// pass holds stage 0, i.e. single-pass plans of the inverse).
template <int LOGM, bool INV, bool SCALE0>
__global__ __launch_bounds__(Row32<LOGM>::NT) void row32_kernel(Args32 a) {
  using C = Row32<LOGM>;
  using S = typename C::S;
  __shared__ uint32_t lds[C::V * C::PITCH];
  const uint32_t tid = threadIdx.x, v = tid / C::T, t = tid % C::T;
  const uint64_t rows = a.n_vec << a.logN1;
  const uint64_t g = (uint64_t)blockIdx.x * C::V + v;
  const bool valid = g < rows;
  const uint64_t vec = valid ? g >> a.logN1 : 0;
  const uint32_t row = (uint32_t)(g & ((1u << a.logN1) - 1));
  const uint32_t limb = (uint32_t)(vec % a.L);
  const uint32_t q = a.q[limb];
  const Tw32* tab = a.tw + ((size_t)limb << a.logN);
  const uint32_t base = (1u << a.logN1) + row;
  gu32* rowp = (gu32*)a.data + (vec << a.logN) + (size_t)row * C::M;
  uint32_t* l = lds + v * C::PITCH;
  uint32_t x[S::R];
  constexpr int first = INV ? S::K - 1 : 0;
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = valid ? rowp[S::template idx<first>(t, u)] : 0u;
  if constexpr (!INV) {
    static_for<0, S::K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k > 0) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k - 1>(t, u))] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
      }
      ct32_step<LOGM, kLR32, k>(x, t, base, tab, q);
    });
#pragma unroll
    for (int u = 0; u < S::R; ++u) x[u] = csub32(csub32(x[u], 2 * q), q);
    if constexpr (S::K > 1) {   // back to natural positions so that stores cover whole lines
#pragma unroll
      for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<S::K - 1>(t, u))] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<0>(t, u))];
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
    }
  } else {
    Tw32 sc0{}, sc1{};
    if constexpr (SCALE0) {
      sc0 = a.scale[2 * limb];
      sc1 = a.scale[2 * limb + 1];
    }
    static_for_down<S::K, 0>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k < S::K - 1) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) l[C::at(S::template idx<k + 1>(t, u))] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < S::R; ++u) x[u] = l[C::at(S::template idx<k>(t, u))];
      }
      gs32_step<LOGM, kLR32, k, SCALE0>(x, t, base, tab, q, sc0, sc1);
    });
    if constexpr (SCALE0) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) x[u] = csub32(x[u], q);
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < S::R; ++u) rowp[S::template idx<0>(t, u)] = x[u];
    }
  }
}

template <int LOGM>
struct Col32 {
  using S = Steps<LOGM, kLR32>;
  static constexpr int M = 1 << LOGM;
  static constexpr int T = M / S::R;
  // at most 1024 lanes and 32 KB of LDS per workgroup
  static constexpr int W0 = kColWidth32 * T > 1024 ? 1024 / T : kColWidth32;
  static constexpr int W = W0 * M > 8192 ? 8192 / M : W0;
  static constexpr int NT = W * T;
};

// Column pass: W adjacent columns of one vector per workgroup; the first N1 twiddles in LDS.
template <int LOGM, bool INV>
__global__ __launch_bounds__(Col32<LOGM>::NT) void col32_kernel(Args32 a) {
  using C = Col32<LOGM>;
  using S = typename C::S;
  __shared__ uint32_t lds[C::M * C::W];
  __shared__ Tw32 twl[C::M];
  const uint32_t tid = threadIdx.x, c = tid % C::W, t = tid / C::W;
  const uint32_t logN2 = a.logN - LOGM;
  const uint32_t groups = (1u << logN2) / C::W;
  const uint64_t tile = blockIdx.x;
  if (tile >= a.n_vec * groups) return;   // uniform per workgroup
  const uint64_t vec = tile / groups;
  const uint32_t cg = (uint32_t)(tile % groups);
  const uint32_t limb = (uint32_t)(vec % a.L);
  const uint32_t q = a.q[limb];
  const Tw32* tab = a.tw + ((size_t)limb << a.logN);
  gu32* colp = (gu32*)a.data + (vec << a.logN) + cg * C::W + c;
  uint32_t x[S::R];
  constexpr int first = INV ? S::K - 1 : 0;
#pragma unroll
  for (int u = 0; u < S::R; ++u) x[u] = colp[(size_t)S::template idx<first>(t, u) << logN2];
  for (uint32_t i = tid; i < (uint32_t)C::M; i += C::NT) twl[i] = tab[i];
  __syncthreads();
  if constexpr (!INV) {
    static_for<0, S::K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k > 0) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) lds[S::template idx<k - 1>(t, u) * C::W + c] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < S::R; ++u) x[u] = lds[S::template idx<k>(t, u) * C::W + c];
      }
      ct32_step<LOGM, kLR32, k>(x, t, 1u, twl, q);
    });
#pragma unroll
    for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<S::K - 1>(t, u) << logN2] = x[u];
  } else {
    const Tw32 sc0 = a.scale[2 * limb], sc1 = a.scale[2 * limb + 1];
    static_for_down<S::K, 0>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k < S::K - 1) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) lds[S::template idx<k + 1>(t, u) * C::W + c] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < S::R; ++u) x[u] = lds[S::template idx<k>(t, u) * C::W + c];
      }
      gs32_step<LOGM, kLR32, k, true>(x, t, 1u, twl, q, sc0, sc1);
    });
#pragma unroll
    for (int u = 0; u < S::R; ++u) colp[(size_t)S::template idx<0>(t, u) << logN2] = csub32(x[u], q);
  }
}

template <int LOGM, bool INV, bool SCALE0>
static hipError_t go_row32(const Args32& a, hipStream_t st) {
  using C = Row32<LOGM>;
  const uint64_t rows = a.n_vec << a.logN1;
  hipLaunchKernelGGL((row32_kernel<LOGM, INV, SCALE0>), dim3((uint32_t)((rows + C::V - 1) / C::V)), dim3(C::NT), 0,
                     st, a);
  return hipGetLastError();
}

template <int LOGM, bool INV>
static hipError_t go_col32(const Args32& a, hipStream_t st) {
  using C = Col32<LOGM>;
  const uint64_t blocks = a.n_vec * ((1u << (a.logN - LOGM)) / C::W);
  hipLaunchKernelGGL((col32_kernel<LOGM, INV>), dim3((uint32_t)blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

static hipError_t row32(const Args32& a, int logm, bool inv, bool scale0, hipStream_t st) {
  switch (logm) {
#define X(LM)                                                 \
  case LM:                                                    \
    if (!inv) return go_row32<LM, false, false>(a, st);       \
    return scale0 ? go_row32<LM, true, true>(a, st) : go_row32<LM, true, false>(a, st);
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#undef X
  }
  return hipErrorInvalidValue;
}

static hipError_t col32(const Args32& a, int logm, bool inv, hipStream_t st) {
  switch (logm) {
#define X(LM) \
  case LM:    \
    return inv ? go_col32<LM, true>(a, st) : go_col32<LM, false>(a, st);
    X(5) X(6) X(7) X(8) X(9) X(10)
#undef X
  }
  return hipErrorInvalidValue;
}

// Split N = N1 x N2 with columns of 2^5 .. 2^10 points and rows of 2^5 .. 2^12 points (the
// column tile needs N2 >= 32), or one row pass (N1 = 1) for N <= 2^12.
bool shape32_supported(uint32_t logN, uint32_t logN1) {
  if (logN < 1 || logN > 17) return false;
  if (logN1 == 0) return logN <= 12;
  const uint32_t logN2 = logN - logN1;
  return logN1 >= 5 && logN1 <= 10 && logN2 >= 5 && logN2 <= 12;
}

hipError_t launch_transform32(uint32_t* data, const void* tw, const void* scale, const uint32_t* q, uint64_t n_vec,
                              uint32_t L, uint32_t logN, uint32_t logN1, bool inverse, hipStream_t st) {
  if (!shape32_supported(logN, logN1)) return hipErrorInvalidValue;
  Args32 a{data, static_cast<const Tw32*>(tw), static_cast<const Tw32*>(scale), q, n_vec, L, logN, logN1};
  if (logN1 == 0) return row32(a, (int)logN, inverse, true, st);
  hipError_t e;
  if (!inverse) {
    if ((e = col32(a, (int)logN1, false, st)) != hipSuccess) return e;
    return row32(a, (int)(logN - logN1), false, false, st);
  }
  if ((e = row32(a, (int)(logN - logN1), true, false, st)) != hipSuccess) return e;
  return col32(a, (int)logN1, true, st);
}

// c = a * b mod q_l element-wise over [n_vec][N] uint32 (64-bit product, Barrett with
// mu = floor(2^64 / q): the estimate undershoots by at most 1).
__global__ __launch_bounds__(256) void pointwise32_kernel(const uint32_t* __restrict__ A, const uint32_t* __restrict__ B,
                                                          uint32_t* __restrict__ Cc, const uint32_t* __restrict__ qs,
                                                          const uint64_t* __restrict__ mus, uint64_t n,
                                                          uint32_t logN, uint32_t L) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t limb = (uint32_t)((i >> logN) % L);
    const uint32_t q = qs[limb];
    const uint64_t x = (uint64_t)A[i] * B[i];
    const uint64_t r = x - __umul64hi(x, mus[limb]) * q;
    Cc[i] = csub32((uint32_t)r, q);
  }
}

hipError_t launch_pointwise32(const uint32_t* A, const uint32_t* B, uint32_t* Cc, const uint32_t* qs,
                              const uint64_t* mus, uint64_t n, uint32_t logN, uint32_t L, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pointwise32_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, A, B, Cc, qs, mus, n, logN, L);
  return hipGetLastError();
}

}  // namespace nttk
