// RNS <-> integer conversion on either side of the transform (Section III-B): an integer
// coefficient below Q = q_0 ... q_{L-1} is held as its L residues.  Integers are stored as
// little-endian 64-bit words, word-major: word w of coefficient c of polynomial p sits at
// (p*W + w)*N + c, so the lanes of a wave (consecutive coefficients) read consecutive words.
// The tables come from crt_math.hpp (host).
#include "kernels.hpp"
#include "passes.hpp"

namespace nttk {

// b * w mod q in [0, 2q) for any b < 2^64, q < 2^62 (Shoup with the exact quotient).
__device__ __forceinline__ uint64_t shoup_exact(uint64_t b, uint64_t w, uint64_t wb, uint64_t q) {
  return b * w - __umul64hi(b, wb) * q;
}

// residue l of coefficient c:  sum_w x_w * (2^(64 w) mod q_l)  mod q_l
__global__ __launch_bounds__(256) void rns_decompose_kernel(const uint64_t* __restrict__ words, uint32_t W,
                                                            uint64_t* __restrict__ res, uint64_t n_coeffs,
                                                            uint32_t logN, uint32_t L,
                                                            const Tw* __restrict__ pow2, uint32_t pow2_stride,
                                                            const uint64_t* __restrict__ qs) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t l = blockIdx.y;
  if (j >= n_coeffs) return;
  const uint64_t N = 1ull << logN;
  const uint64_t p = j >> logN, c = j & (N - 1);
  const uint64_t q = qs[l], q2 = q << 1;
  const Tw* t = pow2 + (size_t)l * pow2_stride;
  const uint64_t* x = words + p * W * N + c;
  uint64_t acc = 0;
  for (uint32_t w = 0; w < W; ++w) {
    const Tw tw = t[w];
    acc += shoup_exact(x[(size_t)w * N], tw.w, tw.wb, q);   // < 4q
    acc = csub(acc, q2);                                     // < 2q
  }
  res[(p * L + l) * N + c] = csub(acc, q);
}

constexpr int kCrtThreads = 64;

// One coefficient per lane.  y_l = r_l * inv_l mod q_l goes to the lane's LDS column; then
// x' = sum_l y_l M_l is formed word by word (product scanning: column w collects the low
// words of y_l M_l[w] and the high words of y_l M_l[w-1] in a 192-bit accumulator) and
// written out; finally the largest multiple kQ <= x' (k < L) is found by binary search from
// the top words and subtracted, leaving x in [0, Q).
__global__ __launch_bounds__(kCrtThreads) void crt_reconstruct_kernel(const uint64_t* __restrict__ res,
                                                                      uint64_t* __restrict__ out, uint64_t n_coeffs,
                                                                      uint32_t logN, uint32_t L, uint32_t W,
                                                                      const Tw* __restrict__ inv,
                                                                      const uint64_t* __restrict__ M,
                                                                      const uint64_t* __restrict__ kQ,
                                                                      const uint64_t* __restrict__ qs) {
  extern __shared__ uint64_t ys[];   // [L][kCrtThreads]
  const uint64_t j = (uint64_t)blockIdx.x * kCrtThreads + threadIdx.x;
  if (j >= n_coeffs) return;         // no barrier below: each lane uses only its own column
  const uint64_t N = 1ull << logN;
  const uint64_t p = j >> logN, c = j & (N - 1);
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t q = qs[l];
    const Tw t = inv[l];
    ys[l * kCrtThreads + threadIdx.x] = csub(shoup_exact(res[(p * L + l) * N + c], t.w, t.wb, q), q);
  }
  uint64_t* o = out + p * W * N + c;
  uint64_t c0 = 0, c1 = 0, c2 = 0;   // column w
  uint64_t n0 = 0, n1 = 0, n2 = 0;   // column w + 1
  for (uint32_t w = 0; w < W; ++w) {
    for (uint32_t l = 0; l < L; ++l) {
      const uint64_t y = ys[l * kCrtThreads + threadIdx.x], m = M[(size_t)l * W + w];
      const uint64_t lo = y * m, hi = __umul64hi(y, m);
      c0 += lo;
      const uint64_t k0 = c0 < lo;
      c1 += k0;
      c2 += c1 < k0;
      n0 += hi;
      const uint64_t k1 = n0 < hi;
      n1 += k1;
      n2 += n1 < k1;
    }
    o[(size_t)w * N] = c0;
    // the next column takes the carries of this one
    c0 = n0 + c1;
    const uint64_t k0 = c0 < c1;
    const uint64_t t1 = n1 + c2;
    const uint64_t k1 = t1 < c2;
    c1 = t1 + k0;
    c2 = n2 + k1 + (c1 < k0);
    n0 = n1 = n2 = 0;
  }
  const uint64_t top = c0;           // word W of x' (x' < L Q < 2^(64 W + 64))
  // largest k with kQ[k] <= x', k in [0, L - 1]
  uint32_t lo = 0, hi = L - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    const uint64_t* kq = kQ + (size_t)mid * (W + 1);
    int cmp = top > kq[W] ? 1 : (top < kq[W] ? -1 : 0);
    for (uint32_t w = W; cmp == 0 && w-- > 0;) {
      const uint64_t xw = o[(size_t)w * N];
      cmp = xw > kq[w] ? 1 : (xw < kq[w] ? -1 : 0);
    }
    if (cmp >= 0) lo = mid;
    else hi = mid - 1;
  }
  const uint64_t* kq = kQ + (size_t)lo * (W + 1);
  uint64_t borrow = 0;
  for (uint32_t w = 0; w < W; ++w) {
    const uint64_t xw = o[(size_t)w * N], s = kq[w];
    const uint64_t d = xw - s;
    const uint64_t b1 = xw < s;
    const uint64_t d2 = d - borrow;
    const uint64_t b2 = d < borrow;
    o[(size_t)w * N] = d2;
    borrow = b1 | b2;
  }
}

hipError_t launch_rns_decompose(const uint64_t* words, uint32_t W, uint64_t* res, uint32_t n_polys, uint32_t logN,
                                uint32_t L, const Tw* pow2, uint32_t pow2_stride, const uint64_t* qs, hipStream_t st) {
  const uint64_t n = (uint64_t)n_polys << logN;
  const dim3 grid((uint32_t)((n + 255) / 256), L);
  hipLaunchKernelGGL(rns_decompose_kernel, grid, dim3(256), 0, st, words, W, res, n, logN, L, pow2, pow2_stride, qs);
  return hipGetLastError();
}

hipError_t launch_crt_reconstruct(const uint64_t* res, uint64_t* out, uint32_t n_polys, uint32_t logN, uint32_t L,
                                  uint32_t W, const Tw* inv, const uint64_t* M, const uint64_t* kQ, const uint64_t* qs,
                                  hipStream_t st) {
  const uint64_t n = (uint64_t)n_polys << logN;
  const size_t lds = (size_t)L * kCrtThreads * sizeof(uint64_t);
  hipLaunchKernelGGL(crt_reconstruct_kernel, dim3((uint32_t)((n + kCrtThreads - 1) / kCrtThreads)),
                     dim3(kCrtThreads), lds, st, res, out, n, logN, L, W, inv, M, kQ, qs);
  return hipGetLastError();
}

}  // namespace nttk
