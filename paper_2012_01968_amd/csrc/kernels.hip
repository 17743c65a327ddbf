// NTT launch entry points (host) and the element-wise product kernel.
#include "kernels.hpp"
#include "passes.hpp"
#include "fused_args.hpp"

namespace nttk {

template <bool FAST>
hipError_t forward_pass(const PassArgs& a, int ots, int pass, hipStream_t st);
template <bool FAST>
hipError_t inverse_pass(const PassArgs& a, int ots, int pass, hipStream_t st);
template <bool FAST>
hipError_t mul_rows(const PassArgs& af, const PassArgs& ai, int ots, hipStream_t st);
extern template hipError_t forward_pass<true>(const PassArgs&, int, int, hipStream_t);
extern template hipError_t forward_pass<false>(const PassArgs&, int, int, hipStream_t);
extern template hipError_t inverse_pass<true>(const PassArgs&, int, int, hipStream_t);
extern template hipError_t inverse_pass<false>(const PassArgs&, int, int, hipStream_t);
extern template hipError_t mul_rows<true>(const PassArgs&, const PassArgs&, int, hipStream_t);
extern template hipError_t mul_rows<false>(const PassArgs&, const PassArgs&, int, hipStream_t);

// ------------------------------------------------------------------------ element-wise
// c = a * b mod q_l over a [n_vec][N] batch, two elements per lane per iteration.
__global__ __launch_bounds__(256) void pointwise_kernel(const uint64_t* __restrict__ A, const uint64_t* __restrict__ B,
                                                        uint64_t* __restrict__ Cc, const uint64_t* __restrict__ qs,
                                                        const uint64_t* __restrict__ mus,
                                                        const uint32_t* __restrict__ bits, uint64_t n_pairs,
                                                        uint32_t logN, uint32_t L) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pairs;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = i << 1;
    const uint32_t limb = (uint32_t)((e >> logN) % L);
    const uint64_t q = qs[limb], mu = mus[limb];
    const uint32_t s = bits[limb];
    const ulonglong2 va = reinterpret_cast<const ulonglong2*>(A)[i];
    const ulonglong2 vb = reinterpret_cast<const ulonglong2*>(B)[i];
    ulonglong2 vc;
    vc.x = mulmod_barrett(va.x, vb.x, q, mu, s);
    vc.y = mulmod_barrett(va.y, vb.y, q, mu, s);
    reinterpret_cast<ulonglong2*>(Cc)[i] = vc;
  }
}

// Key product over a vector list: vector i (N residues at vecs[i].ptr, prime vecs[i].limb)
// is replaced by its element-wise product with vecs[i].key.
__global__ __launch_bounds__(256) void pointwise_list_kernel(const VecDesc* __restrict__ vecs, uint64_t n_pairs,
                                                             uint32_t logN, const uint64_t* __restrict__ qs,
                                                             const uint64_t* __restrict__ mus,
                                                             const uint32_t* __restrict__ bits) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pairs;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = i << 1;
    const VecDesc d = vecs[e >> logN];
    const uint64_t off = e & ((1ull << logN) - 1);
    const uint64_t q = qs[d.limb], mu = mus[d.limb];
    const uint32_t s = bits[d.limb];
    const ulonglong2 va = *reinterpret_cast<const ulonglong2*>(d.ptr + off);
    const ulonglong2 vk = *reinterpret_cast<const ulonglong2*>(d.key + off);
    ulonglong2 vc;
    vc.x = mulmod_barrett(va.x, vk.x, q, mu, s);
    vc.y = mulmod_barrett(va.y, vk.y, q, mu, s);
    *reinterpret_cast<ulonglong2*>(d.ptr + off) = vc;
  }
}

bool shape_supported(uint32_t logN, uint32_t logN1, int ots) {
  if (logN < 1 || logN > 17) return false;
  if (logN1 == 0) {
    if (logN > 13) return false;
    return ots <= 2 && (ots == 0 || (int)logN >= ots + 1);
  }
  if (logN1 < 4 || logN1 > 10) return false;
  const uint32_t logN2 = logN - logN1;
  if (logN2 < 4 || logN2 > 13) return false;   // column groups of 16 need N2 >= 16
  return ots >= 0 && ots <= 2 && (int)logN2 > ots;
}

hipError_t launch_forward_pass(const PassArgs& a, int ots, int pass, hipStream_t st) {
  if (!shape_supported(a.logN, a.logN1, ots)) return hipErrorInvalidValue;
  return a.fast ? forward_pass<true>(a, ots, pass, st) : forward_pass<false>(a, ots, pass, st);
}

hipError_t launch_inverse_pass(const PassArgs& a, int ots, int pass, hipStream_t st) {
  if (!shape_supported(a.logN, a.logN1, ots)) return hipErrorInvalidValue;
  return a.fast ? inverse_pass<true>(a, ots, pass, st) : inverse_pass<false>(a, ots, pass, st);
}

hipError_t launch_mul_rows(const PassArgs& af, const PassArgs& ai, int ots, hipStream_t st) {
  if (!shape_supported(af.logN, af.logN1, ots)) return hipErrorInvalidValue;
  return af.fast ? mul_rows<true>(af, ai, ots, st) : mul_rows<false>(af, ai, ots, st);
}

hipError_t launch_forward(const PassArgs& a, int ots, hipStream_t st) {
  const int passes = a.logN1 ? 2 : 1;
  for (int p = 0; p < passes; ++p) {
    const hipError_t e = launch_forward_pass(a, ots, p, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_inverse(const PassArgs& a, int ots, hipStream_t st) {
  const int passes = a.logN1 ? 2 : 1;
  for (int p = 0; p < passes; ++p) {
    const hipError_t e = launch_inverse_pass(a, ots, p, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool INV>
hipError_t fused_dispatch(const FusedArgs& f, int ots, uint32_t max_grid, hipStream_t st);
extern template hipError_t fused_dispatch<false>(const FusedArgs&, int, uint32_t, hipStream_t);
extern template hipError_t fused_dispatch<true>(const FusedArgs&, int, uint32_t, hipStream_t);

bool fused_supported(uint32_t logN, uint32_t logN1, int ots) {
  if (ots < 0 || ots > 2) return false;
  const uint32_t n2 = logN - logN1;
  return (logN1 == 6 && n2 == 7) || (logN1 == 7 && n2 == 7) || (logN1 == 7 && n2 == 8) ||
         (logN1 == 8 && n2 == 8) || (logN1 == 8 && n2 == 9);
}

hipError_t launch_fused(const PassArgs& a, int ots, bool inverse, uint32_t* ctr, uint32_t n_polys, uint32_t lag,
                        uint32_t max_grid, hipStream_t st) {
  if (!a.fast || !fused_supported(a.logN, a.logN1, ots)) return hipErrorInvalidValue;
  FusedArgs f;
  f.a = a;
  f.ctr = ctr;
  f.P = n_polys;
  f.lag = lag;
  return inverse ? fused_dispatch<true>(f, ots, max_grid, st) : fused_dispatch<false>(f, ots, max_grid, st);
}

hipError_t launch_pointwise_list(const VecDesc* vecs, uint64_t n_vec, uint32_t logN, const uint64_t* qs,
                                 const uint64_t* mus, const uint32_t* bits, hipStream_t st) {
  const uint64_t pairs = (n_vec << logN) / 2;   // N >= 2: whole pairs per vector
  if (pairs == 0) return hipSuccess;
  uint64_t blocks = (pairs + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pointwise_list_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, vecs, pairs, logN, qs, mus, bits);
  return hipGetLastError();
}

hipError_t launch_pointwise(const uint64_t* A, const uint64_t* B, uint64_t* Cc, const uint64_t* qs,
                            const uint64_t* mus, const uint32_t* bits, uint64_t n_elems, uint32_t logN,
                            uint32_t L, hipStream_t st) {
  const uint64_t pairs = n_elems / 2;   // N >= 2, so every vector holds whole pairs
  if (pairs == 0) return hipSuccess;
  uint64_t blocks = (pairs + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pointwise_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, A, B, Cc, qs, mus, bits, pairs,
                     logN, L);
  return hipGetLastError();
}

}  // namespace nttk
