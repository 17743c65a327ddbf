// Device copy in one pass, one 16-byte vector per lane: the memory-rate yardstick that the
// measurement compares the transform's passes with.  No plan launches it, so it is left out of
// the kernel source hash (build.py) that keys tuned choices and counters.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy16_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// n16 vectors of 16 bytes; the grid's lanes (blocks * 256) must stay below 2^32.
hipError_t launch_copy16(const void* src, void* dst, uint64_t n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const uint64_t blocks = (n16 + 255) / 256;
  if (blocks * 256 >= (1ull << 32)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy16_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, (const v4u*)src, (v4u*)dst, n16);
  return hipGetLastError();
}

}  // namespace nttk
