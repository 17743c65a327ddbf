// Row passes with a key product, primes up to 2^62 (exact quotients).
#include "kernels_impl.hpp"

namespace nttk {
template hipError_t mul_rows<false>(const PassArgs&, const PassArgs&, int, hipStream_t);
}  // namespace nttk
