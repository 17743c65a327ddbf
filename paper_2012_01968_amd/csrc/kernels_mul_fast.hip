// Row passes with a key product, primes below 2^60 (estimated quotients).
#include "kernels_impl.hpp"

namespace nttk {
template hipError_t mul_rows<true>(const PassArgs&, const PassArgs&, int, hipStream_t);
}  // namespace nttk
