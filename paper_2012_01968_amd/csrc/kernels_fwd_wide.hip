// Forward NTT kernels, primes below 2^62 (exact quotients).
#include "kernels_impl.hpp"

namespace nttk {
template hipError_t forward_pass<false>(const PassArgs&, int, int, hipStream_t);
}  // namespace nttk
