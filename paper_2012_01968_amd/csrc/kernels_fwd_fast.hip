// Forward NTT kernels, primes below 2^60 (estimated quotients).
#include "kernels_impl.hpp"

namespace nttk {
template hipError_t forward_pass<true>(const PassArgs&, int, int, hipStream_t);
}  // namespace nttk
