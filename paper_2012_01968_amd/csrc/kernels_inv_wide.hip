// Inverse NTT kernels, primes below 2^62 (exact quotients).
#include "kernels_impl.hpp"

namespace nttk {
// row passes: instantiated in kernels_rows.hip
#define X(LM) NTTK_INV_ROWS(extern, false, LM)
NTTK_ROW_CASES(X)
#undef X
template hipError_t inverse_pass<false>(const PassArgs&, int, int, hipStream_t);
}  // namespace nttk
