// Row passes with a key product, primes up to 2^62 (exact quotients).
#include "kernels_impl.hpp"

namespace nttk {
// row passes: instantiated in kernels_rows.hip
#define X(LM) NTTK_MUL_ROWS(extern, false, LM)
NTTK_ROW_CASES(X)
#undef X
template hipError_t mul_rows<false>(const PassArgs&, const PassArgs&, int, hipStream_t);
}  // namespace nttk
