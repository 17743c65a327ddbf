// Row passes with a key product, primes below 2^60 (estimated quotients).
#include "kernels_impl.hpp"

namespace nttk {
// row passes: instantiated in kernels_rows.hip
#define X(LM) NTTK_MUL_ROWS(extern, true, LM)
NTTK_ROW_CASES(X)
#undef X
template hipError_t mul_rows<true>(const PassArgs&, const PassArgs&, int, hipStream_t);
}  // namespace nttk
