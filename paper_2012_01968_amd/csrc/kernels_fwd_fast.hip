// Forward NTT kernels, primes below 2^60 (estimated quotients).
#include "kernels_impl.hpp"

namespace nttk {
// row passes: instantiated in kernels_rows.hip
#define X(LM) NTTK_FWD_ROWS(extern, true, LM)
NTTK_ROW_CASES(X)
#undef X
template hipError_t forward_pass<true>(const PassArgs&, int, int, hipStream_t);

bool tiles_supported(uint32_t logN, uint32_t logN1, uint32_t row_lr, uint32_t row_nth, uint32_t col_w) {
  if (row_lr != 0 && row_lr != 2 && row_lr != 3) return false;
  if (row_nth != 0 && row_nth != 64 && row_nth != 128 && row_nth != 256) return false;
  // a row's lanes form one workgroup of at most 1024
  const uint32_t logm = logN - logN1, rlr = row_lr ? row_lr : (uint32_t)row_lr_default(logm);
  if (((1u << logm) >> (rlr < logm ? rlr : logm)) > 1024) return false;
  if (col_w == 0) return true;
  if (col_w != 16 && col_w != 32 && col_w != 64 && col_w != 128 && col_w != 256) return false;
  if (logN1 == 0 || logN1 > logN) return false;   // no column pass
  const uint32_t lr = (uint32_t)kLR < logN1 ? (uint32_t)kLR : logN1;
  const uint32_t t = (1u << logN1) >> lr;          // lanes per column
  const uint32_t w = col_w * t > 1024 ? 1024 / t : col_w;
  return (1u << (logN - logN1)) >= w;
}
}  // namespace nttk
