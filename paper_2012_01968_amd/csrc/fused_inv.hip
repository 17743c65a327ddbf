// Fused persistent inverse transform kernels (see fused.hpp).
#include "fused.hpp"

namespace nttk {
template hipError_t fused_dispatch<true>(const FusedArgs&, int, uint32_t, hipStream_t);
}  // namespace nttk
