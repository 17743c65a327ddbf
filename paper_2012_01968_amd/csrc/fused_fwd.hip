// Fused persistent forward transform kernels (see fused.hpp).
#include "fused.hpp"

namespace nttk {
template hipError_t fused_dispatch<false>(const FusedArgs&, int, uint32_t, hipStream_t);
}  // namespace nttk
