// Arguments of the fused persistent transform kernel.
#pragma once
#include "passes.hpp"

namespace nttk {

struct FusedArgs {
  PassArgs a;
  uint32_t* ctr;    // [0..7] XCD queue heads, [8] exit count, [16 + v] per-vector completion counts
  uint32_t P;       // polynomials in the batch
  uint32_t lag;     // how many vectors' first-pass tiles an XCD queue runs ahead
};

}  // namespace nttk
