// Split-precision fused MTTKRP (bfloat16 x3 products, float32 accumulation
// flushed to float64).  Variants are registered below.
#include "jkc_internal.hpp"

namespace jkc {

const std::vector<MttkrpVariant>& mttkrp_split_variants() {
  static const std::vector<MttkrpVariant> v = {};
  return v;
}

}  // namespace jkc
