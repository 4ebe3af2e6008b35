// Cache-sectorized kernel variants for 64-bit words, 4 word(s) per block.
#include "bf_variant_instantiate.hpp"

namespace bfhip {
void register_csbf_u64_s4(VariantRegistry& r) { register_csbf_layout<uint64_t, 4>(r); }
}  // namespace bfhip
