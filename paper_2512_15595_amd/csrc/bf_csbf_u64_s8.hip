// Cache-sectorized kernel variants for 64-bit words, 8 word(s) per block.
#include "bf_variant_instantiate.hpp"

namespace bfhip {
void register_csbf_u64_s8(VariantRegistry& r) { register_csbf_layout<uint64_t, 8>(r); }
}  // namespace bfhip
