// Cache-sectorized kernel variants for 32-bit words, 4 word(s) per block.
#include "bf_variant_instantiate.hpp"

namespace bfhip {
void register_csbf_u32_s4(VariantRegistry& r) { register_csbf_layout<uint32_t, 4>(r); }
}  // namespace bfhip
