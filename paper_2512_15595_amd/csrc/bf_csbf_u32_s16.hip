// Cache-sectorized kernel variants for 32-bit words, 16 word(s) per block.
#include "bf_variant_instantiate.hpp"

namespace bfhip {
void register_csbf_u32_s16(VariantRegistry& r) { register_csbf_layout<uint32_t, 16>(r); }
}  // namespace bfhip
