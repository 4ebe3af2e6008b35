// Cache-sectorized kernel variants for 64-bit words, 16 word(s) per block.
#include "bf_variant_instantiate.hpp"

namespace bfhip {
void register_csbf_u64_s16(VariantRegistry& r) { register_csbf_layout<uint64_t, 16>(r); }
}  // namespace bfhip
