// Kernel variants for 32-bit words, 8 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u32_s8(Registry& r) { register_layout<uint32_t, 8>(r); }
}  // namespace bfhip
