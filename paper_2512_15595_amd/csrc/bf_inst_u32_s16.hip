// Kernel variants for 32-bit words, 16 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u32_s16(Registry& r) { register_layout<uint32_t, 16>(r); }
}  // namespace bfhip
