// Kernel variants for 32-bit words, 2 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u32_s2(Registry& r) { register_layout<uint32_t, 2>(r); }
}  // namespace bfhip
