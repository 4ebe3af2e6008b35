// Kernel variants for 32-bit words, 1 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u32_s1(Registry& r) { register_layout<uint32_t, 1>(r); }
}  // namespace bfhip
