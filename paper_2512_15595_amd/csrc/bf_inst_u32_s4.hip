// Kernel variants for 32-bit words, 4 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u32_s4(Registry& r) { register_layout<uint32_t, 4>(r); }
}  // namespace bfhip
