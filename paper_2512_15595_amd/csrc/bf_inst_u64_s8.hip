// Kernel variants for 64-bit words, 8 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u64_s8(Registry& r) { register_layout<uint64_t, 8>(r); }
}  // namespace bfhip
