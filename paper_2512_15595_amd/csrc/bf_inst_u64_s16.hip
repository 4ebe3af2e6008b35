// Kernel variants for 64-bit words, 16 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u64_s16(Registry& r) { register_layout<uint64_t, 16>(r); }
}  // namespace bfhip
