// Kernel variants for 64-bit words, 2 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u64_s2(Registry& r) { register_layout<uint64_t, 2>(r); }
}  // namespace bfhip
