// Kernel variants for 64-bit words, 1 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u64_s1(Registry& r) { register_layout<uint64_t, 1>(r); }
}  // namespace bfhip
