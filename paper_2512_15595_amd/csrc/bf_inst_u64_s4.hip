// Kernel variants for 64-bit words, 4 word(s) per block.
#include "bf_instantiate.hpp"

namespace bfhip {
void register_u64_s4(Registry& r) { register_layout<uint64_t, 4>(r); }
}  // namespace bfhip
