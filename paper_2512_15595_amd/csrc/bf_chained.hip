// Kernels of the sectorized filter with chained pattern hashing, every
// (word width, words per block, k) and both operations.
#include "bf_variant_kernels.hpp"
#include "bf_variant_registry.hpp"

namespace bfhip {
namespace {

template <typename W, int S_WORDS, int K>
void register_chained_one(VariantRegistry& r) {
  if constexpr (K == 0 || K >= S_WORDS) {
    constexpr int kBits = 8 * static_cast<int>(sizeof(W));
    r.chained[chained_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&chained_kernel<W, S_WORDS, K, kOpAdd>);
    r.chained[chained_index(kOpContains, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&chained_kernel<W, S_WORDS, K, kOpContains>);
  }
}

template <typename W, int S_WORDS>
void register_chained_k(VariantRegistry& r) {
  register_chained_one<W, S_WORDS, 0>(r);
  register_chained_one<W, S_WORDS, 4>(r);
  register_chained_one<W, S_WORDS, 6>(r);
  register_chained_one<W, S_WORDS, 8>(r);
  register_chained_one<W, S_WORDS, 12>(r);
  register_chained_one<W, S_WORDS, 16>(r);
}

template <typename W>
void register_chained_s(VariantRegistry& r) {
  register_chained_k<W, 1>(r);
  register_chained_k<W, 2>(r);
  register_chained_k<W, 4>(r);
  register_chained_k<W, 8>(r);
  register_chained_k<W, 16>(r);
}

}  // namespace

void register_chained(VariantRegistry& r) {
  register_chained_s<uint32_t>(r);
  register_chained_s<uint64_t>(r);
}

}  // namespace bfhip
