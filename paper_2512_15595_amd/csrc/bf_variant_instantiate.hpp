// bf_variant_instantiate.hpp -- instantiates the cache-sectorized kernels of
// one (word width, words per block) layout for every valid (z, k, THETA, KT).
#pragma once

#include "bf_partition.hpp"
#include "bf_variant_kernels.hpp"
#include "bf_variant_registry.hpp"

namespace bfhip {

template <typename W, int S_WORDS, int Z, int K, int THETA, int KT>
void register_csbf_one(VariantRegistry& r) {
  constexpr bool kShapeOk = Z <= S_WORDS && THETA <= Z && (KT == 1 || THETA == 1);
  constexpr bool kKOk = K == 0 ? (THETA == 1 && KT == 1) : (K % Z == 0 && K >= Z);
  if constexpr (kShapeOk && kKOk) {
    constexpr int kBits = 8 * static_cast<int>(sizeof(W));
    r.csbf[csbf_index(kOpAdd, kBits, S_WORDS, Z, k_index(K), THETA, KT)] =
        reinterpret_cast<const void*>(&csbf_add_kernel<W, S_WORDS, Z, K, THETA, KT>);
    r.csbf[csbf_index(kOpContains, kBits, S_WORDS, Z, k_index(K), THETA, KT)] =
        reinterpret_cast<const void*>(&csbf_contains_kernel<W, S_WORDS, Z, K, THETA, KT>);
  }
}

template <typename W, int S_WORDS, int Z, int K>
void register_csbf_part(VariantRegistry& r) {
  if constexpr (Z <= S_WORDS && (K == 0 || (K % Z == 0 && K >= Z))) {
    constexpr int kBits = 8 * static_cast<int>(sizeof(W));
    const int idx = csbf_part_index(kBits, S_WORDS, Z, k_index(K));
    r.csbf_part1[idx] = reinterpret_cast<const void*>(&part_scatter1_kernel<W, S_WORDS, K, Z>);
    r.csbf_part1_chunk[idx] = reinterpret_cast<const void*>(&part_scatter1_kernel<W, S_WORDS, K, Z, false, true>);
    r.csbf_part2[idx] = reinterpret_cast<const void*>(&part_scatter2_kernel<W, S_WORDS, K, Z>);
    r.csbf_apply[idx] = reinterpret_cast<const void*>(&part_apply_kernel<W, S_WORDS, K, Z>);
  }
}

template <typename W, int S_WORDS, int Z, int K>
void register_csbf_theta(VariantRegistry& r) {
  register_csbf_part<W, S_WORDS, Z, K>(r);
  register_csbf_one<W, S_WORDS, Z, K, 1, 1>(r);
  register_csbf_one<W, S_WORDS, Z, K, 1, 2>(r);
  register_csbf_one<W, S_WORDS, Z, K, 2, 1>(r);
  register_csbf_one<W, S_WORDS, Z, K, 4, 1>(r);
  register_csbf_one<W, S_WORDS, Z, K, 8, 1>(r);
  register_csbf_one<W, S_WORDS, Z, K, 16, 1>(r);
}

template <typename W, int S_WORDS, int Z>
void register_csbf_k(VariantRegistry& r) {
  register_csbf_theta<W, S_WORDS, Z, 0>(r);
  register_csbf_theta<W, S_WORDS, Z, 4>(r);
  register_csbf_theta<W, S_WORDS, Z, 6>(r);
  register_csbf_theta<W, S_WORDS, Z, 8>(r);
  register_csbf_theta<W, S_WORDS, Z, 12>(r);
  register_csbf_theta<W, S_WORDS, Z, 16>(r);
}

template <typename W, int S_WORDS>
void register_csbf_layout(VariantRegistry& r) {
  register_csbf_k<W, S_WORDS, 1>(r);
  register_csbf_k<W, S_WORDS, 2>(r);
  register_csbf_k<W, S_WORDS, 4>(r);
  register_csbf_k<W, S_WORDS, 8>(r);
  register_csbf_k<W, S_WORDS, 16>(r);
}

}  // namespace bfhip
