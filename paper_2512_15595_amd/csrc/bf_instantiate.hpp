// bf_instantiate.hpp -- instantiates every kernel variant of one (W, s) layout.
#pragma once

#include <utility>

#include "bf_batch_kernels.hpp"
#include "bf_kernels.hpp"
#include "bf_partition.hpp"
#include "bf_registry.hpp"

namespace bfhip {

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT>
void register_one(Registry& r) {
  constexpr int kBits = 8 * static_cast<int>(sizeof(W));
  constexpr int kIdx = k_index(K);
  if constexpr (THETA * PHI <= S_WORDS && THETA <= 16 && (K == 0 || K >= S_WORDS)) {
    r.fn[registry_index(kOpContains, kBits, S_WORDS, kIdx, THETA, PHI, KT, 0)] =
        reinterpret_cast<const void*>(&bf_contains_kernel<W, S_WORDS, K, THETA, PHI, KT>);
    r.fn[registry_index(kOpAdd, kBits, S_WORDS, kIdx, THETA, PHI, KT, 0)] =
        reinterpret_cast<const void*>(&bf_add_kernel<W, S_WORDS, K, THETA, PHI, KT, false>);
    if constexpr (sizeof(W) == 4 && PHI >= 2) {
      r.fn[registry_index(kOpAdd, kBits, S_WORDS, kIdx, THETA, PHI, KT, 1)] =
          reinterpret_cast<const void*>(&bf_add_kernel<W, S_WORDS, K, THETA, PHI, KT, true>);
    }
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI>
void register_kt(Registry& r) {
  register_one<W, S_WORDS, K, THETA, PHI, 1>(r);
  if constexpr (K != 0) {
    register_one<W, S_WORDS, K, THETA, PHI, 2>(r);
    register_one<W, S_WORDS, K, THETA, PHI, 4>(r);
  }
}

template <typename W, int S_WORDS, int K, int THETA>
void register_phi(Registry& r) {
  register_kt<W, S_WORDS, K, THETA, 1>(r);
  register_kt<W, S_WORDS, K, THETA, 2>(r);
  register_kt<W, S_WORDS, K, THETA, 4>(r);
  register_kt<W, S_WORDS, K, THETA, 8>(r);
  register_kt<W, S_WORDS, K, THETA, 16>(r);
}

template <typename W, int S_WORDS, int K>
void register_theta(Registry& r) {
  register_phi<W, S_WORDS, K, 1>(r);
  if constexpr (K != 0) {
    register_phi<W, S_WORDS, K, 2>(r);
    register_phi<W, S_WORDS, K, 4>(r);
    register_phi<W, S_WORDS, K, 8>(r);
    register_phi<W, S_WORDS, K, 16>(r);
  }
}

template <typename W, int S_WORDS, int K>
void register_batch(Registry& r) {
  constexpr int kBits = 8 * static_cast<int>(sizeof(W));
  if constexpr (K == 0 || K >= S_WORDS) {
    r.batch_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&bf_batch_kernel<W, S_WORDS, K, kOpAdd>);
    r.batch_fn[batch_index(kOpContains, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&bf_batch_kernel<W, S_WORDS, K, kOpContains>);
    r.part1_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&part_scatter1_kernel<W, S_WORDS, K>);
    r.part1_multi_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&part_scatter1_kernel<W, S_WORDS, K, 0, true>);
    r.part1_chunk_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&part_scatter1_kernel<W, S_WORDS, K, 0, false, true>);
    r.part2_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&part_scatter2_kernel<W, S_WORDS, K>);
    r.apply_fn[batch_index(kOpAdd, kBits, S_WORDS, k_index(K))] =
        reinterpret_cast<const void*>(&part_apply_kernel<W, S_WORDS, K>);
  }
}

template <typename W, int S_WORDS>
void register_layout(Registry& r) {
  register_batch<W, S_WORDS, 0>(r);
  register_batch<W, S_WORDS, 4>(r);
  register_batch<W, S_WORDS, 6>(r);
  register_batch<W, S_WORDS, 8>(r);
  register_batch<W, S_WORDS, 12>(r);
  register_batch<W, S_WORDS, 16>(r);
  register_theta<W, S_WORDS, 0>(r);
  register_theta<W, S_WORDS, 4>(r);
  register_theta<W, S_WORDS, 6>(r);
  register_theta<W, S_WORDS, 8>(r);
  register_theta<W, S_WORDS, 12>(r);
  register_theta<W, S_WORDS, 16>(r);
}

}  // namespace bfhip
