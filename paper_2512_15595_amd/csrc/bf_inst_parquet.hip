// Kernel variants of the Parquet split-block filter (bf_parquet.h): every
// mapping of the sectorized 8 x 32-bit, k = 8 layout, in the same registry
// slots, the persistent batched kernels, and the partitioned-construction
// kernels (single-filter and multi-filter first pass).
#include <utility>

#include "bf_parquet.hpp"
#include "bf_registry.hpp"

namespace bfhip {
namespace {

constexpr int kIdxK = k_index(kParquetK);

template <int THETA, int PHI, int KT>
void register_one(Registry& r) {
  if constexpr (THETA * PHI <= kParquetWords) {
    r.fn[registry_index(kOpContains, 32, kParquetWords, kIdxK, THETA, PHI, KT, 0)] =
        reinterpret_cast<const void*>(&parquet_contains_kernel<THETA, PHI, KT>);
    r.fn[registry_index(kOpAdd, 32, kParquetWords, kIdxK, THETA, PHI, KT, 0)] =
        reinterpret_cast<const void*>(&parquet_add_kernel<THETA, PHI, KT, false>);
    if constexpr (PHI >= 2)
      r.fn[registry_index(kOpAdd, 32, kParquetWords, kIdxK, THETA, PHI, KT, 1)] =
          reinterpret_cast<const void*>(&parquet_add_kernel<THETA, PHI, KT, true>);
  }
}

template <int THETA, int PHI>
void register_kt(Registry& r) {
  register_one<THETA, PHI, 1>(r);
  register_one<THETA, PHI, 2>(r);
  register_one<THETA, PHI, 4>(r);
}

template <int THETA>
void register_phi(Registry& r) {
  register_kt<THETA, 1>(r);
  register_kt<THETA, 2>(r);
  register_kt<THETA, 4>(r);
  register_kt<THETA, 8>(r);
}

}  // namespace

void register_parquet(Registry& r) {
  register_phi<1>(r);
  register_phi<2>(r);
  register_phi<4>(r);
  register_phi<8>(r);
  r.batch_fn[batch_index(kOpAdd, 32, kParquetWords, kIdxK)] =
      reinterpret_cast<const void*>(&parquet_batch_kernel<kOpAdd>);
  r.batch_fn[batch_index(kOpContains, 32, kParquetWords, kIdxK)] =
      reinterpret_cast<const void*>(&parquet_batch_kernel<kOpContains>);
  const int slot = batch_index(kOpAdd, 32, kParquetWords, kIdxK);
  r.part1_fn[slot] =
      reinterpret_cast<const void*>(&part_scatter1_kernel<uint32_t, kParquetWords, kParquetK, kZParquet>);
  r.part1_multi_fn[slot] = reinterpret_cast<const void*>(
      &part_scatter1_kernel<uint32_t, kParquetWords, kParquetK, kZParquet, true>);
  r.part1_chunk_fn[slot] = reinterpret_cast<const void*>(
      &part_scatter1_kernel<uint32_t, kParquetWords, kParquetK, kZParquet, false, true>);
  r.part2_fn[slot] =
      reinterpret_cast<const void*>(&part_scatter2_kernel<uint32_t, kParquetWords, kParquetK, kZParquet>);
  r.apply_fn[slot] =
      reinterpret_cast<const void*>(&part_apply_kernel<uint32_t, kParquetWords, kParquetK, kZParquet>);
}

}  // namespace bfhip
