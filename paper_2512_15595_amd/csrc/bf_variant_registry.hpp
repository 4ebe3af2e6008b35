// bf_variant_registry.hpp -- compiled kernel variants of the classic and the
// cache-sectorized layouts.
//
// Classic: (op, k, keys per lane KT in {1,2,4}, power-of-two m).
// Cache-sectorized partitioned construction: (word bits, s, z, k).
// Cache-sectorized: (op, word bits, s, z, k, THETA <= z, KT), with KT in
// {1, 2} for THETA = 1 and KT = 1 otherwise.  Compiled k are 4, 6, 8, 12,
// 16 (for the cache-sectorized layout those that are multiples of z); any
// other k uses a runtime-k variant (classic: every KT; cache-sectorized:
// THETA = 1, KT = 1).
#pragma once

#include <stdint.h>

#include "bf_registry.hpp"

namespace bfhip {

constexpr int kClassicSize = 2 * kNumK * kKtLog2Max * 2;

inline int classic_index(int op, int kidx, int kt, int pow2) {
  return ((op * kNumK + kidx) * kKtLog2Max + ilog2(kt)) * 2 + pow2;
}

constexpr int kCsbfKtLog2Max = 2;
constexpr int kCsbfSize = 2 * 2 * kLog2Max * kLog2Max * kNumK * kLog2Max * kCsbfKtLog2Max;

inline int csbf_index(int op, int word_bits, int s, int z, int kidx, int theta, int kt) {
  int idx = op;
  idx = idx * 2 + (word_bits == 64 ? 1 : 0);
  idx = idx * kLog2Max + ilog2(s);
  idx = idx * kLog2Max + ilog2(z);
  idx = idx * kNumK + kidx;
  idx = idx * kLog2Max + ilog2(theta);
  idx = idx * kCsbfKtLog2Max + ilog2(kt);
  return idx;
}

// Partitioned construction of the cache-sectorized layout: (word bits, s,
// z, k).
constexpr int kCsbfPartSize = 2 * kLog2Max * kLog2Max * kNumK;

inline int csbf_part_index(int word_bits, int s, int z, int kidx) {
  return (((word_bits == 64 ? 1 : 0) * kLog2Max + ilog2(s)) * kLog2Max + ilog2(z)) * kNumK + kidx;
}

// Chained pattern hashing: (op, word bits, s, k).
constexpr int kChainedSize = 2 * 2 * kLog2Max * kNumK;

inline int chained_index(int op, int word_bits, int s, int kidx) {
  return ((op * 2 + (word_bits == 64 ? 1 : 0)) * kLog2Max + ilog2(s)) * kNumK + kidx;
}

struct VariantRegistry {
  const void* chained[kChainedSize];
  const void* classic[kClassicSize];
  const void* csbf[kCsbfSize];
  const void* classic_part1[kNumK * 2];  // (k, power-of-two m)
  const void* classic_part2;
  const void* classic_apply;
  const void* csbf_part1[kCsbfPartSize];
  const void* csbf_part1_chunk[kCsbfPartSize];  // one pass into chunk buckets
  const void* csbf_part2[kCsbfPartSize];
  const void* csbf_apply[kCsbfPartSize];
};

VariantRegistry& variant_registry();
void ensure_variant_registry();

void register_classic(VariantRegistry&);
void register_chained(VariantRegistry&);
void register_csbf_u32_s1(VariantRegistry&);
void register_csbf_u32_s2(VariantRegistry&);
void register_csbf_u32_s4(VariantRegistry&);
void register_csbf_u32_s8(VariantRegistry&);
void register_csbf_u32_s16(VariantRegistry&);
void register_csbf_u64_s1(VariantRegistry&);
void register_csbf_u64_s2(VariantRegistry&);
void register_csbf_u64_s4(VariantRegistry&);
void register_csbf_u64_s8(VariantRegistry&);
void register_csbf_u64_s16(VariantRegistry&);

}  // namespace bfhip
