// bf_registry.hpp -- table of compiled (layout, k, mapping) kernel variants.
//
// Each translation unit bf_inst_<S>_<s>.hip instantiates the add and contains
// kernels for one word width S and one words-per-block s:
//   - for each compiled pattern-bit count k in {4, 6, 8, 12, 16} with k >= s,
//     every valid mapping (THETA, PHI powers of two, THETA * PHI <= s,
//     THETA <= 16; KT in {1, 2, 4}; for add on 32-bit words with PHI >= 2
//     also the 64-bit atomic variant);
//   - for any other k, a runtime-k variant with THETA = 1, KT = 1 and every
//     PHI.
// and records their host entry addresses here.
#pragma once

#include <stdint.h>

namespace bfhip {

enum Op : int { kOpAdd = 0, kOpContains = 1 };

constexpr int kLog2Max = 5;    // log2 of s, THETA, PHI: 0..4
constexpr int kKtLog2Max = 3;  // log2 KT: 0..2
constexpr int kNumK = 6;       // runtime k, then 4, 6, 8, 12, 16

// Index of a compiled k (0 = the runtime-k variants).
constexpr int k_index(uint32_t k) {
  return k == 4 ? 1 : k == 6 ? 2 : k == 8 ? 3 : k == 12 ? 4 : k == 16 ? 5 : 0;
}

inline int ilog2(uint32_t v) {
  int r = 0;
  while ((1u << r) < v) ++r;
  return r;
}

inline int registry_index(int op, int word_bits, int s, int kidx, int theta, int phi, int kt,
                          int atom64) {
  int idx = op;
  idx = idx * 2 + (word_bits == 64 ? 1 : 0);
  idx = idx * kLog2Max + ilog2(s);
  idx = idx * kNumK + kidx;
  idx = idx * kLog2Max + ilog2(theta);
  idx = idx * kLog2Max + ilog2(phi);
  idx = idx * kKtLog2Max + ilog2(kt);
  idx = idx * 2 + atom64;
  return idx;
}

constexpr int kRegistrySize = 2 * 2 * kLog2Max * kNumK * kLog2Max * kLog2Max * kKtLog2Max * 2;

inline int batch_index(int op, int word_bits, int s, int kidx) {
  return ((op * 2 + (word_bits == 64 ? 1 : 0)) * kLog2Max + ilog2(s)) * kNumK + kidx;
}

constexpr int kBatchRegistrySize = 2 * 2 * kLog2Max * kNumK;

struct Registry {
  const void* fn[kRegistrySize];
  const void* batch_fn[kBatchRegistrySize];  // persistent batched kernels
  const void* part1_fn[kBatchRegistrySize];  // partitioned add: first scatter (op slot 0)
  const void* part1_multi_fn[kBatchRegistrySize];  // ... of a multi-filter plan
  const void* part1_chunk_fn[kBatchRegistrySize];  // ... into chunk buckets (one pass)
  const void* part2_fn[kBatchRegistrySize];  // partitioned add: second scatter
  const void* apply_fn[kBatchRegistrySize];  // partitioned add: per-chunk apply
};

Registry& registry();

// Fills the registry on first use (thread-safe).
void ensure_registry();

// Registration hooks, one per (word width, words per block).
void register_u32_s1(Registry&);
void register_u32_s2(Registry&);
void register_u32_s4(Registry&);
void register_u32_s8(Registry&);
void register_u32_s16(Registry&);
void register_u64_s1(Registry&);
void register_u64_s2(Registry&);
void register_u64_s4(Registry&);
void register_u64_s8(Registry&);
void register_u64_s16(Registry&);

// The same table for the Parquet split-block filter (bf_parquet.h): the
// 32-bit, s = 8, k = 8 slots only (add and lookup for every mapping, the
// partitioned kernels in the single-filter slots; no batched kernels).
Registry& parquet_registry();
void ensure_parquet_registry();
void register_parquet(Registry&);

// The filled table of a filter's pattern multipliers: the Parquet format's
// (parquet) or the derived salts.
const Registry& kernel_table(bool parquet);

}  // namespace bfhip
