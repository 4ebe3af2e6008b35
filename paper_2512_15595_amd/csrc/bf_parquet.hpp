// bf_parquet.hpp -- the Apache Parquet split-block Bloom filter as a
// configuration of the sectorized filter (the Arrow / Parquet-compatible
// configuration of Sec. I and Sec. VI).
//
// The format is the sectorized filter with B = 256 (eight 32-bit words),
// k = 8 and one pattern bit per word: value x hashes to h = xxHash64 of its
// 8-byte little-endian encoding with seed 0, the block is the upper 32 bits
// of h scaled to the block count (floor(hi32 * b / 2^32), the rule of
// bf_hash.hpp), and word i of the block gets bit (lo32(h) * c_i mod 2^32)
// >> 27 for the format's eight odd constants c_i.  Only the constants differ
// from the salts of bf_hash.hpp, so every kernel of the sectorized 8 x 32,
// k = 8 layout serves the format once its pattern generator takes this
// table: the direct add and lookup for every mapping, and the partitioned
// construction through the block rule below.
#pragma once

#include <stdint.h>

#include "bf_batch_kernels.hpp"
#include "bf_hash.hpp"
#include "bf_kernels.hpp"
#include "bf_partition.hpp"

namespace bfhip {

// The eight odd multipliers of the Parquet split-block Bloom filter, c_0..c_7.
constexpr uint32_t kParquetSalt[8] = {0x47b6137bu, 0x44974d91u, 0x8824ad5bu, 0xa2b7289du,
                                      0x705495c7u, 0x2df1424bu, 0x9efc4947u, 0x5c6bfb31u};

// Salt j of the format: c_j for the eight pattern bits; the generator's
// other slots (j >= 8) are never read at k = 8.
struct ParquetSalts {
  static constexpr uint32_t at(int j) { return j < 8 ? kParquetSalt[j] : 1u; }
};

constexpr int kParquetWords = 8;  // 32-bit words per block
constexpr int kParquetK = 8;      // pattern bits per value, one per word

// Template tag of the partitioned kernels' block rule for the format (the
// sectorized rule Z = 0 with the format's salts).
constexpr int kZParquet = -2;

template <>
struct BlockRule<uint32_t, kParquetWords, kParquetK, kZParquet>
    : BlockRule<uint32_t, kParquetWords, kParquetK, 0> {
  __device__ __forceinline__ BlockRule() {
    this->lp = LanePatterns<uint32_t, kParquetWords, kParquetK, 1, kParquetWords>(0, ParquetSalts{});
  }
};

template <int THETA, int PHI, int KT, bool ATOM64>
__global__ __launch_bounds__(kBlockThreads) void parquet_add_kernel(BfArgs a) {
  const LanePatterns<uint32_t, kParquetWords, kParquetK, THETA, PHI> lp((threadIdx.x & 63u) & (THETA - 1),
                                                                       ParquetSalts{});
  add_keys<uint32_t, kParquetWords, kParquetK, THETA, PHI, KT, ATOM64>(a, lp);
}

template <int THETA, int PHI, int KT>
__global__ __launch_bounds__(kBlockThreads) void parquet_contains_kernel(BfArgs a) {
  const LanePatterns<uint32_t, kParquetWords, kParquetK, THETA, PHI> lp((threadIdx.x & 63u) & (THETA - 1),
                                                                       ParquetSalts{});
  contains_keys<uint32_t, kParquetWords, kParquetK, THETA, PHI, KT>(a, lp);
}

// The persistent kernel of batched plans and servers over Parquet filters.
template <int OP>
__global__ __launch_bounds__(kBlockThreads) void parquet_batch_kernel(BatchArgs a) {
  batch_tiles<uint32_t, kParquetWords, kParquetK, OP, ParquetSalts>(a);
}

}  // namespace bfhip
