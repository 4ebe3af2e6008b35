// bf_batch_kernels.hpp -- one persistent kernel over the tiles of many filters.
//
// Each tile is up to 256 * KT keys of one filter.  The tile list is ordered
// on the host so that slot i is only ever taken by workgroups with
// blockIdx.x = i (mod 8) (the grid is a multiple of 8 and strides over the
// slots); workgroups are dispatched to the 8 XCDs round-robin, so all tiles
// of a filter run on one XCD and the filter's lines stay in that XCD's L2.
// The execution mapping of a tile is compiled per size class of its filter
// from the autotuned table, so one launch uses several mappings.
#pragma once

#include "bf_kernels.hpp"
#include "bf_tuned.hpp"

namespace bfhip {

struct BatchFilter {  // 48 bytes: one filter (or one request on a filter)
  void* words;
  uint64_t hash_init;
  uint32_t nb_lo;
  uint32_t nb_hi_mask;
  const uint64_t* keys;  // tile key_start indexes into keys / out
  uint8_t* out;
  uint64_t reserved;
};

struct BatchTile {  // 16 bytes
  uint64_t key_start;  // offset of the tile's first key in the key / result arrays
  uint32_t filter;
  uint32_t meta;       // bits 0..15 key count, 16..17 size class, 18 packed loads allowed
};

constexpr uint32_t kTileCountMask = 0xffffu;
constexpr int kTileClassShift = 16;
constexpr uint32_t kTileVecBit = 1u << 18;

struct BatchArgs {
  const BatchFilter* filters;
  const BatchTile* tiles;
  uint64_t ntiles;
  uint32_t k;
  uint32_t pad;
};

// The mapping a size class runs with (256-thread workgroups: tiles are
// planned on the host at that size).  Runtime-k layouts use one lane per key
// and one key per lane, as the single-filter path does.
template <typename W, int S_WORDS, int K, int OP, int CLS>
constexpr MapSpec batch_map() {
  if constexpr (K == 0) {
    return MapSpec{1, static_cast<uint32_t>(S_WORDS), 1, 32, 0, kBlockThreads, true};
  } else {
    // batched launches are large: the tuned rows of large batches at k
    return tuned_map(OP, 8 * static_cast<int>(sizeof(W)), S_WORDS, CLS, K, 1);
  }
}

template <typename W, int S_WORDS, int K, int OP, int CLS, typename SALTS>
__device__ __forceinline__ void batch_tile(const BatchArgs& a, const BatchTile& t,
                                           const BatchFilter& f, const FilterView& fv) {
  constexpr MapSpec m = batch_map<W, S_WORDS, K, OP, CLS>();
  constexpr int kTheta = static_cast<int>(m.theta);
  constexpr int kPhi = static_cast<int>(m.phi);
  constexpr int kKt = static_cast<int>(m.kt);
  static_assert(kTheta * kPhi <= S_WORDS && kTheta <= 16, "tuned mapping fits the block");
  constexpr bool kAtom64 = OP == 0 && sizeof(W) == 4 && kPhi >= 2 && m.atomic_bits == 64;
  const LanePatterns<W, S_WORDS, K, kTheta, kPhi> lp((threadIdx.x & 63u) & (kTheta - 1), SALTS{});
  const uint32_t count = t.meta & kTileCountMask;
  const bool vec_ok = (t.meta & kTileVecBit) != 0;
  if constexpr (OP == 0) {
    add_tile<W, S_WORDS, K, kTheta, kPhi, kKt, kAtom64>(fv, f.keys + t.key_start, count, vec_ok,
                                                        a.k, lp);
  } else {
    contains_tile<W, S_WORDS, K, kTheta, kPhi, kKt>(fv, f.keys + t.key_start, f.out + t.key_start,
                                                    count, vec_ok, a.k, lp);
  }
}

// The tile walk, for the pattern multipliers SALTS (bf_hash.hpp's salts,
// or another filter format's table).
template <typename W, int S_WORDS, int K, int OP, typename SALTS>
__device__ __forceinline__ void batch_tiles(const BatchArgs& a) {
  for (uint64_t i = blockIdx.x; i < a.ntiles; i += gridDim.x) {
    const BatchTile t = a.tiles[i];
    if ((t.meta & kTileCountMask) == 0) continue;  // padding slot
    const BatchFilter f = a.filters[t.filter];
    const FilterView fv{f.words, f.hash_init, f.nb_lo, f.nb_hi_mask};
    switch ((t.meta >> kTileClassShift) & 3u) {
      case 0: batch_tile<W, S_WORDS, K, OP, 0, SALTS>(a, t, f, fv); break;
      case 1: batch_tile<W, S_WORDS, K, OP, 1, SALTS>(a, t, f, fv); break;
      default: batch_tile<W, S_WORDS, K, OP, 2, SALTS>(a, t, f, fv); break;
    }
  }
}

template <typename W, int S_WORDS, int K, int OP>
__global__ __launch_bounds__(kBlockThreads) void bf_batch_kernel(BatchArgs a) {
  batch_tiles<W, S_WORDS, K, OP, PaperSalts>(a);
}

}  // namespace bfhip
