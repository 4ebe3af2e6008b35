// bf_variant_kernels.hpp -- bulk add / contains for the two filter layouts
// beside the sectorized one: the classic filter (Sec. II-A-1) and the
// cache-sectorized filter (Sec. II-A-5, with the execution rule of Sec. V-A).
//
// Both reuse the per-key hash of bf_hash.hpp and the tile walk of the
// sectorized kernels: a 256-thread workgroup takes tiles of 256 * KT
// consecutive keys in a grid-stride loop, each lane loading and hashing KT
// keys; only the last tile takes the guarded path.
//
// Classic filter.  Key x with h = xxHash64(x) sets bits
//   p_j = floor(((h * A_j) mod 2^64) * m / 2^64),  j < k,
// of an m-bit array (bit p in 32-bit word p / 32, bit p mod 32: the byte
// layout of the oracle).  Every position is an independent random word, so a
// key is k uncoalesced 4-byte atomics (add) or loads (contains); the lane
// issues all k (times KT keys) before it consumes any, which keeps k * KT
// requests in flight per lane.  For a power-of-two m the reduction is the
// top log2(m) bits of the product (POW2).
//
// Cache-sectorized filter.  The s words of a block form z groups of s/z
// consecutive words; group g takes the word g*s/z + top log2(s/z) bits of
// (lo32(h) * c_g), and pattern bits j = g, g + z, g + 2z, ... (k/z of them,
// placed as in the sectorized filter).  A key therefore touches z words
// rather than s.  THETA lanes may share a key (Sec. IV-A); lane rank q
// then owns the z/THETA consecutive groups q*z/THETA .. -- a vertical chunk
// of s/THETA words that contains whole groups, which is the s/z <= Phi rule
// of Sec. V-A, so the word choice never crosses lanes.  (block, lo32) is
// broadcast within the group and a lookup's group AND is one ballot.
//
// Chained pattern hashing (the prior-art rule of Sec. IV-B, kept for the
// optimization breakdown of Sec. V-E): the sectorized layout and block rule,
// but bit j comes from h_{j+1} = xxHash64(key, seed = h_j) -- k dependent
// hash evaluations per key instead of k independent multiplies.  One lane
// per key, whole-block loads / one atomic per word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "bf_hash.hpp"
#include "bf_kernels.hpp"
#include "bf_registry.hpp"

namespace bfhip {

// ---------------------------------------------------------------------------
// Classic filter
// ---------------------------------------------------------------------------
struct ClassicArgs {
  uint32_t* words;        // m / 32 words
  const uint64_t* keys;
  uint8_t* out;           // contains only
  uint64_t n;
  uint64_t hash_init;     // xxh64_u64_init(seed)
  uint64_t num_bits;      // m, a multiple of 64
  uint32_t shift;         // 64 - log2(m) when m is a power of two
  uint32_t k;
};

template <bool POW2>
__device__ __forceinline__ uint64_t classic_position(uint64_t h, uint64_t salt, uint64_t m,
                                                     uint32_t shift) {
  const uint64_t prod = h * salt;  // mod 2^64
  if constexpr (POW2)
    return prod >> shift;
  else
    return __umul64hi(prod, m);
}

template <int KT>
__device__ __forceinline__ void load_tile_keys(const uint64_t* keys, uint32_t count, bool vec_ok,
                                               uint64_t (&key)[KT]) {
  const uint32_t first = threadIdx.x * KT;
  if (vec_ok) {
    load_keys<KT>(keys + first, key);
  } else {
#pragma unroll
    for (int t = 0; t < KT; ++t) key[t] = (first + t < count) ? keys[first + t] : 0;
  }
}

template <int K, bool POW2, int KT>
__device__ __forceinline__ void classic_add_tile(const ClassicArgs& a, const uint64_t* keys,
                                                 uint32_t count, bool vec_ok) {
  uint64_t key[KT];
  load_tile_keys<KT>(keys, count, vec_ok, key);
  const uint32_t first = threadIdx.x * KT;
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    if (!(vec_ok || first + t < count)) continue;
    const uint64_t h = xxh64_u64(key[t], a.hash_init);
    if constexpr (K > 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint64_t p = classic_position<POW2>(h, kSalts64.a[j], a.num_bits, a.shift);
        __hip_atomic_fetch_or(a.words + (p >> 5), 1u << (p & 31u), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      for (uint32_t j = 0; j < a.k; ++j) {
        const uint64_t p = classic_position<POW2>(h, kSalts64.a[j], a.num_bits, a.shift);
        __hip_atomic_fetch_or(a.words + (p >> 5), 1u << (p & 31u), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

template <int K, bool POW2, int KT>
__device__ __forceinline__ void classic_contains_tile(const ClassicArgs& a, const uint64_t* keys,
                                                      uint8_t* out, uint32_t count, bool vec_ok) {
  uint64_t key[KT];
  load_tile_keys<KT>(keys, count, vec_ok, key);
  uint32_t res[KT];
  if constexpr (K > 0) {
    // All K * KT loads are issued before any is consumed.
    uint32_t w[KT][K];
    uint32_t bit[KT][K];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const uint64_t h = xxh64_u64(key[t], a.hash_init);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint64_t p = classic_position<POW2>(h, kSalts64.a[j], a.num_bits, a.shift);
        w[t][j] = a.words[p >> 5];
        bit[t][j] = static_cast<uint32_t>(p) & 31u;
      }
    }
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      uint32_t miss = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) miss |= ~(w[t][j] >> bit[t][j]) & 1u;
      res[t] = miss ? 0u : 1u;
    }
  } else {
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const uint64_t h = xxh64_u64(key[t], a.hash_init);
      uint32_t miss = 0;
      for (uint32_t j = 0; j < a.k; ++j) {
        const uint64_t p = classic_position<POW2>(h, kSalts64.a[j], a.num_bits, a.shift);
        miss |= ~(a.words[p >> 5] >> (static_cast<uint32_t>(p) & 31u)) & 1u;
      }
      res[t] = miss ? 0u : 1u;
    }
  }
  const uint32_t first = threadIdx.x * KT;
  if (vec_ok) {
    store_results<KT>(out + first, res);
  } else {
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (first + t < count) out[first + t] = static_cast<uint8_t>(res[t]);
  }
}

template <int K, bool POW2, int KT>
__global__ __launch_bounds__(kBlockThreads) void classic_add_kernel(ClassicArgs a) {
  constexpr uint64_t kTile = static_cast<uint64_t>(kBlockThreads) * KT;
  const uint64_t ntiles = (a.n + kTile - 1) / kTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = tile * kTile;
    const uint32_t count = static_cast<uint32_t>(a.n - base < kTile ? a.n - base : kTile);
    classic_add_tile<K, POW2, KT>(a, a.keys + base, count, count == kTile);
  }
}

template <int K, bool POW2, int KT>
__global__ __launch_bounds__(kBlockThreads) void classic_contains_kernel(ClassicArgs a) {
  constexpr uint64_t kTile = static_cast<uint64_t>(kBlockThreads) * KT;
  const uint64_t ntiles = (a.n + kTile - 1) / kTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = tile * kTile;
    const uint32_t count = static_cast<uint32_t>(a.n - base < kTile ? a.n - base : kTile);
    classic_contains_tile<K, POW2, KT>(a, a.keys + base, a.out + base, count, count == kTile);
  }
}

// ---------------------------------------------------------------------------
// Cache-sectorized filter
// ---------------------------------------------------------------------------
constexpr int ilog2_c(int v) { return v <= 1 ? 0 : 1 + ilog2_c(v / 2); }

// The groups one lane owns and their salts.  K = 0 means a runtime k (then
// every slot is guarded by the wave-uniform bits-per-group count).
template <typename W, int S_WORDS, int Z, int K, int THETA>
struct CsbfLane {
  static constexpr int kGroups = Z / THETA;            // groups per lane
  static constexpr int kWidth = S_WORDS / Z;           // words per group
  static constexpr int kLogWidth = ilog2_c(kWidth);
  static constexpr int kSlots = K > 0 ? K / Z : kMaxK / Z;  // bits per group word
  static_assert(THETA <= Z && Z <= S_WORDS, "lanes must own whole groups");
  static_assert(K == 0 || K % Z == 0, "k must be a multiple of z");

  uint32_t gsalt[kGroups];
  uint32_t salt[kGroups][kSlots];
  uint32_t q;

  __device__ __forceinline__ explicit CsbfLane(uint32_t rank) : q(rank) {
#pragma unroll
    for (int i = 0; i < kGroups; ++i) {
      uint32_t c = kGroupSalts.c[i];
#pragma unroll
      for (int r = 1; r < THETA; ++r)
        c = (rank == static_cast<uint32_t>(r)) ? kGroupSalts.c[r * kGroups + i] : c;
      gsalt[i] = c;
#pragma unroll
      for (int t = 0; t < kSlots; ++t) {
        uint32_t v = kSalts.a[i + Z * t];
#pragma unroll
        for (int r = 1; r < THETA; ++r)
          v = (rank == static_cast<uint32_t>(r)) ? kSalts.a[r * kGroups + i + Z * t] : v;
        salt[i][t] = v;
      }
    }
  }

  // Word (within the block) of this lane's i-th group.
  __device__ __forceinline__ uint32_t word(int i, uint32_t lo) const {
    uint32_t w = (q * kGroups + static_cast<uint32_t>(i)) * kWidth;
    if constexpr (kWidth > 1) w += (lo * gsalt[i]) >> (32 - kLogWidth);
    return w;
  }

  // Pattern of this lane's i-th group word; bits_rt = k / z (runtime k only).
  __device__ __forceinline__ W pattern(int i, uint32_t lo, uint32_t bits_rt) const {
    W pat = 0;
#pragma unroll
    for (int t = 0; t < kSlots; ++t) {
      if (K > 0 || static_cast<uint32_t>(t) < bits_rt) pat |= pattern_bit<W>(lo, salt[i][t]);
    }
    return pat;
  }
};

template <typename W, int S_WORDS, int Z, int K, int THETA>
__device__ __forceinline__ void csbf_add_block(W* words, uint32_t blk, uint32_t lo,
                                               const CsbfLane<W, S_WORDS, Z, K, THETA>& ln,
                                               uint32_t bits_rt) {
  W* base = words + static_cast<uint64_t>(blk) * S_WORDS;
#pragma unroll
  for (int i = 0; i < CsbfLane<W, S_WORDS, Z, K, THETA>::kGroups; ++i)
    __hip_atomic_fetch_or(base + ln.word(i, lo), ln.pattern(i, lo, bits_rt), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

template <typename W, int S_WORDS, int Z, int K, int THETA>
__device__ __forceinline__ bool csbf_test_block(const W* words, uint32_t blk, uint32_t lo,
                                                const CsbfLane<W, S_WORDS, Z, K, THETA>& ln,
                                                uint32_t bits_rt) {
  constexpr int kG = CsbfLane<W, S_WORDS, Z, K, THETA>::kGroups;
  const W* base = words + static_cast<uint64_t>(blk) * S_WORDS;
  W v[kG];
#pragma unroll
  for (int i = 0; i < kG; ++i) v[i] = base[ln.word(i, lo)];
  W miss = 0;
#pragma unroll
  for (int i = 0; i < kG; ++i) {
    const W pat = ln.pattern(i, lo, bits_rt);
    miss |= pat & ~v[i];
  }
  return miss == 0;
}

template <typename W, int S_WORDS, int Z, int K, int THETA, int KT>
__device__ __forceinline__ void csbf_add_tile(const FilterView& fv, const uint64_t* keys,
                                              uint32_t count, bool vec_ok, uint32_t bits_rt,
                                              const CsbfLane<W, S_WORDS, Z, K, THETA>& ln) {
  const uint32_t lane = threadIdx.x & 63u;
  W* words = static_cast<W*>(fv.words);
  uint32_t blk[KT], lo[KT];
  hash_tile_keys<KT>(fv, keys, count, vec_ok, blk, lo);
  if constexpr (THETA == 1) {
    const uint32_t first = threadIdx.x * KT;
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (vec_ok || first + t < count)
        csbf_add_block<W, S_WORDS, Z, K, 1>(words, blk[t], lo[t], ln, bits_rt);
  } else {
    const uint32_t group_first = (threadIdx.x & ~static_cast<uint32_t>(THETA - 1)) * KT;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      [&]<int... R>(std::integer_sequence<int, R...>) {
        ([&] {
          const uint32_t b = group_bcast<THETA, R>(blk[t], lane);
          const uint32_t l = group_bcast<THETA, R>(lo[t], lane);
          if (vec_ok || group_first + static_cast<uint32_t>(R) * KT + t < count)
            csbf_add_block<W, S_WORDS, Z, K, THETA>(words, b, l, ln, bits_rt);
        }(), ...);
      }(std::make_integer_sequence<int, THETA>{});
    }
  }
}

template <typename W, int S_WORDS, int Z, int K, int THETA, int KT>
__device__ __forceinline__ void csbf_contains_tile(const FilterView& fv, const uint64_t* keys,
                                                   uint8_t* out, uint32_t count, bool vec_ok,
                                                   uint32_t bits_rt,
                                                   const CsbfLane<W, S_WORDS, Z, K, THETA>& ln) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t rank = lane & (THETA - 1);
  const W* words = static_cast<const W*>(fv.words);
  uint32_t blk[KT], lo[KT];
  hash_tile_keys<KT>(fv, keys, count, vec_ok, blk, lo);
  uint32_t res[KT];
  if constexpr (THETA == 1) {
#pragma unroll
    for (int t = 0; t < KT; ++t)
      res[t] = csbf_test_block<W, S_WORDS, Z, K, 1>(words, blk[t], lo[t], ln, bits_rt) ? 1u : 0u;
  } else {
    const uint32_t group_shift = lane & ~static_cast<uint32_t>(THETA - 1);
    constexpr uint64_t kGroupMask = (1ull << THETA) - 1ull;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      res[t] = 0;
      [&]<int... R>(std::integer_sequence<int, R...>) {
        ([&] {
          const uint32_t b = group_bcast<THETA, R>(blk[t], lane);
          const uint32_t l = group_bcast<THETA, R>(lo[t], lane);
          const bool ok = csbf_test_block<W, S_WORDS, Z, K, THETA>(words, b, l, ln, bits_rt);
          const uint64_t fails = __ballot(!ok);
          const bool group_ok = ((fails >> group_shift) & kGroupMask) == 0;
          if (rank == static_cast<uint32_t>(R)) res[t] = group_ok ? 1u : 0u;
        }(), ...);
      }(std::make_integer_sequence<int, THETA>{});
    }
  }
  const uint32_t first = threadIdx.x * KT;
  if (vec_ok) {
    store_results<KT>(out + first, res);
  } else {
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (first + t < count) out[first + t] = static_cast<uint8_t>(res[t]);
  }
}

// BfArgs.k carries k / z (bits per group word) for the cache-sectorized kernels.
template <typename W, int S_WORDS, int Z, int K, int THETA, int KT>
__global__ __launch_bounds__(kBlockThreads) void csbf_add_kernel(BfArgs a) {
  const CsbfLane<W, S_WORDS, Z, K, THETA> ln((threadIdx.x & 63u) & (THETA - 1));
  const FilterView fv{a.words, a.hash_init, a.nb_lo, a.nb_hi_mask};
  constexpr uint64_t kTile = static_cast<uint64_t>(kBlockThreads) * KT;
  const uint64_t ntiles = (a.n + kTile - 1) / kTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = tile * kTile;
    const uint32_t count = static_cast<uint32_t>(a.n - base < kTile ? a.n - base : kTile);
    csbf_add_tile<W, S_WORDS, Z, K, THETA, KT>(fv, a.keys + base, count, count == kTile, a.k, ln);
  }
}

template <typename W, int S_WORDS, int Z, int K, int THETA, int KT>
__global__ __launch_bounds__(kBlockThreads) void csbf_contains_kernel(BfArgs a) {
  const CsbfLane<W, S_WORDS, Z, K, THETA> ln((threadIdx.x & 63u) & (THETA - 1));
  const FilterView fv{a.words, a.hash_init, a.nb_lo, a.nb_hi_mask};
  constexpr uint64_t kTile = static_cast<uint64_t>(kBlockThreads) * KT;
  const uint64_t ntiles = (a.n + kTile - 1) / kTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = tile * kTile;
    const uint32_t count = static_cast<uint32_t>(a.n - base < kTile ? a.n - base : kTile);
    csbf_contains_tile<W, S_WORDS, Z, K, THETA, KT>(fv, a.keys + base, a.out + base, count,
                                                    count == kTile, a.k, ln);
  }
}

// ---------------------------------------------------------------------------
// Chained pattern hashing
// ---------------------------------------------------------------------------
template <typename W, int S_WORDS, int K>
__device__ __forceinline__ void chained_pattern(uint64_t key, uint64_t h, uint32_t k,
                                                W (&pat)[S_WORDS]) {
#pragma unroll
  for (int f = 0; f < S_WORDS; ++f) pat[f] = 0;
  if constexpr (K > 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      h = xxh64_u64(key, xxh64_u64_init(h));
      pat[j % S_WORDS] |= W(1) << (static_cast<uint32_t>(h) >> (32 - WordBits<W>::kLog2));
    }
  } else {
    for (uint32_t j = 0; j < k; ++j) {
      h = xxh64_u64(key, xxh64_u64_init(h));
      const W bit = W(1) << (static_cast<uint32_t>(h) >> (32 - WordBits<W>::kLog2));
      const uint32_t w = j & (S_WORDS - 1);
#pragma unroll
      for (int f = 0; f < S_WORDS; ++f) pat[f] |= (w == static_cast<uint32_t>(f)) ? bit : W(0);
    }
  }
}

template <typename W, int S_WORDS, int K, int OP>
__global__ __launch_bounds__(kBlockThreads) void chained_kernel(BfArgs a) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlockThreads;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlockThreads + threadIdx.x; i < a.n;
       i += stride) {
    const uint64_t key = a.keys[i];
    const uint64_t h = xxh64_u64(key, a.hash_init);
    const uint32_t blk = block_of(h, a.nb_lo, a.nb_hi_mask);
    W pat[S_WORDS];
    chained_pattern<W, S_WORDS, K>(key, h, a.k, pat);
    W* base = static_cast<W*>(a.words) + static_cast<uint64_t>(blk) * S_WORDS;
    if constexpr (OP == kOpAdd) {
#pragma unroll
      for (int f = 0; f < S_WORDS; ++f)
        __hip_atomic_fetch_or(base + f, pat[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      W v[S_WORDS];
      load_words<W, S_WORDS>(base, v);
      W miss = 0;
#pragma unroll
      for (int f = 0; f < S_WORDS; ++f) miss |= pat[f] & ~v[f];
      a.out[i] = miss == 0 ? 1 : 0;
    }
  }
}

}  // namespace bfhip
