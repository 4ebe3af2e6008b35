// bf_kernels.hpp -- bulk add / contains kernels for gfx950 (wave64).
//
// Execution mapping (paper Sec. IV-A, IV-C), as template parameters:
//   THETA  lanes per key (horizontal): a group of THETA adjacent lanes of a
//          wave shares one key at a time;
//   PHI    words per lane per step (vertical): one wide load / atomic group;
//   KT     keys per lane: each lane loads and hashes KT consecutive keys.
// A block of S_WORDS words is covered in S_WORDS / (THETA * PHI) steps.
//
// Work-efficient cooperation (Sec. IV-C): every lane hashes its own keys;
// a group then walks its THETA lanes, broadcasting (block, lo32) of one key
// at a time, and all lanes of the group apply their words of that block.
// Lookup results stay with the lane that owns the key, so the byte stores
// are coalesced.  With THETA = 1 there is no cross-lane traffic at all.
//
// Salts (Sec. IV-B): the salt index of every pattern bit is a compile-time
// constant for THETA = 1.  For THETA > 1 a lane's salts depend on its rank in
// the group; they are selected once per thread at kernel entry (a short
// compare/select chain per salt) and kept in VGPRs for every key the thread
// processes, instead of being re-selected per key.
//
// Tail handling: the grid walks tiles of 256 * KT keys; only the last tile
// (uniform test) takes the guarded path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "bf_hash.hpp"

namespace bfhip {

constexpr int kBlockThreads = 256;

// Kernel arguments, passed by value.
struct BfArgs {
  void* words;            // b * s words of S bits
  const uint64_t* keys;   // n keys
  uint8_t* out;           // n result bytes (contains only)
  uint64_t n;
  uint64_t hash_init;     // xxh64_u64_init(seed)
  uint32_t nb_lo;         // num_blocks mod 2^32
  uint32_t nb_hi_mask;    // 0xffffffff iff num_blocks == 2^32, else 0
  uint32_t k;             // pattern bits per key, s <= k <= 32
  uint32_t pad;
};

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Loads of PHI contiguous words (PHI * sizeof(W) bytes, naturally aligned):
// 16-byte vector loads where the chunk allows, else 8 / 4 bytes.
// ---------------------------------------------------------------------------
template <typename W, int PHI>
__device__ __forceinline__ void load_words(const W* p, W (&v)[PHI]) {
  constexpr int kBytes = PHI * static_cast<int>(sizeof(W));
  if constexpr (kBytes >= 16) {
    constexpr int kVec = kBytes / 16;
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int i = 0; i < kVec; ++i) {
      u32x4 x = q[i];
      __builtin_memcpy(reinterpret_cast<char*>(v) + 16 * i, &x, 16);
    }
  } else if constexpr (kBytes == 8) {
    u32x2 x = *reinterpret_cast<const u32x2*>(p);
    __builtin_memcpy(v, &x, 8);
  } else {
    uint32_t x = *reinterpret_cast<const uint32_t*>(p);
    __builtin_memcpy(v, &x, 4);
  }
}

// Keys of one lane: KT consecutive 8-byte keys (8*KT-byte aligned).  Keys
// and results stream through once, so they are loaded and stored as
// non-temporal: the lines the filter's random reads bring in then keep more
// of the caches (measured on MI355X: a 1 GiB lookup of 2^28 keys 5.23 ->
// 5.12 ms).
template <int KT>
__device__ __forceinline__ void load_keys(const uint64_t* p, uint64_t (&v)[KT]) {
  if constexpr (KT == 1) {
    v[0] = __builtin_nontemporal_load(p);
  } else {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int i = 0; i < KT / 2; ++i) {
      u32x4 x = __builtin_nontemporal_load(q + i);
      __builtin_memcpy(reinterpret_cast<char*>(v) + 16 * i, &x, 16);
    }
  }
}

// KT result bytes of one lane, packed into one store.
template <int KT>
__device__ __forceinline__ void store_results(uint8_t* p, const uint32_t (&r)[KT]) {
  if constexpr (KT == 1) {
    __builtin_nontemporal_store(static_cast<uint8_t>(r[0]), p);
  } else if constexpr (KT == 2) {
    __builtin_nontemporal_store(static_cast<uint16_t>(r[0] | (r[1] << 8)), reinterpret_cast<uint16_t*>(p));
  } else {
    static_assert(KT == 4, "KT");
    __builtin_nontemporal_store(r[0] | (r[1] << 8) | (r[2] << 16) | (r[3] << 24), reinterpret_cast<uint32_t*>(p));
  }
}

// ---------------------------------------------------------------------------
// Per-lane pattern generator for the words this lane owns.
//
// Lane rank q in its group owns, in step st, words
//   w = st*THETA*PHI + q*PHI + f,  f = 0..PHI-1,
// and word w receives pattern bits j = w + i*S_WORDS (i = 0..32/S_WORDS-1)
// with j < k.
// ---------------------------------------------------------------------------
template <typename W, int S_WORDS, int K, int THETA, int PHI>
struct LanePatterns {
  static constexpr int kSteps = S_WORDS / (THETA * PHI);
  static constexpr int kSlots = kMaxK / S_WORDS;  // bits per word, at most
  static_assert(kSteps >= 1, "THETA * PHI must not exceed the block");

  uint32_t salt[kSteps][PHI][kSlots];
  uint32_t q;

  // SALTS::at(j) is salt j (PaperSalts: the derivation of bf_hash.hpp).
  template <typename SALTS = PaperSalts>
  __device__ __forceinline__ explicit LanePatterns(uint32_t lane_rank, SALTS = SALTS{}) : q(lane_rank) {
#pragma unroll
    for (int st = 0; st < kSteps; ++st)
#pragma unroll
      for (int f = 0; f < PHI; ++f)
#pragma unroll
        for (int i = 0; i < kSlots; ++i) {
          uint32_t v = SALTS::at(st * THETA * PHI + f + i * S_WORDS);
#pragma unroll
          for (int r = 1; r < THETA; ++r)
            v = (lane_rank == static_cast<uint32_t>(r))
                    ? SALTS::at(st * THETA * PHI + r * PHI + f + i * S_WORDS)
                    : v;
          salt[st][f][i] = v;
        }
  }

  // Pattern of this lane's word (st, f) for hash low word lo.  With K > 0
  // every guard below is a compile-time constant after unrolling; with K = 0
  // (any other k) the guards test the runtime k.
  __device__ __forceinline__ W word(int st, int f, uint32_t lo, uint32_t k_runtime) const {
    const uint32_t k = K > 0 ? static_cast<uint32_t>(K) : k_runtime;
    W pat = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
      const uint32_t jmin = st * THETA * PHI + f + i * S_WORDS;     // rank 0
      const uint32_t jmax = jmin + (THETA - 1) * PHI;               // rank THETA-1
      if (jmin < k) {                                               // uniform
        W bit = pattern_bit<W>(lo, salt[st][f][i]);
        if (jmax >= k) {                                            // uniform
          const uint32_t jl = jmin + q * PHI;
          bit = (jl < k) ? bit : W(0);
        }
        pat |= bit;
      }
    }
    return pat;
  }
};

// Broadcast of a 32-bit value from rank R of each THETA-lane group.
template <int THETA, int R>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v, uint32_t lane) {
  if constexpr (THETA == 1) {
    return v;
  } else {
    const int src = static_cast<int>((lane & ~static_cast<uint32_t>(THETA - 1)) + R);
    return static_cast<uint32_t>(__shfl(static_cast<int>(v), src, 64));
  }
}

// ---------------------------------------------------------------------------
// One key's block operation by one group (all THETA lanes call this with the
// broadcast block / lo of the same key).
// ---------------------------------------------------------------------------
template <typename W, int S_WORDS, int K, int THETA, int PHI, bool ATOM64>
__device__ __forceinline__ void add_block(W* words, uint32_t blk, uint32_t lo,
                                          const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp,
                                          uint32_t k) {
  W* base = words + static_cast<uint64_t>(blk) * S_WORDS + lp.q * PHI;
#pragma unroll
  for (int st = 0; st < LanePatterns<W, S_WORDS, K, THETA, PHI>::kSteps; ++st) {
    W* p = base + st * THETA * PHI;
    if constexpr (ATOM64 && sizeof(W) == 4 && PHI >= 2) {
#pragma unroll
      for (int f = 0; f < PHI; f += 2) {
        uint64_t v = static_cast<uint64_t>(lp.word(st, f, lo, k)) |
                     (static_cast<uint64_t>(lp.word(st, f + 1, lo, k)) << 32);
        __hip_atomic_fetch_or(reinterpret_cast<uint64_t*>(p + f), v, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
#pragma unroll
      for (int f = 0; f < PHI; ++f) {
        W v = lp.word(st, f, lo, k);
        __hip_atomic_fetch_or(p + f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI>
__device__ __forceinline__ bool test_block(const W* words, uint32_t blk, uint32_t lo,
                                           const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp,
                                           uint32_t k) {
  const W* base = words + static_cast<uint64_t>(blk) * S_WORDS + lp.q * PHI;
  constexpr int kSteps = LanePatterns<W, S_WORDS, K, THETA, PHI>::kSteps;
  W v[kSteps][PHI];
#pragma unroll
  for (int st = 0; st < kSteps; ++st) load_words<W, PHI>(base + st * THETA * PHI, v[st]);
  W miss = 0;
#pragma unroll
  for (int st = 0; st < kSteps; ++st)
#pragma unroll
    for (int f = 0; f < PHI; ++f) {
      W pat = lp.word(st, f, lo, k);
      miss |= pat & ~v[st][f];
    }
  return miss == 0;
}

// ---------------------------------------------------------------------------
// One tile: up to 256 * KT consecutive keys handled by one 256-thread
// workgroup, thread i taking keys [i*KT, i*KT + KT).  `count` is the number
// of valid keys in the tile; `vec_ok` says the tile may use the packed
// 8*KT-byte key loads and KT-byte result stores (full and aligned).
// ---------------------------------------------------------------------------
struct FilterView {
  void* words;
  uint64_t hash_init;
  uint32_t nb_lo;
  uint32_t nb_hi_mask;
};

template <int KT>
__device__ __forceinline__ void hash_tile_keys(const FilterView& fv, const uint64_t* keys,
                                               uint32_t count, bool vec_ok, uint32_t (&blk)[KT],
                                               uint32_t (&lo)[KT]) {
  const uint32_t first = threadIdx.x * KT;
  uint64_t key[KT];
  if (vec_ok) {
    load_keys<KT>(keys + first, key);
  } else {
#pragma unroll
    for (int t = 0; t < KT; ++t) key[t] = (first + t < count) ? __builtin_nontemporal_load(keys + first + t) : 0;
  }
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const uint64_t h = xxh64_u64(key[t], fv.hash_init);
    blk[t] = block_of(h, fv.nb_lo, fv.nb_hi_mask);
    lo[t] = static_cast<uint32_t>(h);
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT, bool ATOM64>
__device__ __forceinline__ void add_tile(const FilterView& fv, const uint64_t* keys, uint32_t count,
                                         bool vec_ok, uint32_t k,
                                         const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp) {
  const uint32_t lane = threadIdx.x & 63u;
  W* words = static_cast<W*>(fv.words);
  uint32_t blk[KT], lo[KT];
  hash_tile_keys<KT>(fv, keys, count, vec_ok, blk, lo);
  if constexpr (THETA == 1) {
    const uint32_t first = threadIdx.x * KT;
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (vec_ok || first + t < count)
        add_block<W, S_WORDS, K, 1, PHI, ATOM64>(words, blk[t], lo[t], lp, k);
  } else {
    const uint32_t group_first = (threadIdx.x & ~static_cast<uint32_t>(THETA - 1)) * KT;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      [&]<int... R>(std::integer_sequence<int, R...>) {
        ([&] {
          const uint32_t b = group_bcast<THETA, R>(blk[t], lane);
          const uint32_t l = group_bcast<THETA, R>(lo[t], lane);
          if (vec_ok || group_first + static_cast<uint32_t>(R) * KT + t < count)
            add_block<W, S_WORDS, K, THETA, PHI, ATOM64>(words, b, l, lp, k);
        }(), ...);
      }(std::make_integer_sequence<int, THETA>{});
    }
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT>
__device__ __forceinline__ void contains_tile(const FilterView& fv, const uint64_t* keys,
                                              uint8_t* out, uint32_t count, bool vec_ok,
                                              uint32_t k,
                                              const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t rank = lane & (THETA - 1);
  const W* words = static_cast<const W*>(fv.words);
  uint32_t blk[KT], lo[KT];
  hash_tile_keys<KT>(fv, keys, count, vec_ok, blk, lo);
  uint32_t res[KT];
  if constexpr (THETA == 1) {
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      // Out-of-range keys of a partial tile are hashed as key 0 and read an
      // in-range block; their result is never stored.
      res[t] = test_block<W, S_WORDS, K, 1, PHI>(words, blk[t], lo[t], lp, k) ? 1u : 0u;
    }
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
          const bool ok = test_block<W, S_WORDS, K, THETA, PHI>(words, b, l, lp, k);
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

// ---------------------------------------------------------------------------
// Single-filter kernels: a grid-stride walk over the tiles of one key array,
// a tile being blockDim.x * KT keys (the workgroup size is a tuned knob: 64,
// 128 or 256 threads, whole wavefronts).  The host guarantees 8*KT-byte
// aligned keys and KT-byte aligned results.
// ---------------------------------------------------------------------------
template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT, bool ATOM64>
__device__ __forceinline__ void add_keys(const BfArgs& a, const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp) {
  const FilterView fv{a.words, a.hash_init, a.nb_lo, a.nb_hi_mask};
  const uint64_t tile = static_cast<uint64_t>(blockDim.x) * KT;
  const uint64_t stride = tile * gridDim.x;
  for (uint64_t base = blockIdx.x * tile; base < a.n; base += stride) {
    const uint32_t count = static_cast<uint32_t>(a.n - base < tile ? a.n - base : tile);
    add_tile<W, S_WORDS, K, THETA, PHI, KT, ATOM64>(fv, a.keys + base, count, count == tile,
                                                    a.k, lp);
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT>
__device__ __forceinline__ void contains_keys(const BfArgs& a,
                                              const LanePatterns<W, S_WORDS, K, THETA, PHI>& lp) {
  const FilterView fv{a.words, a.hash_init, a.nb_lo, a.nb_hi_mask};
  const uint64_t tile = static_cast<uint64_t>(blockDim.x) * KT;
  const uint64_t stride = tile * gridDim.x;
  for (uint64_t base = blockIdx.x * tile; base < a.n; base += stride) {
    const uint32_t count = static_cast<uint32_t>(a.n - base < tile ? a.n - base : tile);
    contains_tile<W, S_WORDS, K, THETA, PHI, KT>(fv, a.keys + base, a.out + base, count,
                                                 count == tile, a.k, lp);
  }
}

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT, bool ATOM64>
__global__ __launch_bounds__(kBlockThreads) void bf_add_kernel(BfArgs a) {
  const LanePatterns<W, S_WORDS, K, THETA, PHI> lp((threadIdx.x & 63u) & (THETA - 1));
  add_keys<W, S_WORDS, K, THETA, PHI, KT, ATOM64>(a, lp);
}

template <typename W, int S_WORDS, int K, int THETA, int PHI, int KT>
__global__ __launch_bounds__(kBlockThreads) void bf_contains_kernel(BfArgs a) {
  const LanePatterns<W, S_WORDS, K, THETA, PHI> lp((threadIdx.x & 63u) & (THETA - 1));
  contains_keys<W, S_WORDS, K, THETA, PHI, KT>(a, lp);
}

}  // namespace bfhip
