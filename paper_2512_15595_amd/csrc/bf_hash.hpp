// bf_hash.hpp -- per-key hash / block / pattern unit for gfx950.
//
// One 64-bit xxHash64 base hash per key (paper Sec. IV-B), the block from its
// upper 32 bits by a multiply-high (fastrange), and k bit positions from the
// lower 32 bits multiplied by odd salts, bit j going to word j mod s
// (Sec. II-A-4).  The salts are computed at compile time by a constexpr
// xxHash64 of the salt index under a fixed salt seed, so every kernel sees
// them as literal operands (Sec. IV-B, "inlining salts"): on CDNA they are
// materialised into SGPRs by s_mov and never loaded from memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfhip {

// xxHash64 primes, from the published xxHash64 algorithm.
constexpr uint64_t kXX1 = 0x9E3779B185EBCA87ull;
constexpr uint64_t kXX2 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kXX3 = 0x165667B19E3779F9ull;
constexpr uint64_t kXX4 = 0x85EBCA77C2B2AE63ull;
constexpr uint64_t kXX5 = 0x27D4EB2F165667C5ull;

// ASCII "bf-salts" read as a little-endian 64-bit integer.
constexpr uint64_t kSaltSeed = 0x73746c61732d6662ull;
constexpr int kMaxK = 32;

__host__ __device__ constexpr uint64_t rotl64(uint64_t x, int r) {
  return (x << r) | (x >> (64 - r));
}

// The seed-dependent constant of a single-lane (8-byte) xxHash64: the
// accumulator starts at seed + P5 + input length.  Computed once on the host.
__host__ __device__ constexpr uint64_t xxh64_u64_init(uint64_t seed) {
  return seed + kXX5 + 8ull;
}

// xxHash64 of exactly 8 bytes (the key, little-endian), given the
// precomputed init value: one lane round, one merge, the final avalanche.
// Five 64-bit multiplies, no data-dependent control flow.
__host__ __device__ constexpr uint64_t xxh64_u64(uint64_t key, uint64_t init) {
  uint64_t lane = rotl64(key * kXX2, 31) * kXX1;
  uint64_t h = init ^ lane;
  h = rotl64(h, 27) * kXX1 + kXX4;
  h ^= h >> 33;
  h *= kXX2;
  h ^= h >> 29;
  h *= kXX3;
  h ^= h >> 32;
  return h;
}

struct SaltTable {
  uint32_t a[kMaxK];
};

__host__ __device__ constexpr SaltTable make_salts() {
  SaltTable t{};
  for (int j = 0; j < kMaxK; ++j) {
    uint64_t h = xxh64_u64(static_cast<uint64_t>(j), xxh64_u64_init(kSaltSeed));
    t.a[j] = static_cast<uint32_t>(h) | 1u;
  }
  return t;
}

constexpr SaltTable kSalts = make_salts();

// Salt j as a compile-time constant.
template <int J>
__device__ __forceinline__ constexpr uint32_t salt() {
  static_assert(J >= 0 && J < kMaxK, "salt index");
  return kSalts.a[J];
}

// The salt table as a type, for pattern generators that take it as a
// template argument (another table gives another filter format).
struct PaperSalts {
  static constexpr uint32_t at(int j) { return kSalts.a[j]; }
};

// A few values are checked at compile time against the derivation above
// (the salts are odd by construction).
static_assert((kSalts.a[0] & kSalts.a[31] & 1u) == 1u, "salts are odd");

// Classic filter (Sec. II-A-1): the same derivation kept at 64 bits,
// A_j = xxHash64(LE64(j), salt seed) | 1; the low halves are the a_j above.
struct Salt64Table {
  uint64_t a[kMaxK];
};

__host__ __device__ constexpr Salt64Table make_salts64() {
  Salt64Table t{};
  for (int j = 0; j < kMaxK; ++j)
    t.a[j] = xxh64_u64(static_cast<uint64_t>(j), xxh64_u64_init(kSaltSeed)) | 1ull;
  return t;
}

constexpr Salt64Table kSalts64 = make_salts64();
static_assert(static_cast<uint32_t>(kSalts64.a[7]) == kSalts.a[7], "salt halves");

// Cache-sectorized filter (Sec. II-A-5 with the group index of Sec. V-A):
// one further odd multiplier per group, c_g = (xxHash64(LE64(32 + g), salt
// seed) mod 2^32) | 1, g < 16, picks the word of group g.
constexpr int kMaxGroups = 16;

struct GroupSaltTable {
  uint32_t c[kMaxGroups];
};

__host__ __device__ constexpr GroupSaltTable make_group_salts() {
  GroupSaltTable t{};
  for (int g = 0; g < kMaxGroups; ++g)
    t.c[g] = static_cast<uint32_t>(
                 xxh64_u64(static_cast<uint64_t>(kMaxK + g), xxh64_u64_init(kSaltSeed))) |
             1u;
  return t;
}

constexpr GroupSaltTable kGroupSalts = make_group_salts();

// Block of a hash: floor(hi32 * b / 2^32) for 1 <= b <= 2^32.  The block
// count is split as b = nb_hi * 2^32 + nb_lo with nb_hi in {0, 1}; then the
// product's high word is umulhi(hi, nb_lo) + nb_hi * hi.
__device__ __forceinline__ uint32_t block_of(uint64_t h, uint32_t nb_lo,
                                             uint32_t nb_hi_mask) {
  uint32_t hi = static_cast<uint32_t>(h >> 32);
  return __umulhi(hi, nb_lo) + (hi & nb_hi_mask);
}

template <typename W>
struct WordBits;
template <>
struct WordBits<uint32_t> {
  static constexpr int kLog2 = 5;
};
template <>
struct WordBits<uint64_t> {
  static constexpr int kLog2 = 6;
};

// One pattern bit: position = top log2(S) bits of lo * a_j (mod 2^32).
template <typename W>
__device__ __forceinline__ W pattern_bit(uint32_t lo, uint32_t a) {
  uint32_t p = (lo * a) >> (32 - WordBits<W>::kLog2);
  return W(1) << p;
}

// Pattern of word W_IDX of an s-word block for a lane-invariant word index:
// OR of bits j = W_IDX, W_IDX + s, ... below k.  k is a kernel argument
// (wave-uniform), so the guards are scalar branches; the salts are literals.
template <typename W, int S_WORDS, int W_IDX>
__device__ __forceinline__ W word_pattern(uint32_t lo, uint32_t k) {
  W pat = 0;
#pragma unroll
  for (int i = 0; i < kMaxK / S_WORDS; ++i) {
    const int j = W_IDX + i * S_WORDS;
    if (static_cast<uint32_t>(j) < k) pat |= pattern_bit<W>(lo, kSalts.a[j]);
  }
  return pat;
}

}  // namespace bfhip
