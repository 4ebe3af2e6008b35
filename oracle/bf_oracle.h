/*
 * bf_oracle.h -- CPU oracle for the blocked / sectorized Bloom filter.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * definition of what the GPU hot path computes.  Only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant generator with the HIP
 * library; the two meet only on seeded input arrays.
 *
 * Method source: "Optimizing Bloom Filters on Modern GPUs" (arXiv 2512.15595).
 *   - filter layouts: Sec. II-A-2 (blocked), II-A-3 (register-blocked),
 *     II-A-4 (sectorized: a block of s = B/S contiguous S-bit words, the k
 *     fingerprint bits spread evenly over the words, k >= s), II-A-5;
 *   - pattern generation: Sec. IV-B (one 64-bit xxHash64 base hash per key,
 *     bit positions from multiplications by odd constants, "salts").
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   hash input  = XXH64 over the key's 8 little-endian bytes, with the filter seed;
 *   block       = floor(hi32(h) * b / 2^32)                 (fastrange);
 *   salts       = a_j = (XXH64(LE64(j), SALT_SEED) mod 2^32) | 1, j = 0..31,
 *                 SALT_SEED = 0x73746c61732d6662 (ASCII "bf-salts", LE);
 *   bit j       = top log2(S) bits of (lo32(h) * a_j mod 2^32), in word j mod s;
 *   layout      = word (blk, w) at byte offset (blk*s + w) * S/8, little-endian,
 *                 bit p of a word is the value 2^p of that word.
 *
 * Parameters accepted: s in {1,2,4,8,16}, S in {32,64}, s <= k <= 32,
 * 1 <= b <= 2^32.  Functions returning int give 0 on success, -1 on a bad
 * parameter (nothing is written then).
 */
#ifndef BF_ORACLE_H
#define BF_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_SALT_SEED 0x73746c61732d6662ULL
#define ORACLE_MAX_K 32

/* XXH64 of an arbitrary byte string (published xxHash64 algorithm). */
uint64_t oracle_xxh64(const uint8_t *data, size_t len, uint64_t seed);

/* XXH64 of the key's 8 little-endian bytes. */
uint64_t oracle_hash_key(uint64_t key, uint64_t seed);

/* The 32 salts a_0..a_31. */
void oracle_salts(uint32_t out[ORACLE_MAX_K]);

/* 0 if (b, s, S, k) is an accepted parameter set, else -1. */
int oracle_check_params(uint64_t num_blocks, uint32_t words_per_block,
                        uint32_t word_bits, uint32_t k);

/* Block of a base hash: floor(hi32(h) * b / 2^32). */
uint64_t oracle_block_index(uint64_t h, uint64_t num_blocks);

/* Pattern words P_0..P_{s-1} of a base hash (each held in a uint64). */
int oracle_pattern(uint64_t h, uint32_t words_per_block, uint32_t word_bits,
                   uint32_t k, uint64_t *patterns);

/* Filter state = num_blocks * s * S/8 bytes.  add: W |= P for each key. */
int oracle_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
               uint32_t word_bits, uint32_t k, uint64_t seed,
               const uint64_t *keys, uint64_t n);

/* out[i] = 1 iff every pattern bit of keys[i] is set in its block, else 0. */
int oracle_contains(const uint8_t *filter, uint64_t num_blocks,
                    uint32_t words_per_block, uint32_t word_bits, uint32_t k,
                    uint64_t seed, const uint64_t *keys, uint64_t n,
                    uint8_t *out);

/* All filter bytes := 0. */
void oracle_clear(uint8_t *filter, uint64_t nbytes);

/*
 * Words of selected blocks only: out holds nsel blocks of s*S/8 bytes, block
 * i being the state of block sel[i] after adding keys[0..n).  sel must hold
 * distinct block indices < num_blocks.  This is the add definition written
 * per block (a block's words are the OR of the patterns of the keys that
 * select it), used to check large filters at sampled blocks.
 */
int oracle_block_words(uint64_t num_blocks, uint32_t words_per_block,
                       uint32_t word_bits, uint32_t k, uint64_t seed,
                       const uint64_t *keys, uint64_t n, const uint64_t *sel,
                       uint64_t nsel, uint8_t *out);

/* ------------------------------------------------------------------------
 * Classic (unblocked) Bloom filter, Sec. II-A-1: m bits, k positions
 * anywhere.  Readings: position j of a key is floor(((h * A_j) mod 2^64) *
 * m / 2^64) with the 64-bit odd salts A_j = XXH64(LE64(j), SALT_SEED) | 1
 * (whose low halves are the 32-bit salts a_j); bit p lives at byte p / 8,
 * bit p % 8.  m is a multiple of 64; 1 <= k <= 32.
 * ------------------------------------------------------------------------ */
void oracle_salts64(uint64_t out[ORACLE_MAX_K]);
uint64_t oracle_classic_position(uint64_t h, uint64_t num_bits, uint32_t j);
int oracle_classic_add(uint8_t *filter, uint64_t num_bits, uint32_t k, uint64_t seed,
                       const uint64_t *keys, uint64_t n);
int oracle_classic_contains(const uint8_t *filter, uint64_t num_bits, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n,
                            uint8_t *out);
/* Selected 64-bit words (indices sel[0..nsel), distinct) after adding keys. */
int oracle_classic_words(uint64_t num_bits, uint32_t k, uint64_t seed,
                         const uint64_t *keys, uint64_t n, const uint64_t *sel,
                         uint64_t nsel, uint64_t *out);

/* ------------------------------------------------------------------------
 * Cache-sectorized Bloom filter, Sec. II-A-5: the s words of a block form z
 * groups of s/z consecutive words; a key selects one word per group and
 * puts its bits j with j mod z == g into group g's selected word.
 * Readings: the word selected in group g is the top log2(s/z) bits of
 * (lo32(h) * c_g mod 2^32), with a further odd multiplier per group
 * c_g = (XXH64(LE64(32 + g), SALT_SEED) mod 2^32) | 1; bit positions are
 * those of the sectorized filter.  z is a power of two, 1 <= z <= s,
 * z <= k <= 32, k a multiple of z (each selected word receives k/z bits).
 * With z = s this is exactly the sectorized filter.
 * ------------------------------------------------------------------------ */
int oracle_check_csbf_params(uint64_t num_blocks, uint32_t words_per_block,
                             uint32_t word_bits, uint32_t groups, uint32_t k);
void oracle_group_salts(uint32_t out[16]);
int oracle_csbf_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
                    uint32_t word_bits, uint32_t groups, uint32_t k, uint64_t seed,
                    const uint64_t *keys, uint64_t n);
int oracle_csbf_contains(const uint8_t *filter, uint64_t num_blocks,
                         uint32_t words_per_block, uint32_t word_bits, uint32_t groups,
                         uint32_t k, uint64_t seed, const uint64_t *keys, uint64_t n,
                         uint8_t *out);
/* Selected blocks after adding keys, as oracle_block_words. */
int oracle_csbf_block_words(uint64_t num_blocks, uint32_t words_per_block,
                            uint32_t word_bits, uint32_t groups, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n,
                            const uint64_t *sel, uint64_t nsel, uint8_t *out);

/* ------------------------------------------------------------------------
 * Sectorized filter with chained pattern hashing: the pattern rule of prior
 * GPU filters that Sec. IV-B replaces (one initial hash, then the key hashed
 * again with the previous hash as the seed).  Used for the optimization
 * breakdown of Sec. V-E.  Readings: h_0 = XXH64(LE64(x), seed) selects the
 * block as in the sectorized filter; h_{j+1} = XXH64(LE64(x), h_j); bit j
 * (j < k) is the top log2(S) bits of lo32(h_{j+1}), in word j mod s.
 * Parameters and layout as the sectorized filter.
 * ------------------------------------------------------------------------ */
int oracle_chained_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
                       uint32_t word_bits, uint32_t k, uint64_t seed, const uint64_t *keys,
                       uint64_t n);
int oracle_chained_contains(const uint8_t *filter, uint64_t num_blocks,
                            uint32_t words_per_block, uint32_t word_bits, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n, uint8_t *out);

/* ------------------------------------------------------------------------
 * Apache Parquet split-block Bloom filter, the Arrow / Parquet-compatible
 * configuration the paper names (Sec. I and Sec. VI).  The format's
 * definition: num_bytes / 32 blocks of eight little-endian 32-bit words; a
 * value hashes to h = XXH64 of its plain encoding with seed 0 (for the
 * 8-byte types INT64 and DOUBLE: its 8 little-endian bytes, i.e. the key);
 * block = ((h >> 32) * num_blocks) >> 32; word i of that block (i = 0..7)
 * gets bit ((lo32(h) * c_i) mod 2^32) >> 27, c_i the format's eight odd
 * constants.  num_bytes: a multiple of 32, 32 <= num_bytes <= 2^37.  The
 * state's bytes are the bitset a Parquet file stores after the filter's
 * header.  Pinned against the bitsets Apache Arrow writes into Parquet
 * files (tests).
 * ------------------------------------------------------------------------ */
int oracle_parquet_add(uint8_t *filter, uint64_t num_bytes, const uint64_t *values,
                       uint64_t n);
int oracle_parquet_contains(const uint8_t *filter, uint64_t num_bytes,
                            const uint64_t *values, uint64_t n, uint8_t *out);
/* The selected blocks' 32 bytes each after adding values (as
 * oracle_block_words: sel distinct, in range). */
int oracle_parquet_block_words(uint64_t num_bytes, const uint64_t *values, uint64_t n,
                               const uint64_t *sel, uint64_t nsel, uint8_t *out);

#ifdef __cplusplus
}
#endif

#endif /* BF_ORACLE_H */
