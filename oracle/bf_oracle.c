/*
 * bf_oracle.c -- CPU oracle for the blocked / sectorized Bloom filter.
 *
 * TEST INFRASTRUCTURE ONLY (see bf_oracle.h).  Plain single-threaded C,
 * written to be checked against the paper by eye, not to be fast.  Nothing
 * here is shared with the HIP library.
 *
 * Parity pins (tests): XXH64 against the independent python-xxhash library;
 * filter bits against a brute-force set model on tiny filters; closed-form
 * false-positive rate and fill fraction; invariants (no false negatives,
 * order independence, union = OR); special cases of the block rule.
 */
#include "bf_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* xxHash64, following the published algorithm description.  The paper uses */
/* a 64-bit xxHash as the per-key base hash (Sec. IV-B).                     */
/* ------------------------------------------------------------------------ */

static const uint64_t XXP1 = 0x9E3779B185EBCA87ULL;
static const uint64_t XXP2 = 0xC2B2AE3D27D4EB4FULL;
static const uint64_t XXP3 = 0x165667B19E3779F9ULL;
static const uint64_t XXP4 = 0x85EBCA77C2B2AE63ULL;
static const uint64_t XXP5 = 0x27D4EB2F165667C5ULL;

static uint64_t rotl64(uint64_t x, unsigned r) {
    return (x << r) | (x >> (64u - r));
}

static uint64_t read_le64(const uint8_t *p) {
    uint64_t v = 0;
    for (int i = 7; i >= 0; --i) v = (v << 8) | p[i];
    return v;
}

static uint32_t read_le32(const uint8_t *p) {
    uint32_t v = 0;
    for (int i = 3; i >= 0; --i) v = (v << 8) | p[i];
    return v;
}

/* One accumulator step: acc + lane*P2, rotate left 31, times P1. */
static uint64_t xx_round(uint64_t acc, uint64_t lane) {
    acc += lane * XXP2;
    acc = rotl64(acc, 31);
    return acc * XXP1;
}

/* Folds one of the four stripe accumulators into the hash. */
static uint64_t xx_merge(uint64_t h, uint64_t acc) {
    h ^= xx_round(0, acc);
    return h * XXP1 + XXP4;
}

uint64_t oracle_xxh64(const uint8_t *data, size_t len, uint64_t seed) {
    const uint8_t *p = data;
    const uint8_t *end = data + len;
    uint64_t h;

    if (len >= 32) {
        /* Four parallel accumulators over 32-byte stripes. */
        uint64_t v1 = seed + XXP1 + XXP2;
        uint64_t v2 = seed + XXP2;
        uint64_t v3 = seed;
        uint64_t v4 = seed - XXP1;
        while ((size_t)(end - p) >= 32) {
            v1 = xx_round(v1, read_le64(p));
            v2 = xx_round(v2, read_le64(p + 8));
            v3 = xx_round(v3, read_le64(p + 16));
            v4 = xx_round(v4, read_le64(p + 24));
            p += 32;
        }
        h = rotl64(v1, 1) + rotl64(v2, 7) + rotl64(v3, 12) + rotl64(v4, 18);
        h = xx_merge(h, v1);
        h = xx_merge(h, v2);
        h = xx_merge(h, v3);
        h = xx_merge(h, v4);
    } else {
        h = seed + XXP5;
    }
    h += (uint64_t)len;

    /* Remaining whole 8-byte lanes. */
    while ((size_t)(end - p) >= 8) {
        h ^= xx_round(0, read_le64(p));
        h = rotl64(h, 27) * XXP1 + XXP4;
        p += 8;
    }
    /* One remaining 4-byte lane. */
    if ((size_t)(end - p) >= 4) {
        h ^= (uint64_t)read_le32(p) * XXP1;
        h = rotl64(h, 23) * XXP2 + XXP3;
        p += 4;
    }
    /* Remaining single bytes. */
    while (p < end) {
        h ^= (uint64_t)(*p) * XXP5;
        h = rotl64(h, 11) * XXP1;
        p += 1;
    }
    /* Final avalanche. */
    h ^= h >> 33;
    h *= XXP2;
    h ^= h >> 29;
    h *= XXP3;
    h ^= h >> 32;
    return h;
}

uint64_t oracle_hash_key(uint64_t key, uint64_t seed) {
    uint8_t bytes[8];
    for (int i = 0; i < 8; ++i) bytes[i] = (uint8_t)(key >> (8 * i));
    return oracle_xxh64(bytes, 8, seed);
}

/* ------------------------------------------------------------------------ */
/* Salts: k odd multipliers (Sec. IV-B).  The paper does not print values;   */
/* they are derived from a fixed seed so that any implementation can         */
/* rebuild them.                                                             */
/* ------------------------------------------------------------------------ */

void oracle_salts(uint32_t out[ORACLE_MAX_K]) {
    for (uint32_t j = 0; j < ORACLE_MAX_K; ++j) {
        uint64_t h = oracle_hash_key((uint64_t)j, ORACLE_SALT_SEED);
        out[j] = (uint32_t)(h & 0xFFFFFFFFULL) | 1u;
    }
}

/* ------------------------------------------------------------------------ */
/* Parameters (Sec. II-A-4: s = B/S words, an SBF needs k >= s).             */
/* ------------------------------------------------------------------------ */

int oracle_check_params(uint64_t num_blocks, uint32_t words_per_block,
                        uint32_t word_bits, uint32_t k) {
    uint32_t s = words_per_block;
    if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return -1;
    if (!(word_bits == 32 || word_bits == 64)) return -1;
    if (k < s || k > ORACLE_MAX_K) return -1;
    if (num_blocks < 1 || num_blocks > (1ULL << 32)) return -1;
    return 0;
}

/* One block per key, chosen uniformly from the upper 32 hash bits
 * (Sec. II-A-2: an additional hash selects the block). */
uint64_t oracle_block_index(uint64_t h, uint64_t num_blocks) {
    uint64_t hi = h >> 32;
    /* hi < 2^32 and num_blocks <= 2^32, so the product fits in 64 bits. */
    return (hi * num_blocks) >> 32;
}

static unsigned log2_word_bits(uint32_t word_bits) {
    return word_bits == 64 ? 6u : 5u;
}

/* Pattern: bit j (j = 0..k-1) sits at position p_j of word j mod s, where
 * p_j is the top log2(S) bits of the 32-bit product lo32(h) * a_j
 * (Sec. II-A-4 for the word split, Sec. IV-B for the salted products). */
static void pattern_with_salts(uint64_t h, uint32_t words_per_block,
                               uint32_t word_bits, uint32_t k,
                               const uint32_t *salts, uint64_t *patterns) {
    uint32_t lo = (uint32_t)(h & 0xFFFFFFFFULL);
    unsigned L = log2_word_bits(word_bits);
    for (uint32_t w = 0; w < words_per_block; ++w) patterns[w] = 0;
    for (uint32_t j = 0; j < k; ++j) {
        uint32_t product = lo * salts[j];          /* mod 2^32 */
        uint32_t p = product >> (32u - L);         /* in [0, S) */
        patterns[j % words_per_block] |= 1ULL << p;
    }
}

int oracle_pattern(uint64_t h, uint32_t words_per_block, uint32_t word_bits,
                   uint32_t k, uint64_t *patterns) {
    if (oracle_check_params(1, words_per_block, word_bits, k) != 0) return -1;
    uint32_t salts[ORACLE_MAX_K];
    oracle_salts(salts);
    pattern_with_salts(h, words_per_block, word_bits, k, salts, patterns);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Filter state as bytes: word (blk, w) at (blk*s + w) * S/8, little-endian. */
/* ------------------------------------------------------------------------ */

static int get_bit(const uint8_t *words, uint64_t word_index,
                   uint32_t word_bits, unsigned p) {
    uint64_t byte = word_index * (word_bits / 8) + p / 8;
    return (words[byte] >> (p % 8)) & 1;
}

static void set_bit(uint8_t *words, uint64_t word_index, uint32_t word_bits,
                    unsigned p) {
    uint64_t byte = word_index * (word_bits / 8) + p / 8;
    words[byte] = (uint8_t)(words[byte] | (1u << (p % 8)));
}

int oracle_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
               uint32_t word_bits, uint32_t k, uint64_t seed,
               const uint64_t *keys, uint64_t n) {
    if (oracle_check_params(num_blocks, words_per_block, word_bits, k) != 0)
        return -1;
    uint64_t patterns[16];
    uint32_t salts[ORACLE_MAX_K];
    oracle_salts(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint64_t blk = oracle_block_index(h, num_blocks);
        pattern_with_salts(h, words_per_block, word_bits, k, salts, patterns);
        for (uint32_t w = 0; w < words_per_block; ++w) {
            for (unsigned p = 0; p < word_bits; ++p) {
                if ((patterns[w] >> p) & 1ULL)
                    set_bit(filter, blk * words_per_block + w, word_bits, p);
            }
        }
    }
    return 0;
}

int oracle_contains(const uint8_t *filter, uint64_t num_blocks,
                    uint32_t words_per_block, uint32_t word_bits, uint32_t k,
                    uint64_t seed, const uint64_t *keys, uint64_t n,
                    uint8_t *out) {
    if (oracle_check_params(num_blocks, words_per_block, word_bits, k) != 0)
        return -1;
    uint64_t patterns[16];
    uint32_t salts[ORACLE_MAX_K];
    oracle_salts(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint64_t blk = oracle_block_index(h, num_blocks);
        pattern_with_salts(h, words_per_block, word_bits, k, salts, patterns);
        int all_set = 1;
        for (uint32_t w = 0; w < words_per_block; ++w) {
            for (unsigned p = 0; p < word_bits; ++p) {
                if (((patterns[w] >> p) & 1ULL) &&
                    !get_bit(filter, blk * words_per_block + w, word_bits, p))
                    all_set = 0;
            }
        }
        out[i] = (uint8_t)all_set;
    }
    return 0;
}

void oracle_clear(uint8_t *filter, uint64_t nbytes) {
    for (uint64_t i = 0; i < nbytes; ++i) filter[i] = 0;
}

int oracle_block_words(uint64_t num_blocks, uint32_t words_per_block,
                       uint32_t word_bits, uint32_t k, uint64_t seed,
                       const uint64_t *keys, uint64_t n, const uint64_t *sel,
                       uint64_t nsel, uint8_t *out) {
    if (oracle_check_params(num_blocks, words_per_block, word_bits, k) != 0)
        return -1;
    /* slot_of[blk] = 1 + position of blk in sel, 0 if blk is not selected. */
    uint32_t *slot_of = (uint32_t *)calloc(num_blocks, sizeof(uint32_t));
    if (!slot_of) return -1;
    for (uint64_t i = 0; i < nsel; ++i) {
        if (sel[i] >= num_blocks || slot_of[sel[i]] != 0 || nsel >= 0xFFFFFFFFULL) {
            free(slot_of);
            return -1;
        }
        slot_of[sel[i]] = (uint32_t)(i + 1);
    }
    uint64_t block_bytes = (uint64_t)words_per_block * (word_bits / 8);
    memset(out, 0, nsel * block_bytes);
    uint64_t patterns[16];
    uint32_t salts[ORACLE_MAX_K];
    oracle_salts(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint64_t blk = oracle_block_index(h, num_blocks);
        uint32_t slot = slot_of[blk];
        if (slot == 0) continue;
        pattern_with_salts(h, words_per_block, word_bits, k, salts, patterns);
        uint8_t *dst = out + (uint64_t)(slot - 1) * block_bytes;
        for (uint32_t w = 0; w < words_per_block; ++w) {
            for (unsigned p = 0; p < word_bits; ++p) {
                if ((patterns[w] >> p) & 1ULL) set_bit(dst, w, word_bits, p);
            }
        }
    }
    free(slot_of);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Classic (unblocked) filter, Sec. II-A-1.                                  */
/* ------------------------------------------------------------------------ */

void oracle_salts64(uint64_t out[ORACLE_MAX_K]) {
    for (uint32_t j = 0; j < ORACLE_MAX_K; ++j)
        out[j] = oracle_hash_key((uint64_t)j, ORACLE_SALT_SEED) | 1ULL;
}

static uint64_t classic_position_with_salt(uint64_t h, uint64_t num_bits, uint64_t salt) {
    uint64_t product = h * salt;                              /* mod 2^64 */
    return (uint64_t)(((unsigned __int128)product * num_bits) >> 64);
}

uint64_t oracle_classic_position(uint64_t h, uint64_t num_bits, uint32_t j) {
    uint64_t salts[ORACLE_MAX_K];
    oracle_salts64(salts);
    return classic_position_with_salt(h, num_bits, salts[j % ORACLE_MAX_K]);
}

static int classic_ok(uint64_t num_bits, uint32_t k) {
    return num_bits >= 64 && num_bits % 64 == 0 && k >= 1 && k <= ORACLE_MAX_K;
}

int oracle_classic_add(uint8_t *filter, uint64_t num_bits, uint32_t k, uint64_t seed,
                       const uint64_t *keys, uint64_t n) {
    if (!classic_ok(num_bits, k)) return -1;
    uint64_t salts[ORACLE_MAX_K];
    oracle_salts64(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        for (uint32_t j = 0; j < k; ++j) {
            uint64_t p = classic_position_with_salt(h, num_bits, salts[j]);
            filter[p / 8] = (uint8_t)(filter[p / 8] | (1u << (p % 8)));
        }
    }
    return 0;
}

int oracle_classic_contains(const uint8_t *filter, uint64_t num_bits, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n,
                            uint8_t *out) {
    if (!classic_ok(num_bits, k)) return -1;
    uint64_t salts[ORACLE_MAX_K];
    oracle_salts64(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        int all_set = 1;
        for (uint32_t j = 0; j < k; ++j) {
            uint64_t p = classic_position_with_salt(h, num_bits, salts[j]);
            if (!((filter[p / 8] >> (p % 8)) & 1)) all_set = 0;
        }
        out[i] = (uint8_t)all_set;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cache-sectorized filter, Sec. II-A-5.                                     */
/* ------------------------------------------------------------------------ */

int oracle_check_csbf_params(uint64_t num_blocks, uint32_t words_per_block,
                             uint32_t word_bits, uint32_t groups, uint32_t k) {
    uint32_t s = words_per_block, z = groups;
    if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return -1;
    if (!(word_bits == 32 || word_bits == 64)) return -1;
    if (!(z == 1 || z == 2 || z == 4 || z == 8 || z == 16) || z > s) return -1;
    if (k < z || k > ORACLE_MAX_K || k % z != 0) return -1;
    if (num_blocks < 1 || num_blocks > (1ULL << 32)) return -1;
    return 0;
}

void oracle_group_salts(uint32_t out[16]) {
    for (uint32_t g = 0; g < 16; ++g) {
        uint64_t h = oracle_hash_key((uint64_t)(32 + g), ORACLE_SALT_SEED);
        out[g] = (uint32_t)(h & 0xFFFFFFFFULL) | 1u;
    }
}

static unsigned log2u(uint32_t v) {
    unsigned r = 0;
    while ((1u << r) < v) ++r;
    return r;
}

/* Word index (within the block) of group g for hash low word lo. */
static uint32_t csbf_word(uint32_t lo, uint32_t s, uint32_t z, uint32_t g,
                          const uint32_t *gsalts) {
    uint32_t width = s / z;                 /* words per group */
    uint32_t sel = 0;
    if (width > 1) sel = (lo * gsalts[g]) >> (32u - log2u(width));
    return g * width + sel;
}

/* Apply (do_set) or test one key's bits in the block whose first word is
 * first_word.  Group g = j mod z receives bit j in its selected word. */
static int csbf_touch(uint8_t *filter, uint64_t first_word, uint64_t h, uint32_t s,
                      uint32_t S, uint32_t z, uint32_t k, const uint32_t *salts,
                      const uint32_t *gsalts, int do_set) {
    uint32_t lo = (uint32_t)(h & 0xFFFFFFFFULL);
    unsigned L = log2_word_bits(S);
    int all_set = 1;
    for (uint32_t j = 0; j < k; ++j) {
        uint32_t g = j % z;
        uint32_t w = csbf_word(lo, s, z, g, gsalts);
        unsigned p = (lo * salts[j]) >> (32u - L);
        if (do_set)
            set_bit(filter, first_word + w, S, p);
        else if (!get_bit(filter, first_word + w, S, p))
            all_set = 0;
    }
    return all_set;
}

int oracle_csbf_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
                    uint32_t word_bits, uint32_t groups, uint32_t k, uint64_t seed,
                    const uint64_t *keys, uint64_t n) {
    if (oracle_check_csbf_params(num_blocks, words_per_block, word_bits, groups, k) != 0)
        return -1;
    uint32_t salts[ORACLE_MAX_K], gsalts[16];
    oracle_salts(salts);
    oracle_group_salts(gsalts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint64_t blk = oracle_block_index(h, num_blocks);
        csbf_touch(filter, blk * words_per_block, h, words_per_block, word_bits, groups,
                   k, salts, gsalts, 1);
    }
    return 0;
}

int oracle_csbf_contains(const uint8_t *filter, uint64_t num_blocks,
                         uint32_t words_per_block, uint32_t word_bits, uint32_t groups,
                         uint32_t k, uint64_t seed, const uint64_t *keys, uint64_t n,
                         uint8_t *out) {
    if (oracle_check_csbf_params(num_blocks, words_per_block, word_bits, groups, k) != 0)
        return -1;
    uint32_t salts[ORACLE_MAX_K], gsalts[16];
    oracle_salts(salts);
    oracle_group_salts(gsalts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint64_t blk = oracle_block_index(h, num_blocks);
        out[i] = (uint8_t)csbf_touch((uint8_t *)filter, blk * words_per_block, h,
                                     words_per_block, word_bits, groups, k, salts, gsalts, 0);
    }
    return 0;
}

/* Selected 64-bit words of a classic filter, computed from the keys alone:
 * out[i] = word sel[i] (bits sel[i]*64 .. +63, little-endian) after adding
 * keys[0..n).  sel holds distinct word indices < num_bits / 64. */
int oracle_classic_words(uint64_t num_bits, uint32_t k, uint64_t seed,
                         const uint64_t *keys, uint64_t n, const uint64_t *sel,
                         uint64_t nsel, uint64_t *out) {
    if (!classic_ok(num_bits, k)) return -1;
    uint64_t nwords = num_bits / 64;
    uint32_t *slot_of = (uint32_t *)calloc(nwords, sizeof(uint32_t));
    if (!slot_of) return -1;
    for (uint64_t i = 0; i < nsel; ++i) {
        if (sel[i] >= nwords || slot_of[sel[i]] != 0) { free(slot_of); return -1; }
        slot_of[sel[i]] = (uint32_t)(i + 1);
        out[i] = 0;
    }
    uint64_t salts[ORACLE_MAX_K];
    oracle_salts64(salts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        for (uint32_t j = 0; j < k; ++j) {
            uint64_t p = classic_position_with_salt(h, num_bits, salts[j]);
            uint32_t slot = slot_of[p / 64];
            if (slot) out[slot - 1] |= 1ULL << (p % 64);
        }
    }
    free(slot_of);
    return 0;
}

/* Selected blocks of a cache-sectorized filter (as oracle_block_words). */
int oracle_csbf_block_words(uint64_t num_blocks, uint32_t words_per_block,
                            uint32_t word_bits, uint32_t groups, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n,
                            const uint64_t *sel, uint64_t nsel, uint8_t *out) {
    if (oracle_check_csbf_params(num_blocks, words_per_block, word_bits, groups, k) != 0)
        return -1;
    uint32_t *slot_of = (uint32_t *)calloc(num_blocks, sizeof(uint32_t));
    if (!slot_of) return -1;
    for (uint64_t i = 0; i < nsel; ++i) {
        if (sel[i] >= num_blocks || slot_of[sel[i]] != 0) { free(slot_of); return -1; }
        slot_of[sel[i]] = (uint32_t)(i + 1);
    }
    uint64_t block_bytes = (uint64_t)words_per_block * word_bits / 8;
    memset(out, 0, nsel * block_bytes);
    uint32_t salts[ORACLE_MAX_K], gsalts[16];
    oracle_salts(salts);
    oracle_group_salts(gsalts);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = oracle_hash_key(keys[i], seed);
        uint32_t slot = slot_of[oracle_block_index(h, num_blocks)];
        if (!slot) continue;
        /* The add rule, applied to the copy of the selected block. */
        csbf_touch(out, (uint64_t)(slot - 1) * words_per_block, h, words_per_block,
                   word_bits, groups, k, salts, gsalts, 1);
    }
    free(slot_of);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Chained pattern hashing (prior-art rule of Sec. IV-B).                    */
/* ------------------------------------------------------------------------ */

/* Sets (do_set) or tests the k bits of one key; returns 1 iff all were set. */
static int chained_touch(uint8_t *filter, uint64_t key, uint64_t seed, uint64_t num_blocks,
                         uint32_t s, uint32_t S, uint32_t k, int do_set) {
    uint64_t h = oracle_hash_key(key, seed);
    uint64_t blk = oracle_block_index(h, num_blocks);
    unsigned L = log2_word_bits(S);
    int all_set = 1;
    for (uint32_t j = 0; j < k; ++j) {
        h = oracle_hash_key(key, h);                       /* h_{j+1} */
        unsigned p = (uint32_t)(h & 0xFFFFFFFFULL) >> (32u - L);
        uint64_t word_index = blk * s + j % s;
        if (do_set)
            set_bit(filter, word_index, S, p);
        else if (!get_bit(filter, word_index, S, p))
            all_set = 0;
    }
    return all_set;
}

int oracle_chained_add(uint8_t *filter, uint64_t num_blocks, uint32_t words_per_block,
                       uint32_t word_bits, uint32_t k, uint64_t seed, const uint64_t *keys,
                       uint64_t n) {
    if (oracle_check_params(num_blocks, words_per_block, word_bits, k) != 0) return -1;
    for (uint64_t i = 0; i < n; ++i)
        chained_touch(filter, keys[i], seed, num_blocks, words_per_block, word_bits, k, 1);
    return 0;
}

int oracle_chained_contains(const uint8_t *filter, uint64_t num_blocks,
                            uint32_t words_per_block, uint32_t word_bits, uint32_t k,
                            uint64_t seed, const uint64_t *keys, uint64_t n, uint8_t *out) {
    if (oracle_check_params(num_blocks, words_per_block, word_bits, k) != 0) return -1;
    for (uint64_t i = 0; i < n; ++i)
        out[i] = (uint8_t)chained_touch((uint8_t *)filter, keys[i], seed, num_blocks,
                                        words_per_block, word_bits, k, 0);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Parquet split-block Bloom filter (the Apache Parquet format; the paper's  */
/* Arrow / Parquet-compatible configuration, Sec. I and Sec. VI).            */
/* ------------------------------------------------------------------------ */

/* The format's eight odd multipliers, one per word of a block. */
static const uint32_t PARQUET_SALT[8] = {
    0x47b6137bu, 0x44974d91u, 0x8824ad5bu, 0xa2b7289du,
    0x705495c7u, 0x2df1424bu, 0x9efc4947u, 0x5c6bfb31u,
};

static int parquet_ok(uint64_t num_bytes) {
    return num_bytes >= 32 && num_bytes % 32 == 0 && num_bytes / 32 <= (1ULL << 32);
}

/* The block a value maps to and the bit it sets in each of the block's
 * eight words. */
static uint64_t parquet_locate(uint64_t value, uint64_t num_blocks, unsigned bit[8]) {
    uint64_t h = oracle_hash_key(value, 0);       /* XXH64(8 LE bytes, seed 0) */
    uint32_t lo = (uint32_t)(h & 0xFFFFFFFFULL);
    for (int i = 0; i < 8; ++i) {
        uint32_t product = lo * PARQUET_SALT[i];  /* mod 2^32 */
        bit[i] = product >> 27;                   /* in [0, 32) */
    }
    return ((h >> 32) * num_blocks) >> 32;
}

int oracle_parquet_add(uint8_t *filter, uint64_t num_bytes, const uint64_t *values,
                       uint64_t n) {
    if (!parquet_ok(num_bytes)) return -1;
    uint64_t num_blocks = num_bytes / 32;
    unsigned bit[8];
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t blk = parquet_locate(values[v], num_blocks, bit);
        for (int i = 0; i < 8; ++i) set_bit(filter, blk * 8 + (uint64_t)i, 32, bit[i]);
    }
    return 0;
}

int oracle_parquet_contains(const uint8_t *filter, uint64_t num_bytes,
                            const uint64_t *values, uint64_t n, uint8_t *out) {
    if (!parquet_ok(num_bytes)) return -1;
    uint64_t num_blocks = num_bytes / 32;
    unsigned bit[8];
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t blk = parquet_locate(values[v], num_blocks, bit);
        int all_set = 1;
        for (int i = 0; i < 8; ++i)
            if (!get_bit(filter, blk * 8 + (uint64_t)i, 32, bit[i])) all_set = 0;
        out[v] = (uint8_t)all_set;
    }
    return 0;
}

int oracle_parquet_block_words(uint64_t num_bytes, const uint64_t *values, uint64_t n,
                               const uint64_t *sel, uint64_t nsel, uint8_t *out) {
    if (!parquet_ok(num_bytes)) return -1;
    uint64_t num_blocks = num_bytes / 32;
    uint32_t *slot_of = (uint32_t *)calloc(num_blocks, sizeof(uint32_t));
    if (!slot_of) return -1;
    for (uint64_t i = 0; i < nsel; ++i) {
        if (sel[i] >= num_blocks || slot_of[sel[i]] != 0 || nsel >= 0xFFFFFFFFULL) {
            free(slot_of);
            return -1;
        }
        slot_of[sel[i]] = (uint32_t)(i + 1);
    }
    memset(out, 0, nsel * 32);
    unsigned bit[8];
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t blk = parquet_locate(values[v], num_blocks, bit);
        uint32_t slot = slot_of[blk];
        if (slot == 0) continue;
        uint8_t *dst = out + (uint64_t)(slot - 1) * 32;
        for (int i = 0; i < 8; ++i) set_bit(dst, (uint64_t)i, 32, bit[i]);
    }
    free(slot_of);
    return 0;
}
