/*
 * bf_variants.h -- C ABI: the filter layouts beside the sectorized one.
 *
 * Filters made here are used through the calls of bf.h (bf_add,
 * bf_contains, bf_clear, bf_export_words, bf_import_words, bf_info,
 * bf_set_mapping[_ex], bf_destroy), with the same conventions for pointers,
 * streams, errors and concurrency.  They are not accepted by batched plans
 * (bf_batch.h) or servers (bf_serve.h), which give BF_EUNSUPPORTED.  Adds
 * to a cache-sectorized filter, and to a classic filter with k in
 * {4, 6, 8, 12, 16} and at most 2^37 bits (each key then counts as k
 * records), choose between the direct and the partitioned strategy as bf.h
 * describes; other classic and all chained-hash adds are direct
 * (BF_STRATEGY_PARTITIONED gives BF_EUNSUPPORTED).
 *
 * Every layout takes the per-key base hash h = xxHash64 of the key's 8
 * little-endian bytes with the filter seed (paper Sec. IV-B).
 */
#ifndef BF_VARIANTS_H
#define BF_VARIANTS_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Classic Bloom filter of Sec. II-A-1: an array of m = num_bits bits; key x
 * sets (add) or tests (contains) the bits
 *   p_j = floor(((h * A_j) mod 2^64) * m / 2^64),   j = 0..k-1,
 * with the 64-bit odd salts A_j = xxHash64(LE64(j), 0x73746c61732d6662) | 1
 * (their low halves are the a_j of bf.h).  Bit p is bit p mod 8 of byte
 * p / 8 of the state.  num_bits: a multiple of 64, 64 <= num_bits <= 2^40;
 * 1 <= k <= 32.  Allocates num_bits / 8 bytes (zeroed synchronously).
 * Mapping: lanes_per_key = words_per_lane = 1, keys_per_lane in {1, 2, 4}. */
bf_status bf_create_classic(uint64_t num_bits, uint32_t k, uint64_t seed, bf_filter **out);

/* Cache-sectorized Bloom filter of Sec. II-A-5: blocks of s = words_per_block
 * S-bit words (layout, block rule and bit positions of bf.h) whose words form
 * z = groups groups of s/z consecutive words.  Key x uses, in group g, the
 * single word g*s/z + top log2(s/z) bits of (lo32(h) * c_g mod 2^32), with
 * c_g = (xxHash64(LE64(32 + g), 0x73746c61732d6662) mod 2^32) | 1 (the
 * further odd multiplier of Sec. V-A), and puts there its pattern bits j
 * with j mod z = g -- k/z bits per selected word.  z = s is exactly the
 * sectorized filter of bf.h.  z in {1,2,4,8,16}, z <= s; k a multiple of z
 * with z <= k <= 32; other parameters as bf_create.
 * Mapping: lanes_per_key THETA a power of two <= z (lane rank q owns groups
 * q*z/THETA .. (q+1)*z/THETA - 1, the s/z <= Phi rule of Sec. V-A);
 * words_per_lane 0 or s/THETA; keys_per_lane 1, or 2 with THETA = 1;
 * strategy as bf.h. */
bf_status bf_create_csbf(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                         uint32_t groups, uint32_t k, uint64_t seed, bf_filter **out);

/* Sectorized filter with chained pattern hashing, the rule of prior GPU
 * filters that Sec. IV-B replaces by multiplicative hashing; kept as the
 * baseline of the optimization breakdown (Sec. V-E).  Layout, parameters and
 * block rule as bf_create; bit j (j < k) is the top log2(S) bits of
 * lo32(h_{j+1}) with h_{j+1} = xxHash64(LE64(key), seed = h_j), h_0 the
 * base hash, in word j mod s.  One lane per key; the only mapping is the
 * default (set_mapping accepts lanes_per_key = 1, words_per_lane = s,
 * keys_per_lane = 1) and adds are always direct. */
bf_status bf_create_chained(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                            uint32_t k, uint64_t seed, bf_filter **out);

#ifdef __cplusplus
}
#endif

#endif /* BF_VARIANTS_H */
