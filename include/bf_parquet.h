/*
 * bf_parquet.h -- C ABI: the Apache Parquet split-block Bloom filter, the
 * Arrow / Parquet-compatible configuration the paper names as its production
 * use (Sec. I and Sec. VI: row-group pruning of Parquet scans).
 *
 * The format is a sectorized filter of bf.h with words_per_block = 8,
 * word_bits = 32, k = 8 and seed 0, whose pattern multipliers are the
 * format's eight odd constants
 *   c = 0x47b6137b 0x44974d91 0x8824ad5b 0xa2b7289d
 *       0x705495c7 0x2df1424b 0x9efc4947 0x5c6bfb31
 * instead of the a_j of bf.h:
 *   h     = xxHash64 of the value's 8 little-endian bytes, seed 0;
 *   blk   = floor(hi32(h) * num_blocks / 2^32), num_blocks = num_bytes / 32;
 *   add   : word i of block blk |= 1 << ((lo32(h) * c_i mod 2^32) >> 27),
 *           i = 0..7;
 *   contains: 1 iff all eight bits are set.
 * The words (word (blk, i) at byte (8 * blk + i) * 4, little-endian) are
 * byte for byte the bitset a Parquet file stores after a column chunk's
 * bloom filter header, so a filter built here can be written into a file and
 * a file's filter can be loaded here (bf_import_words or
 * bf_create_parquet_in) and queried in bulk.  Values are the 8-byte physical
 * types: INT64 (two's complement) and DOUBLE (IEEE-754 bits) hash their
 * plain encoding, which is the key's 8 bytes; 4-byte and variable-length
 * types hash other encodings and are not covered.
 *
 * Filters made here use the calls of bf.h (bf_add, bf_contains, bf_clear,
 * bf_export_words, bf_import_words, bf_info, bf_set_mapping[_ex],
 * bf_add_strategy, bf_add_noalloc, bf_destroy) with its conventions; every
 * mapping of the 8 x 32-bit, k = 8 sectorized layout applies, and adds
 * choose between the direct and the partitioned construction by the same
 * measured crossover.  bf_info reports layout BF_LAYOUT_PARQUET.  Batched
 * plans (bf_batch.h) and servers (bf_serve.h) take them -- the pruning shape
 * of a Parquet scan, a few values looked up in the filter of every row
 * group, is one batched lookup -- provided every filter of the plan or
 * server is a Parquet filter (else BF_EINVAL).
 */
#ifndef BF_PARQUET_H
#define BF_PARQUET_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A zeroed Parquet split-block filter of num_bytes bytes on the current HIP
 * device.  num_bytes: a multiple of 32 in [32, 2^37] (the format's writers
 * use powers of two up to 128 MiB; a header encodes at most 2^31 - 1).
 * Allocation as bf_create; *out unchanged on error. */
bf_status bf_create_parquet(uint64_t num_bytes, bf_filter **out);

/* The same over caller-owned device words (for instance a bitset read from a
 * file): d_words 256-byte aligned, num_bytes as above; neither zeroed nor
 * freed by the library (bf_create_in's contract). */
bf_status bf_create_parquet_in(void *d_words, uint64_t num_bytes, bf_filter **out);

/* The format's bloom filter header (BloomFilterHeader in the Thrift compact
 * protocol: numBytes = num_bytes, algorithm BLOCK, hash XXHASH, compression
 * UNCOMPRESSED) that precedes the bitset in a file.  Writes at most cap
 * bytes to out (host memory) and the header length to *len (at most 20
 * bytes).  BF_EINVAL for a num_bytes that is not a multiple of 32 in
 * [32, 2^31 - 1], a NULL pointer or cap < *len.  Host only. */
bf_status bf_parquet_header(uint64_t num_bytes, uint8_t *out, uint64_t cap, uint64_t *len);

/* Reads a bloom filter header at the start of blob (len bytes, host
 * memory): *num_bytes receives numBytes and *header_len the header's
 * length, so the bitset is blob[*header_len, *header_len + *num_bytes).
 * Fields the format may add are skipped.  BF_EINVAL for a NULL pointer, a
 * truncated or malformed header, or numBytes not a positive multiple of 32;
 * BF_EUNSUPPORTED for an algorithm, hash or compression other than BLOCK,
 * XXHASH and UNCOMPRESSED.  Host only. */
bf_status bf_parquet_parse_header(const uint8_t *blob, uint64_t len, uint64_t *num_bytes,
                                  uint64_t *header_len);

#ifdef __cplusplus
}
#endif

#endif /* BF_PARQUET_H */
