/*
 * bf.h -- C ABI of the MI355X (gfx950) blocked / sectorized Bloom filter.
 *
 * The operations are those of the paper "Optimizing Bloom Filters on Modern
 * GPUs" (arXiv 2512.15595): bulk construction and bulk lookup of an
 * approximate-membership filter that never reports a false negative
 * (Sec. I, Sec. II-A-1), in the sectorized layout of Sec. II-A-4 (a block of
 * s contiguous S-bit words, one block per key, k pattern bits spread over
 * the words), with the per-key pattern generation of Sec. IV-B and the
 * tunable execution mapping of Sec. IV-A / IV-C.
 *
 * Definition computed (exactly; OR is commutative and idempotent, so every
 * execution order gives the same words):
 *   h      = xxHash64 of the key's 8 little-endian bytes with the filter seed;
 *   blk    = floor(hi32(h) * num_blocks / 2^32);
 *   a_j    = (xxHash64(LE64(j), 0x73746c61732d6662) mod 2^32) | 1, j < 32;
 *   bit j  = top log2(S) bits of (lo32(h) * a_j mod 2^32), in word j mod s,
 *            for j = 0..k-1;
 *   add      : word (blk, w) |= pattern word w, for all w;
 *   contains : 1 iff (word & pattern) == pattern for all w of the block.
 * Word (blk, w) lives at byte offset (blk*s + w) * S/8, little-endian.
 *
 * Conventions for every call:
 *   - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *     data_ptr); the caller owns them and keeps them alive until the stream
 *     has run the work.  Keys are 8-byte aligned uint64 values; results are
 *     one byte (0 or 1) per key.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue and return; they never synchronize, except bf_create
 *     (which zeroes the new words and waits for that).
 *   - Arguments are validated before anything is enqueued; on error nothing
 *     is enqueued and the status says why.  Launch failures are BF_EDEVICE.
 *     Faults inside a kernel surface at the caller's next synchronization.
 *   - Concurrency: bf_add calls on one filter from any streams commute, as
 *     OR does (Sec. II-A-1), under every construction strategy, with no
 *     events of the caller's: the library records each call's last use of
 *     the filter on its stream, makes a partitioned add (which loads whole
 *     64 KiB chunks of words and stores them back) wait for every earlier
 *     call on the filter, and makes a direct add wait for the last
 *     partitioned add.  The calls of one filter are enqueued under that
 *     filter's lock, so several host threads may call them at once.
 *     bf_contains, bf_clear, bf_export_words and bf_import_words are ordered
 *     by the caller against adds on other streams (stream order or events);
 *     a bf_contains not ordered after a bf_add may see any state between
 *     "before" and "after" that add.  Work enqueued while the stream is
 *     being captured into a HIP graph is ordered by the capturing caller
 *     (events recorded outside a capture cannot be waited on inside it).
 *     Batched plans (bf_batch.h) and servers (bf_serve.h) order their own
 *     launches; the caller orders them against bf.h calls on their filters.
 */
#ifndef BF_H
#define BF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bf_status;
#define BF_OK 0
#define BF_EINVAL (-1)        /* bad argument: nothing enqueued */
#define BF_ENOMEM (-2)        /* device allocation failed */
#define BF_EDEVICE (-3)       /* HIP runtime / launch error */
#define BF_EUNSUPPORTED (-4)  /* valid request this build has no kernel for */
#define BF_ESCRATCH (-5)      /* bf_add_noalloc: the add needs more workspace than
                                 BF_NOALLOC_SCRATCH_BYTES; nothing enqueued */

#define BF_OP_ADD 0
#define BF_OP_CONTAINS 1

typedef struct bf_filter bf_filter; /* opaque handle, owns the device words */

/* Construction strategies (bf_mapping_t.strategy, add only). */
#define BF_STRATEGY_AUTO 0        /* partitioned for dense batches, else direct */
#define BF_STRATEGY_DIRECT 1      /* one atomic OR group per key into the filter */
#define BF_STRATEGY_PARTITIONED 2 /* keys grouped by filter chunk; each chunk is
                                     updated in LDS and stored back */

/* Execution mapping of one operation (Sec. IV-A and IV-C).  A field left 0
 * means "use the default for this layout".
 *   lanes_per_key   Theta: lanes cooperating on one key, power of two <= 16;
 *   words_per_lane  Phi:   contiguous words per lane per step, power of two,
 *                          with Theta * Phi <= words_per_block;
 *   keys_per_lane   keys loaded and hashed per lane: 1, 2 or 4;
 *   atomic_bits     add only, 32-bit words only: 64 merges two adjacent
 *                   words into one 64-bit atomic OR (needs Phi >= 2); 32 or
 *                   0 otherwise;
 *   max_workgroups  grid cap of the grid-stride launch (0 = one workgroup
 *                   per workgroup_threads * keys_per_lane keys);
 *   strategy        add only: BF_STRATEGY_*.  The partitioned strategy
 *                   radix-partitions the keys by 64 KiB filter chunk and
 *                   updates each chunk in LDS, so a bulk add performs no
 *                   global atomics; it takes a workspace of 14-22 bytes per key
 *                   (about 6 for a filter of at most 1024 chunks, 64 MiB,
 *                   which is partitioned in one pass)
 *                   from a per-device stream-ordered memory pool and returns
 *                   it at its end on the same stream (no device
 *                   synchronization; the pool keeps its peak size reserved
 *                   for later adds); the library orders it against the
 *                   filter's other adds on any stream (see Concurrency).
 *                   Mapping fields other than strategy do not apply to it.
 *                   Results are identical;
 *   workgroup_threads threads per workgroup of the launch: 64, 128 or 256
 *                   (sectorized layout; the other layouts run 256).
 * The defaults come from a table measured on gfx950 per (operation, word
 * bits, words per block, filter size class, k, batch size class: up to 2^16
 * keys or more), so the mapping a call runs with may depend on n; bf_info
 * reports the one for large batches. */
typedef struct {
  uint32_t lanes_per_key;
  uint32_t words_per_lane;
  uint32_t keys_per_lane;
  uint32_t atomic_bits;
  uint32_t max_workgroups;
  uint32_t strategy;
  uint32_t workgroup_threads;
} bf_mapping_t;

/* Filter layouts (bf_info_t.layout).  bf_create makes the sectorized
 * layout; bf_variants.h creates the next three, bf_parquet.h the last. */
#define BF_LAYOUT_SECTORIZED 0       /* Sec. II-A-4 (s = 1: register-blocked) */
#define BF_LAYOUT_CLASSIC 1          /* Sec. II-A-1: k positions over m bits */
#define BF_LAYOUT_CACHE_SECTORIZED 2 /* Sec. II-A-5: one word per group of s/z */
#define BF_LAYOUT_SECTORIZED_CHAINED 3 /* sectorized, chained pattern hashing (Sec. IV-B prior art) */
#define BF_LAYOUT_PARQUET 4          /* sectorized 8 x 32, k = 8: the Parquet split-block format */

typedef struct {
  uint64_t num_blocks;     /* 0 for the classic layout */
  uint32_t words_per_block;/* 0 for the classic layout */
  uint32_t word_bits;      /* 32 for the classic layout (its word array) */
  uint32_t k;
  int32_t device;          /* HIP device the words live on */
  uint64_t seed;
  uint64_t size_bytes;     /* bytes of filter state */
  void *d_words;           /* device address of the words (owned by the filter) */
  bf_mapping_t mapping[2]; /* resolved mapping per op, indexed by BF_OP_* */
  uint32_t layout;         /* BF_LAYOUT_* */
  uint32_t groups;         /* z of the cache-sectorized layout, else 0 */
  uint64_t num_bits;       /* size_bytes * 8 */
} bf_info_t;

/* Creates a filter on the current HIP device with all words zero.
 * num_blocks in [1, 2^32]; words_per_block in {1,2,4,8,16}; word_bits in
 * {32, 64}; words_per_block <= k <= 32 (a sectorized block needs at least
 * one bit per word, Sec. II-A-5).  Allocates num_blocks * words_per_block *
 * word_bits / 8 bytes from the device's filter pool (stream-ordered,
 * returned to the device when released) and zeroes them before returning.
 * *out receives the handle (unchanged on error). */
bf_status bf_create(uint64_t num_blocks, uint32_t words_per_block,
                    uint32_t word_bits, uint32_t k, uint64_t seed,
                    bf_filter **out);

/* A filter over caller-owned device memory (e.g. a torch tensor): as
 * bf_create, but the words are d_words (nbytes must equal num_blocks *
 * words_per_block * word_bits / 8, 256-byte aligned) and are neither zeroed
 * nor freed by the library; the caller keeps them alive until bf_destroy.
 * Use it to adopt saved words in place or to place a filter in memory the
 * caller manages.  Allocates nothing on the device. */
bf_status bf_create_in(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                       uint32_t k, uint64_t seed, void *d_words, uint64_t nbytes,
                       bf_filter **out);

/* Releases the words behind every bf.h call enqueued on this filter, on any
 * stream, and frees the handle.  The words come from a per-device
 * stream-ordered pool and are released on a library stream that waits for
 * the filter's last uses, so the host returns at once and neither other
 * filters' work nor other streams are waited for (should the pool be
 * unavailable, the words are a plain allocation: bf_destroy then waits for
 * the filter's calls on the host before hipFree, which itself waits for the
 * device).  bf_create_in words stay the caller's: bf_destroy waits on the
 * host for the filter's calls and does not free them.  The caller must not
 * destroy a filter that a live batched plan or server still uses.  NULL is
 * accepted and ignored. */
bf_status bf_destroy(bf_filter *f);

/* Bulk construction: adds keys[0..n) (device pointer).  n = 0 is a no-op.
 * keys must be non-NULL when n > 0 and 8-byte aligned. */
bf_status bf_add(bf_filter *f, const uint64_t *d_keys, uint64_t n, void *stream);

/* Bulk lookup: d_out[i] = 1 if keys[i] may be in the filter, 0 if it is
 * certainly absent (Sec. II-A-1).  d_out is a device array of n bytes. */
bf_status bf_contains(const bf_filter *f, const uint64_t *d_keys, uint64_t n,
                      uint8_t *d_out, void *stream);

/* Sets every word to zero (a fill kernel on `stream`). */
bf_status bf_clear(bf_filter *f, void *stream);

/* Copies the filter words (size_bytes, layout as above) to `dst`, which
 * may be device or host memory of at least size_bytes bytes; asynchronous on
 * `stream` (host destinations should be pinned for true asynchrony).  With
 * bf_import_words this is the save / restore path of a filter. */
bf_status bf_export_words(const bf_filter *f, void *dst, uint64_t nbytes, void *stream);

/* Overwrites the filter words from `src` (device or host, nbytes must equal
 * size_bytes), asynchronous on `stream`. */
bf_status bf_import_words(bf_filter *f, const void *src, uint64_t nbytes, void *stream);

/* Parameters, size, word address and resolved mappings. */
bf_status bf_info(const bf_filter *f, bf_info_t *out);

/* Selects the execution mapping of one operation; results do not depend on
 * it.  lanes_per_key = words_per_lane = keys_per_lane = 0 restores the
 * default.  Invalid combinations give BF_EINVAL. */
bf_status bf_set_mapping(bf_filter *f, int op, uint32_t lanes_per_key,
                         uint32_t words_per_lane, uint32_t keys_per_lane);

/* Full form of bf_set_mapping (all fields of bf_mapping_t). */
bf_status bf_set_mapping_ex(bf_filter *f, int op, const bf_mapping_t *m);

/* The construction strategy bf_add(f, keys, n, ...) takes with f's current
 * add mapping: BF_STRATEGY_DIRECT or BF_STRATEGY_PARTITIONED, the automatic
 * choice resolved by the measured crossover (partitioned from about 1.5 M
 * keys + filter bytes / 80; for the classic layout n counts k records per
 * key).  For callers that plan workspace memory (14-22 bytes per key for a
 * partitioned add, about 6 into a filter of at most 64 MiB).  Host only:
 * enqueues nothing and touches no device.
 * BF_EINVAL if f or out is NULL. */
bf_status bf_add_strategy(const bf_filter *f, uint64_t n, uint32_t *out);

/* The mapping (and, for add, the construction strategy) that a sectorized
 * filter of these parameters would run an operation of n keys with by
 * default: the tuned row of (op, word_bits, words_per_block, size class of
 * num_blocks * words_per_block * word_bits / 8 bytes, k, batch class of n)
 * and, for add, the measured crossover of the layout.  Host only: touches no
 * device.  BF_EINVAL for parameters bf_create rejects or a NULL out. */
bf_status bf_tuned_mapping(int op, uint64_t num_blocks, uint32_t words_per_block,
                           uint32_t word_bits, uint32_t k, uint64_t n, bf_mapping_t *out);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: bf_add with
 * the same result, whose partitioned construction takes its workspace from
 * a static device array of BF_NOALLOC_SCRATCH_BYTES instead of the memory
 * pool.  It calls no hipMalloc, hipFree or other device allocation (the
 * first call on a device resolves the array's address and creates one
 * event; a filter's first call on a stream creates that stream's event, as
 * every bf.h call does).  Each device holds one array, loaded with the
 * library's code on the first call there and kept until the process ends.
 * An add the automatic rule builds directly (one atomic OR group per key)
 * needs no workspace and is bf_add itself.  A partitioned add must fit one
 * pass of the array (at most 2^28 records; the workspace is about 6 bytes
 * per key into a filter of at most 64 MiB, which is partitioned in one
 * pass, so up to about 43 M keys, and 14-22 bytes per key into a larger
 * one, the most for few keys into a large filter, so about 12 M into a
 * 1 GiB filter):
 * larger adds give BF_ESCRATCH with nothing enqueued.  Calls on one device
 * share the array, which keeps the last call's contents (the kernels clear
 * the counters they need): outside graph capture the library orders them
 * with one event per device, so they never overlap; calls captured into
 * graphs are ordered by their caller, and captured calls that overlap on
 * one device race on the array.  The current device must be the filter's
 * (else BF_EINVAL). */
#define BF_NOALLOC_SCRATCH_BYTES (256ull << 20)
bf_status bf_add_noalloc(bf_filter *f, const uint64_t *d_keys, uint64_t n, void *stream);

/* Static description of a status code. */
const char *bf_strerror(bf_status s);

#ifdef __cplusplus
}
#endif

#endif /* BF_H */
