/*
 * bf_batch.h -- batched bulk add / contains over many independent filters in
 * one persistent launch, replayed from a HIP graph.
 *
 * The per-key operation is exactly that of bf_add / bf_contains (include/
 * bf.h; paper Sec. II-A-4, IV-B), applied to each filter with its own words,
 * block count and seed; only the launch changes.  A plan groups the work of
 * many filters (for instance thousands of filters of uneven sizes) into
 * fixed-size tiles, orders them so that the tiles of one filter run
 * together on one XCD (the filter stays hot in that XCD's L2), picks each
 * tile's execution mapping (paper Sec. IV-A: lanes per key, words per lane,
 * keys per lane) by the filter's size class from the autotuned table, and
 * records one persistent kernel launch in a HIP graph.
 *
 * An add plan with enough keys on filters that are dense (at least their
 * bytes / 80 keys each: the per-filter form of the BF_STRATEGY_AUTO rule in
 * bf.h) and at least 512 chunks among them is instead planned as one
 * partitioned construction over the dense filters: the filters' blocks are
 * laid end to end in one block space, one radix partition groups their keys
 * by 64 KiB chunk, and each chunk is updated in LDS (four kernels in the
 * graph); the keys of the sparse filters go to the tiled launch, recorded
 * after them, so no sparse filter's words are streamed.  Filter 0's add
 * strategy (bf_set_mapping_ex) can force BF_STRATEGY_DIRECT (tiles only) or
 * BF_STRATEGY_PARTITIONED (every filter partitioned).  Launches of a plan
 * (all three forms) are ordered by the caller against other work on its
 * filters -- stream order or events; they take no part in the per-filter
 * stream order of bf.h calls.
 *
 * All filters of a plan must share words_per_block, word_bits and k.  Keys
 * of filter i are d_keys[h_offsets[i] .. h_offsets[i+1]) (device memory,
 * one concatenated array); lookup results go to d_out at the same offsets.
 * The plan keeps the device pointers: the caller keeps the filters, keys
 * and results alive and unmoved while the plan is used, and may change the
 * key values in place between launches.  Calls validate first (BF_EINVAL,
 * nothing enqueued); plan creation allocates and synchronizes; launches only
 * enqueue on `stream` (a hipStream_t as void*, NULL = null stream).
 */
#ifndef BF_BATCH_H
#define BF_BATCH_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_batch bf_batch;

typedef struct {
  uint32_t op;             /* BF_OP_ADD or BF_OP_CONTAINS */
  uint32_t nfilters;
  uint64_t nkeys;          /* h_offsets[nfilters] - h_offsets[0] */
  uint64_t ntiles;         /* tile slots in the launch (including padding); of a
                              partitioned plan: those of its sparse filters */
  uint32_t grid;           /* workgroups of the persistent launch (first pass if
                              partitioned with no tiles) */
  uint32_t tiles_per_class[3]; /* L2 / Infinity-Cache / HBM sized filters */
  bf_mapping_t mapping[3]; /* mapping compiled in per size class */
  uint32_t strategy;       /* BF_STRATEGY_DIRECT (tiles) or BF_STRATEGY_PARTITIONED */
} bf_batch_info_t;

/* Plans one batched operation (op = BF_OP_ADD or BF_OP_CONTAINS) over
 * filters[0..nfilters).  h_offsets is a host array of nfilters + 1
 * non-decreasing key offsets; d_out is required for contains and ignored for
 * add.  Every filter must have the sectorized layout of bf.h, with one
 * (s, S, k), one device and one salt table -- all of them Parquet filters
 * (bf_parquet.h) or none (else BF_EUNSUPPORTED / BF_EINVAL).  On success
 * *out receives the plan. */
bf_status bf_batch_plan(int op, bf_filter *const *filters, uint32_t nfilters,
                        const uint64_t *d_keys, const uint64_t *h_offsets,
                        uint8_t *d_out, bf_batch **out);

/* Replays the plan's HIP graph (one persistent kernel launch) on `stream`. */
bf_status bf_batch_launch(bf_batch *b, void *stream);

/* Launches the same persistent kernel directly, without the graph (for
 * callers that capture it into graphs of their own). */
bf_status bf_batch_launch_direct(bf_batch *b, void *stream);

/* The plain alternative the batch replaces: the launch a bf_add /
 * bf_contains of each filter's keys makes, one per filter, in filter order,
 * each with the filter's own mapping and strategy. */
bf_status bf_batch_launch_per_filter(bf_batch *b, void *stream);

bf_status bf_batch_info(const bf_batch *b, bf_batch_info_t *out);

/* Frees the plan.  The host waits for the plan's own launches
 * (bf_batch_launch and bf_batch_launch_direct on streams that were not
 * being captured) and for no other work of the device; the plan's device
 * memory then returns to the device in stream order.  A graph of the
 * caller's that captured bf_batch_launch_direct must not run after this
 * call.  NULL is ignored. */
bf_status bf_batch_destroy(bf_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* BF_BATCH_H */
