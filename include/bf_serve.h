/*
 * bf_serve.h -- a request loop serving bulk add / contains requests against
 * device-resident filters with continuous batching.
 *
 * Each request is one bulk operation of include/bf.h (paper Sec. II-A-4,
 * IV-B: hash, block, pattern, atomic OR or test) on one registered filter;
 * its result is exactly what that operation gives when the requests are run
 * one after another in submission order.  The server (a native scheduler
 * thread) keeps that meaning while it
 *   - admits requests in submission order whenever a launch slot is free and
 *     the request's payload (8 bytes per key, plus 1 result byte per key for
 *     contains) fits the HBM working budget still unused by requests in
 *     flight;
 *   - overlaps admitted work on several device streams (default priority);
 *   - orders work per filter: a contains waits for every earlier add on its
 *     filter, an add for every earlier contains on it (adds commute with
 *     each other);
 *   - coalesces runs of small requests of one kind into a single batched
 *     launch (the persistent kernel of include/bf_batch.h, one descriptor
 *     per request);
 * and reports per request when it arrived, was launched and was seen
 * complete.
 *
 * All registered filters must share words_per_block, word_bits and k.
 * Request keys and results are device pointers owned by the caller, which
 * keeps them alive until the request completes.  Streams are hipStream_t.
 */
#ifndef BF_SERVE_H
#define BF_SERVE_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_server bf_server;

typedef struct {
  uint64_t hbm_budget_bytes;      /* device bytes allowed in flight: keys, results and the
                                     workspace of partitioned adds (>= the largest request) */
  uint32_t max_inflight;          /* launches in flight at most (>= 1) */
  uint32_t nstreams;              /* device streams used (1..64) */
  uint64_t coalesce_max_keys;     /* requests of at most this many keys may share a launch (0: never) */
  uint32_t coalesce_max_requests; /* requests per shared launch at most (>= 1 when coalescing) */
  uint32_t coalesce_max_tiles;    /* tiles per shared launch at most (sizes device buffers) */
} bf_server_config_t;

typedef struct {
  uint32_t op;             /* BF_OP_ADD or BF_OP_CONTAINS */
  uint32_t filter;         /* index into the filters given at creation */
  const uint64_t *d_keys;  /* device, 8-byte aligned */
  uint64_t n;              /* keys (>= 1) */
  uint8_t *d_out;          /* device, n bytes; contains only */
  uint64_t arrival_ns;     /* replay only: arrival offset from the start of the replay */
} bf_request_t;

typedef struct {
  uint64_t arrival_ns;     /* ns since the replay (or server) start */
  uint64_t admit_ns;       /* launch enqueued */
  uint64_t complete_ns;    /* completion observed by the scheduler */
  uint32_t launch;         /* index of the launch that carried the request */
  int32_t status;          /* BF_OK, or why the request was refused */
} bf_request_result_t;

typedef struct {
  uint64_t requests;
  uint64_t launches;
  uint64_t coalesced_launches;    /* launches carrying more than one request */
  uint64_t peak_inflight_bytes;
  uint64_t peak_inflight_launches;
} bf_server_stats_t;

/* Creates a server over filters[0..nfilters) (which must outlive it) and
 * starts its scheduler thread.  cfg == NULL takes defaults (16 GiB budget,
 * 16 launches in flight, 8 streams, coalescing below 65,536 keys, up to 256
 * requests or 16,384 tiles per shared launch).  The filters must have the
 * sectorized layout of bf.h, one (s, S, k), one device and one salt table --
 * all of them Parquet filters (bf_parquet.h) or none (else BF_EUNSUPPORTED /
 * BF_EINVAL). */
bf_status bf_server_create(bf_filter *const *filters, uint32_t nfilters,
                           const bf_server_config_t *cfg, bf_server **out);

/* Online use: submits one request now (never blocks on the device); *id
 * receives its id (0, 1, 2, ... in submission order). */
bf_status bf_server_submit(bf_server *srv, const bf_request_t *req, uint64_t *id);

/* Waits until every submitted request has completed, then copies the
 * result of request ids[i] to results[i] for i < count (ids from
 * bf_server_submit). */
bf_status bf_server_wait(bf_server *srv, const uint64_t *ids, uint64_t count,
                         bf_request_result_t *results);

/* Replay: submits reqs[i] at reqs[i].arrival_ns after the call starts (the
 * calling thread keeps the schedule), waits for all of them and fills
 * results[i].  Times are relative to the start of the replay. */
bf_status bf_server_replay(bf_server *srv, const bf_request_t *reqs, uint64_t nreq,
                           bf_request_result_t *results);

/* The plain alternative: one request at a time in arrival order on one
 * stream, each launched when it has arrived and the previous one finished. */
bf_status bf_server_replay_serial(bf_server *srv, const bf_request_t *reqs, uint64_t nreq,
                                  bf_request_result_t *results);

bf_status bf_server_stats(const bf_server *srv, bf_server_stats_t *out);

/* Stops the scheduler (after in-flight work completes, waiting on the
 * server's own streams) and frees the server.  Releasing its pinned host
 * staging (hipHostFree) also waits for the rest of the device's work. */
bf_status bf_server_destroy(bf_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* BF_SERVE_H */
