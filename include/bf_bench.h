/*
 * bf_bench.h -- C ABI of the random-access roofline microbenchmarks.
 *
 * The paper expresses DRAM-resident filter throughput as a fraction of a
 * measured random-access bound: random 64-bit loads / stores in giga-updates
 * per second (GUPS), drawn as the "SOL" line of its throughput figures
 * (Sec. V-B).  These kernels measure that bound on the local GPU at the
 * access shapes of the filter kernels, so that add and contains can be
 * reported against it.  Each call enqueues one kernel on `stream` (a
 * hipStream_t passed as void*; NULL = null stream) and returns; the caller
 * times it with events.  All pointers are device pointers owned by the
 * caller.  Segment addresses are uniform over the buffer and aligned to the
 * segment size.  Return values: BFB_OK, BFB_EINVAL (bad argument or an
 * unsupported shape; nothing enqueued), BFB_EDEVICE (launch failed).
 */
#ifndef BF_BENCH_H
#define BF_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFB_OK 0
#define BFB_EINVAL (-1)
#define BFB_EDEVICE (-3)

/* n_access random aligned reads of seg_bytes bytes from buf (buf_bytes
 * bytes, buf_bytes / seg_bytes <= 2^32 segments).  Each segment is read by
 * lanes_per_seg adjacent lanes.  Shapes (seg_bytes, lanes_per_seg):
 * (4,1) (8,1) (16,1) (32,1) (32,2) (64,1) (64,4) (128,1) (128,8).
 * Addresses come from an in-register hash of the access number and seed.
 * sink: one device uint32 that is practically never written (keeps the
 * loads alive).  n_access <= 2^32. */
int bfb_random_read(const void *d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                    uint32_t lanes_per_seg, uint64_t n_access, uint32_t seed,
                    uint32_t *d_sink, void *stream);

/* As bfb_random_read with one lane per segment (seg_bytes 32 or 128), each
 * 16-byte load issued with a cache policy: 1 = nontemporal hint, 2 = sc1,
 * 3 = sc0 sc1, 4 = nt sc1 (gfx950 cache-coherence / temporal bits). */
int bfb_random_read_policy(const void *d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                           uint32_t policy, uint64_t n_access, uint32_t seed,
                           uint32_t *d_sink, void *stream);

/* Writes n uniform random segment indices in [0, nseg) (nseg <= 2^32). */
int bfb_fill_random_index(uint64_t *d_idx, uint64_t n, uint64_t nseg, uint32_t seed,
                          void *stream);

/* Lookup-shaped gather: for each i < n reads segment d_idx[i] (seg_bytes in
 * {8,16,32,64,128}) and writes one byte d_out[i]; 8 index bytes are
 * streamed in and 1 byte out per access.  Indices >= buf_bytes / seg_bytes
 * read nothing and give 0. */
int bfb_random_read_indexed(const void *d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                            const uint64_t *d_idx, uint64_t n, uint8_t *d_out, void *stream);

/* n_access random aligned atomic ORs on seg_bytes-byte segments; the
 * segment is covered by lanes_per_seg lanes, each issuing seg_bytes /
 * lanes_per_seg / 8 sequential 64-bit atomics (or one 32-bit atomic for
 * 4-byte lanes).  Shapes: (4,1) (8,1) (32,1) (32,4) (32,8) (64,8) (128,16).
 * The buffer contents change (bits are set). */
int bfb_random_atomic_or(void *d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                         uint32_t lanes_per_seg, uint64_t n_access, uint32_t seed,
                         void *stream);

/* GUPS: n_updates random 64-bit words of buf are loaded, xor-ed and stored
 * (non-atomic, as in the HPC Challenge RandomAccess kernel). */
int bfb_gups(void *d_buf, uint64_t buf_bytes, uint64_t n_updates, uint32_t seed, void *stream);

/* Seeded synthetic keys on the device (workload generation, not part of
 * the filter method).  SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): element
 * i of stream `seed` is the SplitMix64 output function of
 * seed + (i + 1) * 0x9E3779B97F4A7C15.  Writes elements first..first+n-1. */
int bfb_fill_splitmix64(uint64_t *d_out, uint64_t n, uint64_t seed, uint64_t first, void *stream);

/* Lookup keys with a hit fraction: out[i] is, when the upper half of mix
 * element i is below hit_q32, source element src_first + j with
 * j = floor(lo32(mix element i) * src_count / 2^32), else fresh element
 * fresh_first + i. */
int bfb_fill_mixed_queries(uint64_t *d_out, uint64_t n, uint64_t src_seed, uint64_t src_first,
                           uint32_t src_count, uint64_t fresh_seed, uint64_t fresh_first,
                           uint32_t hit_q32, uint64_t mix_seed, void *stream);

/* Streaming copy of `bytes` (a multiple of 16) from src to dst. */
int bfb_copy(void *d_dst, const void *d_src, uint64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BF_BENCH_H */
