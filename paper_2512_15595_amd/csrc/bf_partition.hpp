// bf_partition.hpp -- partitioned construction: bulk add without global
// atomics on the filter.
//
// On gfx950 a device-scope atomic OR is executed beyond the XCD's L2, and
// the device sustains only ~20 G such requests per second from HBM; direct
// construction (one atomic group per key) is bound by that rate.  This path
// instead groups the keys by filter chunk -- a range of blocks whose words
// fit in LDS -- and lets one workgroup own each chunk: it loads the chunk
// into LDS, ORs the patterns of its keys with LDS atomics, and writes the
// chunk back with plain coalesced stores.  The filter words it writes are
// exactly those of the direct path (OR is commutative and idempotent).
//
// Grouping is a two-digit radix partition of the chunk index (the CPU
// filter the paper compares with partitions keys by radix for the same
// reason, Sec. V-A), into fixed-capacity buckets:
//   scatter1  keys -> hashed records (block << 32 | lo32) into high-digit
//             buckets;                                        [8 B in, 8 out]
//   scatter2  records -> chunk buckets as (lo32, block within the chunk)
//             pairs in two arrays;                            [8 in, 6 out]
//   apply     per chunk: LDS load, LDS atomic OR, store;      [6 in + chunk]
// A filter of at most kChunkDigits chunks (64 MiB) needs one digit: its
// first pass groups the hashed records by chunk straight into the chunk
// buckets, and the second pass is skipped.
// Each scatter step counting-sorts kPartStep records in LDS, so a digit
// leaves the step as one contiguous run.  Where the run goes:
//   chunk buckets, and the high-digit buckets of multi-filter plans (whose
//     buckets expect uneven loads): one returning atomic add per digit and
//     step reserves the run in a shared bucket;
//   high-digit buckets of one filter (sliced): every first-pass workgroup w
//     owns a private slice (d, w) of every high-digit bucket d and advances
//     an LDS fill counter per digit; at its end it publishes the slices'
//     record counts, and the second pass reads a bucket as the
//     concatenation of its slices (prefix sums of the counts in LDS).  All
//     first-pass workgroups would otherwise update the same f1 counters
//     every step; slicing them took the first pass from 1.65 to 1.36 ms for
//     2^28 keys on MI355X.
// Capacities cover the expected count of uniformly hashed keys plus six
// standard deviations; a record that finds its slice or bucket full
// (repeated keys can do that) is applied at once with direct global atomics
// instead, so results never depend on the capacities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bf_hash.hpp"
#include "bf_kernels.hpp"
#include "bf_variant_kernels.hpp"

namespace bfhip {

constexpr int kPartStep = 8192;                     // records per LDS-staged scatter step
// Workgroup shapes of the scatter passes (threads; each thread holds
// kPartStep / threads records of a step).  Measured on MI355X, one wide
// workgroup per CU with a long step beats several narrow ones: both passes
// run 16 waves of 8 records (a step's 64 KiB stage and the digit tables
// take 88 of the CU's 160 KiB of LDS); the classic first pass keeps 16
// records per thread for up to 16 positions per key.
constexpr int kScatter1Threads = 1024;
constexpr int kScatter2Threads = 1024;
constexpr int kClassicThreads = 512;
constexpr int kZeroThreads = 256;
constexpr int kApplyThreads = 1024;                 // apply: 16 waves share one chunk
constexpr int kChunkBytes = 64 * 1024;              // LDS bytes owned per chunk
constexpr int kSpareSlots = 64;                     // spare record slots per record array (one per lane)
constexpr int kMaxDigits = 1024;                    // digit fan-out limit of the first pass
constexpr int kMaxDigits2 = 512;                    // ... and of the second (chunks per high digit)
constexpr int kChunkDigits = kMaxDigits;            // chunks up to which the first pass writes chunk buckets
constexpr int kMaxSlices = 1024;                    // slices one sliced-mode reader concatenates
constexpr int kVecPerThread = kChunkBytes / 16 / kApplyThreads;  // 16-byte chunk vectors per apply thread
static_assert(kVecPerThread * 16 * kApplyThreads == kChunkBytes, "apply covers a chunk exactly");

// One filter of a multi-filter partitioned add.  Its blocks occupy global
// blocks [block_base, block_base + num_blocks) and its chunks global chunks
// from chunk_base (block_base is a multiple of the blocks per chunk); its
// keys are keys[key_begin, key_end).  A `direct` filter (few keys for its
// size) takes no part: its keys are left to a direct launch, so none of its
// chunks is read or written here.
struct PartFilter {
  void* words;
  uint64_t hash_init;
  uint32_t nb_lo;
  uint32_t nb_hi_mask;
  uint64_t num_blocks;
  uint64_t block_base;
  uint64_t chunk_base;
  uint64_t key_begin;
  uint64_t key_end;
  uint32_t direct;
  uint32_t reserved;
};

struct PartArgs {
  // the single filter (nfilters == 1) ...
  void* words;
  uint64_t num_blocks;
  uint64_t hash_init;
  uint32_t nb_lo;
  uint32_t nb_hi_mask;
  // ... or a table of filters (nfilters > 1) sharing one layout and k
  const PartFilter* filters;
  const uint32_t* chunk_owner;  // global chunk -> filter
  const struct PartRange* work1;  // first-pass workgroup -> its keys (one filter's)
  uint32_t nwork1;
  uint32_t nfilters;
  uint32_t k;
  uint32_t chunk_shift;  // log2(blocks per chunk)
  uint32_t low_bits;     // bits of the low (second-pass) digit
  uint32_t f1;           // high digits
  uint32_t f2;           // low digits = 1 << low_bits
  uint32_t q;            // second-pass workgroups per high-digit bucket
  uint64_t chunks;
  const uint64_t* keys;
  uint64_t n;
  uint64_t range1;       // keys per first-pass workgroup (multiple of kPartStep)
  uint64_t* buf1;        // f1 buckets of cap1 records (or per off1)
  unsigned long long* fill1;
  uint64_t cap1;
  uint32_t* buf2;        // chunk buckets of cap2 records (or per off2): lo32 ...
  uint16_t* blk2;        // ... and block within the chunk (a chunk has at most 2^14 blocks)
  unsigned long long* fill2;
  uint64_t cap2;
  // optional per-bucket extents (multi-filter plans, whose chunks expect
  // different loads): bucket d spans [off[d], off[d + 1]) of its buffer
  const uint64_t* off1;
  const uint64_t* off2;
  // optional work lists splitting heavily loaded buckets over several
  // workgroups (multi-filter plans); without them the second pass uses q
  // slices per high digit and the apply one workgroup per chunk
  const struct PartWork* work2;
  uint32_t nwork2;
  const struct PartWork* work3;
  uint32_t nwork3;
  // without a work list: apply slices per chunk (> 1 for filters of few
  // chunks, so the apply grid still fills the device)
  uint32_t apply_split;
  // classic filter (Z = -1 rule): m and, for a power-of-two m, 64 - log2(m)
  uint64_t num_bits;
  uint32_t bit_shift;
  // sliced high-digit buckets (one filter, no offsets or work lists), when
  // cs1 > 0: buf1 holds f1 * g1 slices of cs1 records (slice d * g1 + w:
  // digit d of pass-1 workgroup w) and fill1 their counts, each written
  // once by the slice's owner
  uint32_t g1;           // pass-1 workgroups
  uint64_t cs1;
  // first of 64 spare record slots at the end of buf1 / of buf2 and blk2:
  // a store loop writes every lane's record slot on every step, those of
  // no record to a spare one, so that the number of stores per step is
  // fixed (see scatter_step_masked)
  uint64_t spare1;
  uint64_t spare2;
};

// The keys [begin, end) of filter `filter`: one first-pass workgroup of a
// multi-filter plan (at most range1 keys, never more than one filter's).
struct PartRange {
  uint64_t begin;
  uint64_t end;
  uint32_t filter;
  uint32_t reserved;
};

// One unit of work: slice `split` of `nsplit` of bucket `bucket`.
struct PartWork {
  uint32_t bucket;
  uint16_t split;
  uint16_t nsplit;
};

__device__ __forceinline__ uint64_t bucket1_base(const PartArgs& a, uint32_t d) {
  return a.off1 ? a.off1[d] : static_cast<uint64_t>(d) * a.cap1;
}
__device__ __forceinline__ uint64_t bucket1_cap(const PartArgs& a, uint32_t d) {
  return a.off1 ? a.off1[d + 1] - a.off1[d] : a.cap1;
}
__device__ __forceinline__ uint64_t bucket2_base(const PartArgs& a, uint64_t c) {
  return a.off2 ? a.off2[c] : c * a.cap2;
}
__device__ __forceinline__ uint64_t bucket2_cap(const PartArgs& a, uint64_t c) {
  return a.off2 ? a.off2[c + 1] - a.off2[c] : a.cap2;
}

__device__ __forceinline__ uint32_t rec_block(uint64_t r) { return static_cast<uint32_t>(r >> 32); }
__device__ __forceinline__ uint32_t rec_lo(uint64_t r) { return static_cast<uint32_t>(r); }

template <typename W>
__device__ __forceinline__ void lds_or(W* p, W v) {
  if constexpr (sizeof(W) == 8)
    atomicOr(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
  else
    atomicOr(reinterpret_cast<unsigned int*>(p), static_cast<unsigned int>(v));
}

// LDS position of word f (of width 4 * PER bytes) of chunk-local block lb:
// word f ^ key(lb) of the block.  With 64 four-byte banks, a block of
// S_WORDS * PER banks starts in one of G = 64 / (S_WORDS * PER) bank groups,
// chosen by the low log2(G) bits of lb.  One LDS instruction of an apply
// touches word f of 64 random blocks.  Unswizzled, they all sit in the G
// banks word f can occupy; keyed by lb mod s, the word within the group is
// still a function of the same low bits, so they reach only max(G, s) banks
// (8 for 8 x 32-bit blocks; measured on MI355X: 82 % of LDS-active cycles
// in bank conflicts).  Keyed by the bits above the group bits,
// key = (lb >> log2 G) mod s, the group and the word within it are
// independent and the lanes spread over all banks (also over 32 banks).
constexpr int log2_floor(int v) { return v > 1 ? 1 + log2_floor(v / 2) : 0; }
template <int S_WORDS, int PER = 1>
__device__ __forceinline__ uint32_t lds_key(uint32_t lb) {
  constexpr int kGroups = 64 / (S_WORDS * PER) > 1 ? 64 / (S_WORDS * PER) : 1;
  return (lb >> log2_floor(kGroups)) & (S_WORDS - 1);
}
template <int S_WORDS, int PER = 1>
__device__ __forceinline__ uint32_t lds_word(uint32_t lb, uint32_t f) {
  return (lb * S_WORDS) | (f ^ lds_key<S_WORDS, PER>(lb));
}
// The same for a 32-bit index t into the chunk image (W of width 4 * PER).
template <int S_WORDS, int PER>
__device__ __forceinline__ uint32_t lds_u32(uint32_t t) {
  const uint32_t e = t / PER;
  return lds_word<S_WORDS, PER>(e / S_WORDS, e & (S_WORDS - 1)) * PER + t % PER;
}

// What a record does to its block, per layout: Z = 0 is the sectorized
// filter (every word of the block gets its pattern), Z > 0 the
// cache-sectorized filter with Z groups (one word per group; `k` then
// carries the bits per selected word).  add_global is the direct fallback
// (device-scope atomics), add_lds the apply step on a block held in LDS.
template <typename W, int S_WORDS, int K, int Z>
struct BlockRule {
  CsbfLane<W, S_WORDS, Z, K, 1> ln;
  __device__ __forceinline__ BlockRule() : ln(0) {}
  __device__ __forceinline__ void add_global(W* words, uint32_t blk, uint32_t lo, uint32_t k) const {
    csbf_add_block<W, S_WORDS, Z, K, 1>(words, blk, lo, ln, k);
  }
  __device__ __forceinline__ void add_lds(W* lds, uint32_t lb, uint32_t lo, uint32_t k) const {
#pragma unroll
    for (int i = 0; i < Z; ++i)
      lds_or<W>(&lds[lds_word<S_WORDS, sizeof(W) / 4>(lb, ln.word(i, lo))], ln.pattern(i, lo, k));
  }
};

template <typename W, int S_WORDS, int K>
struct BlockRule<W, S_WORDS, K, 0> {
  LanePatterns<W, S_WORDS, K, 1, S_WORDS> lp;
  __device__ __forceinline__ BlockRule() : lp(0) {}
  __device__ __forceinline__ void add_global(W* words, uint32_t blk, uint32_t lo, uint32_t k) const {
    add_block<W, S_WORDS, K, 1, S_WORDS, false>(words, blk, lo, lp, k);
  }
  __device__ __forceinline__ void add_lds(W* lds, uint32_t lb, uint32_t lo, uint32_t k) const {
    if constexpr (sizeof(W) == 4 && S_WORDS >= 2) {
      // Words f and f + 1 (f even) sit at positions f ^ key and (f ^ key) ^ 1
      // of the block: one aligned 8-byte pair, so one 64-bit LDS atomic
      // covers both (their order within it flips with the key's low bit).
      const uint32_t key = lds_key<S_WORDS, 1>(lb);
#pragma unroll
      for (int f = 0; f < S_WORDS; f += 2) {
        const uint64_t p0 = lp.word(0, f, lo, k), p1 = lp.word(0, f + 1, lo, k);
        const uint64_t v = (key & 1u) ? (p0 << 32 | p1) : (p1 << 32 | p0);
        if (v) lds_or<uint64_t>(reinterpret_cast<uint64_t*>(lds + lb * S_WORDS + ((f ^ key) & ~1u)), v);
      }
    } else {
#pragma unroll
      for (int f = 0; f < S_WORDS; ++f) {
        const W pat = lp.word(0, f, lo, k);
        if (pat) lds_or<W>(&lds[lds_word<S_WORDS, sizeof(W) / 4>(lb, static_cast<uint32_t>(f))], pat);
      }
    }
  }
};

// Z = -1: the classic filter (Sec. II-A-1) seen as blocks of one 32-bit
// word; its records are (word << 32 | bit), one per pattern bit, so the
// rule sets a single bit.
template <typename W, int S_WORDS, int K>
struct BlockRule<W, S_WORDS, K, -1> {
  static_assert(sizeof(W) == 4 && S_WORDS == 1, "classic records address 32-bit words");
  __device__ __forceinline__ BlockRule() {}
  __device__ __forceinline__ void add_global(W* words, uint32_t blk, uint32_t bit, uint32_t) const {
    __hip_atomic_fetch_or(words + blk, W(1) << bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void add_lds(W* lds, uint32_t lb, uint32_t bit, uint32_t) const {
    lds_or<W>(&lds[lb], W(1) << bit);
  }
};

// Words and local block of a record's global block (direct fallback).
template <typename W>
__device__ __forceinline__ W* record_target(const PartArgs& a, uint32_t gblock, uint32_t& local) {
  if (a.nfilters == 1) {
    local = gblock;
    return static_cast<W*>(a.words);
  }
  const PartFilter& f = a.filters[a.chunk_owner[gblock >> a.chunk_shift]];
  local = static_cast<uint32_t>(gblock - f.block_base);
  return static_cast<W*>(f.words);
}

// Exclusive prefix sums of the record counts of n <= kMaxSlices slices, each
// clamped to cap, into pre[0..n] (pre[n] is the total): the workgroup loads
// the counts into LDS, then one wave scans them in place (a serial run per
// lane, then across lanes).  Ends with a workgroup barrier.
__device__ __forceinline__ void slice_prefix(const unsigned long long* counts, uint32_t n, uint64_t cap,
                                             uint32_t* pre) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
    pre[i] = static_cast<uint32_t>(counts[i] < cap ? counts[i] : cap);
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t per = (n + 63) / 64;
    const uint32_t b = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t i = b; i < b + per && i < n; ++i) sum += pre[i];
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(incl, off, 64);
      if (threadIdx.x >= static_cast<unsigned>(off)) incl += v;
    }
    uint32_t run = incl - sum;
    for (uint32_t i = b; i < b + per && i < n; ++i) {
      const uint32_t v = pre[i];
      pre[i] = run;
      run += v;
    }
    if (threadIdx.x == 63) pre[n] = incl;
  }
  __syncthreads();
}

// Where positions first + tid + j * stride (j < N) of a sliced reader, all
// below pre[n], are stored: position p of slice i (pre[i] <= p < pre[i+1])
// is record p - pre[i] of slice i, i.e. record p + delta of the reader's
// slices laid end to end at `cap` records each, with delta = i * cap -
// pre[i] (at least 0, as each slice holds at most cap records).  The walk
// is uniform over the workgroup: it starts at the slice i0 of an earlier
// position (a reader's positions only increase), moves i0 to the slice of
// `first` and visits each slice up to that of `last` once, so a reader
// visits every slice a bounded number of times over all its steps.
template <int N>
__device__ __forceinline__ void slice_walk(const uint32_t* pre, uint32_t& i0, uint32_t first, uint32_t last,
                                           uint32_t stride, uint32_t cap, uint32_t (&delta)[N]) {
  while (pre[i0 + 1] <= first) ++i0;
  const uint32_t d0 = i0 * cap - pre[i0];
#pragma unroll
  for (int j = 0; j < N; ++j) delta[j] = d0;
  uint32_t i = i0;
  while (pre[i + 1] <= last) {
    ++i;
    const uint32_t b = pre[i];
    const uint32_t d = i * cap - b;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (first + threadIdx.x + j * stride >= b) delta[j] = d;
    }
  }
  i0 = i;
}

// One LDS-staged scatter step.  The records r[] of this thread that take
// part (valid_of(j); record j sits at position tid + j * THREADS) with
// digits dg[] are grouped by digit; *ntotal (LDS) receives their number
// over the workgroup.
// For every digit d with records, claim(d, cnt, gbase[d], room[d]) reserves
// a run of cnt records in digit d's destination: the run starts at record
// gbase[d] of the destination, where store(i, v) puts record v at index i,
// and its first room[d] <= cnt records fit; the thread that reads one of the
// others in the store loop hands it to `overflow`.  The per-digit figures
// live in LDS so that the store loop reads nothing else.
// cnt holds this step's digit counts and is zero on entry; the step zeroes
// cnt_next for the next one, so the counts need no reset of their own.
// after_claims() runs once the claims are done: a caller loads the next
// step's records there.  Every lane stores PER records per step, the slots
// of no record going to spare + lane, so the stores of a step are a fixed
// number and a caller can wait for loads it issued before them with a
// vmcnt that leaves the stores in flight.
template <int THREADS, typename ValidOf, typename Store, typename DigitOf, typename Claim, typename Overflow,
          typename AfterClaims>
__device__ __forceinline__ void scatter_step_masked(
    const uint64_t (&r)[kPartStep / THREADS], const uint32_t (&dg)[kPartStep / THREADS], ValidOf valid_of,
    uint32_t ndigits, uint64_t* stage, uint32_t* cnt, uint32_t* cnt_next, uint32_t* start, uint64_t* gbase,
    uint32_t* room, uint32_t* ntotal, uint64_t spare, Store store, DigitOf digit_of, Claim claim,
    Overflow overflow, AfterClaims after_claims) {
  constexpr int PER = kPartStep / THREADS;
  uint32_t rank[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (valid_of(j)) rank[j] = atomicAdd(&cnt[dg[j]], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < ndigits; d += THREADS)
    if (cnt[d]) claim(d, cnt[d], gbase[d], room[d]);
  // exclusive scan of cnt into start (one wave: a serial slice per lane,
  // then across lanes)
  if (threadIdx.x < 64) {
    const uint32_t per = (ndigits + 63) / 64;
    const uint32_t b = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t d = b; d < b + per && d < ndigits; ++d) sum += cnt[d];
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(incl, off, 64);
      if (threadIdx.x >= static_cast<unsigned>(off)) incl += v;
    }
    uint32_t run = incl - sum;
    for (uint32_t d = b; d < b + per && d < ndigits; ++d) {
      start[d] = run;
      run += cnt[d];
    }
    if (threadIdx.x == 63) *ntotal = incl;
  }
  __syncthreads();
  after_claims();
  const uint32_t total = *ntotal;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (valid_of(j)) stage[start[dg[j]] + rank[j]] = r[j];
  }
  for (uint32_t d = threadIdx.x; d < ndigits; d += THREADS) cnt_next[d] = 0;
  __syncthreads();
  const uint64_t lane_spare = spare + (threadIdx.x & 63u);
#pragma unroll
  for (int j = 0; j < PER; ++j) {  // total <= kPartStep
    const uint32_t p = threadIdx.x + j * THREADS;
    const bool in = p < total;
    const uint64_t v = stage[p];  // stale past total: not used then
    const uint32_t d = in ? digit_of(v) : 0u;
    const uint32_t q = p - start[d];
    const bool fits = in && q < room[d];
    if (in && !fits) overflow(v);  // past its destination's capacity: applied directly
    store(fits ? gbase[d] + q : lane_spare, v);
  }
}

// The common case: the first `valid` positions p = tid + j * THREADS.
template <int THREADS, typename Store, typename DigitOf, typename Claim, typename Overflow, typename AfterClaims>
__device__ __forceinline__ void scatter_step(const uint64_t (&r)[kPartStep / THREADS],
                                             const uint32_t (&dg)[kPartStep / THREADS], uint32_t valid,
                                             uint32_t ndigits, uint64_t* stage, uint32_t* cnt, uint32_t* cnt_next,
                                             uint32_t* start, uint64_t* gbase, uint32_t* room, uint32_t* ntotal,
                                             uint64_t spare, Store store, DigitOf digit_of, Claim claim,
                                             Overflow overflow, AfterClaims after_claims) {
  scatter_step_masked<THREADS>(
      r, dg, [valid](int j) { return threadIdx.x + j * THREADS < valid; }, ndigits, stage, cnt, cnt_next, start,
      gbase, room, ntotal, spare, store, digit_of, claim, overflow, after_claims);
}

// s_waitcnt operands (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8) that wait until at most N vector memory operations
// are outstanding and leave the other counters alone.
constexpr int wait_vmcnt(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// A run of c records at offset b of a destination of cap records: how many fit.
__device__ __forceinline__ uint32_t run_room(uint64_t b, uint32_t c, uint64_t cap) {
  return b >= cap ? 0u : (cap - b < c ? static_cast<uint32_t>(cap - b) : c);
}

// LDS scratch of one scatter pass over at most D digits.
template <int D>
struct ScatterLds {
  uint64_t stage[kPartStep];
  uint64_t gbase[D];
  uint32_t cnt[2][D];  // digit counts of even and odd steps
  uint32_t start[D];
  uint32_t room[D];
  uint32_t fill[D];  // sliced mode: records written to this workgroup's slice
  uint32_t total;    // records of the current step
};

// Destination of the first pass's digit d: slice (d, this workgroup) in
// sliced mode, else the shared bucket d (reserved by atomic add).
template <int D, int THREADS>
struct Pass1Dest {
  const PartArgs& a;
  ScatterLds<D>& l;
  __device__ __forceinline__ void claim(uint32_t d, uint32_t c, uint64_t& gb, uint32_t& rm) const {
    if (a.cs1) {
      const uint32_t b = l.fill[d];
      l.fill[d] = b + c;
      gb = (static_cast<uint64_t>(d) * a.g1 + blockIdx.x) * a.cs1 + b;
      rm = run_room(b, c, a.cs1);
    } else {
      const uint64_t b = atomicAdd(&a.fill1[d], static_cast<unsigned long long>(c));
      gb = bucket1_base(a, d) + b;
      rm = run_room(b, c, bucket1_cap(a, d));
    }
  }
  // sliced mode: publish the record count of every slice of this workgroup
  __device__ __forceinline__ void publish() const {
    if (!a.cs1) return;
    for (uint32_t d = threadIdx.x; d < a.f1; d += THREADS)
      a.fill1[static_cast<uint64_t>(d) * a.g1 + blockIdx.x] = l.fill[d] < a.cs1 ? l.fill[d] : a.cs1;
  }
};

// First pass: hash keys and group the records by high digit.  MULTI: the
// workgroup's keys are one work item of a multi-filter plan, a key range of
// one filter, whose fields are read once before the key loop (per-key
// lookups of the filter inside the loop would make the compiler wait for
// every outstanding load, the prefetched keys included, before hashing).
// CHUNK: a filter of at most kChunkDigits chunks, whose digit is the chunk
// itself: the pass writes the chunk buckets of the apply step directly
// (6-byte records, runs claimed in the shared buckets), and there is no
// second pass.
template <typename W, int S_WORDS, int K, int Z, bool MULTI, bool CHUNK = false>
__device__ __forceinline__ void scatter1_loop(const PartArgs& a, ScatterLds<kMaxDigits>& l) {
  constexpr int kPer1 = kPartStep / kScatter1Threads;
  const BlockRule<W, S_WORDS, K, Z> rule;
  const Pass1Dest<kMaxDigits, kScatter1Threads> dst{a, l};
  const uint32_t shift = a.chunk_shift + a.low_bits;
  const uint32_t local_mask = (1u << a.chunk_shift) - 1;
  uint64_t begin, end, hinit = a.hash_init, base = 0;
  uint32_t nb_lo = a.nb_lo, nb_hi = a.nb_hi_mask;
  if constexpr (MULTI) {
    const PartRange w = a.work1[blockIdx.x];
    const PartFilter& f = a.filters[w.filter];
    begin = w.begin;
    end = w.end;
    hinit = f.hash_init;
    nb_lo = f.nb_lo;
    nb_hi = f.nb_hi_mask;
    base = f.block_base;
  } else {
    begin = static_cast<uint64_t>(blockIdx.x) * a.range1;
    end = begin + a.range1 < a.n ? begin + a.range1 : a.n;
  }
  // The keys of the next step are loaded while this step hashes and sorts
  // (workgroup barriers do not wait for global loads), so their latency is
  // paid once per workgroup rather than once per step.  With chunk buckets
  // they are loaded once the step's claims are done: a claim is then a
  // returning atomic, whose wait would take them too.
  uint64_t next[kPer1];
  auto load_keys = [&](uint64_t s0) {
    const uint64_t v0 = end - s0 < kPartStep ? end - s0 : kPartStep;
#pragma unroll
    for (int j = 0; j < kPer1; ++j) {
      const uint32_t p = threadIdx.x + j * kScatter1Threads;
      next[j] = p < v0 ? __builtin_nontemporal_load(a.keys + s0 + p) : 0;
    }
  };
  if (begin < end) load_keys(begin);
  // the first keys are waited for here, so that at the top of every step
  // the outstanding operations are those of the previous step
  __builtin_amdgcn_s_waitcnt(wait_vmcnt(0));
  uint32_t par = 0;  // which digit-count buffer this step uses
  for (uint64_t s = begin; s < end; s += kPartStep, par ^= 1u) {
    // this step's keys were loaded before the previous step's record stores
    // (one per record, two with chunk buckets): wait for them only
    __builtin_amdgcn_s_waitcnt(wait_vmcnt(CHUNK ? 2 * kPer1 : kPer1));
    const uint32_t valid = static_cast<uint32_t>(end - s < kPartStep ? end - s : kPartStep);
    uint64_t key[kPer1];
#pragma unroll
    for (int j = 0; j < kPer1; ++j) key[j] = next[j];
    const uint64_t s_next = s + kPartStep;
    if constexpr (!CHUNK) {
      if (s_next < end) load_keys(s_next);
    }
    uint64_t r[kPer1];
    uint32_t dg[kPer1];
#pragma unroll
    for (int j = 0; j < kPer1; ++j) {
      const uint64_t h = xxh64_u64(key[j], hinit);
      const uint32_t blk = static_cast<uint32_t>(base + block_of(h, nb_lo, nb_hi));
      r[j] = (static_cast<uint64_t>(blk) << 32) | static_cast<uint32_t>(h);
      dg[j] = blk >> shift;
    }
    auto overflow = [&](uint64_t v) {
      uint32_t local;
      W* w = record_target<W>(a, rec_block(v), local);
      rule.add_global(w, local, rec_lo(v), a.k);
    };
    auto digit_of = [shift](uint64_t v) { return rec_block(v) >> shift; };
    if constexpr (CHUNK) {
      scatter_step<kScatter1Threads>(
          r, dg, valid, a.f1, l.stage, l.cnt[par], l.cnt[par ^ 1], l.start, l.gbase, l.room, &l.total,
          a.spare2,
          [&a, local_mask](uint64_t i, uint64_t v) {
            a.buf2[i] = rec_lo(v);
            a.blk2[i] = static_cast<uint16_t>(rec_block(v) & local_mask);
          },
          digit_of,
          [&a](uint32_t d, uint32_t c, uint64_t& gb, uint32_t& rm) {
            const uint64_t b = atomicAdd(&a.fill2[d], static_cast<unsigned long long>(c));
            gb = bucket2_base(a, d) + b;
            rm = run_room(b, c, bucket2_cap(a, d));
          },
          overflow,
          [&] {
            if (s_next < end) load_keys(s_next);
          });
    } else {
      scatter_step<kScatter1Threads>(
          r, dg, valid, a.f1, l.stage, l.cnt[par], l.cnt[par ^ 1], l.start, l.gbase, l.room, &l.total,
          a.spare1, [&a](uint64_t i, uint64_t v) { a.buf1[i] = v; }, digit_of,
          [&dst](uint32_t d, uint32_t c, uint64_t& gb, uint32_t& rm) { dst.claim(d, c, gb, rm); }, overflow,
          [] {});
    }
  }
  if constexpr (!CHUNK) dst.publish();
}

// MULTI: the kernel of multi-filter plans (one work item per workgroup);
// CHUNK: the one-pass form for filters of at most kChunkDigits chunks.
template <typename W, int S_WORDS, int K, int Z = 0, bool MULTI = false, bool CHUNK = false>
__global__ __launch_bounds__(kScatter1Threads) void part_scatter1_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) ScatterLds<kMaxDigits> l;
  for (uint32_t d = threadIdx.x; d < a.f1; d += kScatter1Threads) {
    l.cnt[0][d] = 0;
    l.cnt[1][d] = 0;
    l.fill[d] = 0;
  }
  __syncthreads();
  scatter1_loop<W, S_WORDS, K, Z, MULTI, CHUNK>(a, l);
}

// First pass of the classic filter: each key gives K records, one per
// position p (word p / 32, bit p mod 32); a thread hashes kPer / K keys
// per step.  a.n and a.range1 count keys.
template <int K, bool POW2>
__global__ __launch_bounds__(kClassicThreads) void part_scatter1_classic_kernel(PartArgs a) {
  constexpr int kPer = kPartStep / kClassicThreads;  // records per thread per step
  constexpr int kKeys = kPer / K;                    // keys per thread per step
  constexpr int kRecs = kKeys * K;                   // records of them
  static_assert(kKeys >= 1, "at most kPer positions per key");
  __shared__ __attribute__((aligned(16))) ScatterLds<kMaxDigits> l;
  for (uint32_t d = threadIdx.x; d < a.f1; d += kClassicThreads) {
    l.cnt[0][d] = 0;
    l.cnt[1][d] = 0;
    l.fill[d] = 0;
  }
  __syncthreads();
  const BlockRule<uint32_t, 1, K, -1> rule;
  const Pass1Dest<kMaxDigits, kClassicThreads> dst{a, l};
  const uint32_t shift = a.chunk_shift + a.low_bits;
  constexpr uint64_t kStepKeys = static_cast<uint64_t>(kClassicThreads) * kKeys;
  const uint64_t begin = static_cast<uint64_t>(blockIdx.x) * a.range1;
  const uint64_t end = begin + a.range1 < a.n ? begin + a.range1 : a.n;
  uint32_t par = 0;  // which digit-count buffer this step uses
  for (uint64_t s = begin; s < end; s += kStepKeys, par ^= 1u) {
    const uint32_t vkeys = static_cast<uint32_t>(end - s < kStepKeys ? end - s : kStepKeys);
    bool ok[kKeys];
    uint64_t r[kPer];
    uint32_t dg[kPer];
#pragma unroll
    for (int u = 0; u < kKeys; ++u) {
      const uint32_t idx = threadIdx.x + u * kClassicThreads;
      ok[u] = idx < vkeys;
      const uint64_t key = ok[u] ? a.keys[s + idx] : 0;
      const uint64_t h = xxh64_u64(key, a.hash_init);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint64_t p = classic_position<POW2>(h, kSalts64.a[j], a.num_bits, a.bit_shift);
        const uint32_t word = static_cast<uint32_t>(p >> 5);
        r[u * K + j] = (static_cast<uint64_t>(word) << 32) | (static_cast<uint32_t>(p) & 31u);
        dg[u * K + j] = word >> shift;
      }
    }
#pragma unroll
    for (int j = kRecs; j < kPer; ++j) {
      r[j] = 0;
      dg[j] = 0;
    }
    scatter_step_masked<kClassicThreads>(
        r, dg, [&](int j) { return j < kRecs && ok[j / K]; }, a.f1, l.stage, l.cnt[par], l.cnt[par ^ 1],
        l.start, l.gbase, l.room, &l.total, a.spare1, [&a](uint64_t i, uint64_t v) { a.buf1[i] = v; },
        [shift](uint64_t v) { return rec_block(v) >> shift; },
        [&dst](uint32_t d, uint32_t c, uint64_t& gb, uint32_t& rm) { dst.claim(d, c, gb, rm); },
        [&](uint64_t v) {
          rule.add_global(static_cast<uint32_t*>(a.words), rec_block(v), rec_lo(v), 0);
        },
        [] {});
  }
  dst.publish();
}

// Second pass: workgroup (d1, qi) groups the qi-th share of high-digit
// bucket d1 by chunk.  With sliced high-digit buckets its share is the
// slices of pass-1 workgroups [g1 * qi / q, g1 * (qi + 1) / q), read as one
// sequence.
template <typename W, int S_WORDS, int K, int Z = 0>
__global__ __launch_bounds__(kScatter2Threads) void part_scatter2_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) ScatterLds<kMaxDigits2> l;
  __shared__ uint32_t pre[kMaxSlices + 1];
  for (uint32_t d = threadIdx.x; d < a.f2; d += kScatter2Threads) {
    l.cnt[0][d] = 0;
    l.cnt[1][d] = 0;
    l.fill[d] = 0;
  }
  __syncthreads();
  constexpr int kPer2 = kPartStep / kScatter2Threads;
  const BlockRule<W, S_WORDS, K, Z> rule;
  const bool sliced = a.cs1 != 0;  // reads pass-1 slices
  uint32_t d1, qi, nq;
  if (a.work2) {
    if (blockIdx.x >= a.nwork2) return;
    const PartWork w = a.work2[blockIdx.x];
    d1 = w.bucket;
    qi = w.split;
    nq = w.nsplit;
  } else {
    d1 = blockIdx.x / a.q;
    qi = blockIdx.x % a.q;
    nq = a.q;
  }
  uint64_t begin, end;
  const uint64_t* src;
  uint32_t w0 = 0, nsl = 0;
  if (sliced) {
    w0 = static_cast<uint32_t>(static_cast<uint64_t>(a.g1) * qi / nq);
    nsl = static_cast<uint32_t>(static_cast<uint64_t>(a.g1) * (qi + 1) / nq) - w0;
    slice_prefix(a.fill1 + static_cast<uint64_t>(d1) * a.g1 + w0, nsl, a.cs1, pre);
    begin = 0;
    end = pre[nsl];
    src = a.buf1 + (static_cast<uint64_t>(d1) * a.g1 + w0) * a.cs1;
  } else {
    const uint64_t cap = bucket1_cap(a, d1);
    const uint64_t filled = a.fill1[d1] < cap ? a.fill1[d1] : cap;
    begin = filled * qi / nq;
    end = filled * (qi + 1) / nq;
    src = a.buf1 + bucket1_base(a, d1);
  }
  const uint32_t cshift = a.chunk_shift, mask = a.f2 - 1, f2 = a.f2;
  const uint32_t local_mask = (1u << a.chunk_shift) - 1;
  const uint64_t cbase = static_cast<uint64_t>(d1) * f2;  // global chunk of digit 0
  uint32_t i0 = 0;  // sliced mode: slice of the last position loaded
  // The records of the next step are loaded once this step's claims are
  // done (a claim is a returning atomic, whose wait would take them too),
  // while the step stages and stores its own.
  uint64_t next[kPer2];
  auto load_records = [&](uint64_t s0) {
    const uint32_t v0 = static_cast<uint32_t>(end - s0 < kPartStep ? end - s0 : kPartStep);
    uint32_t delta[kPer2];
#pragma unroll
    for (int j = 0; j < kPer2; ++j) delta[j] = 0;
    if (sliced)
      slice_walk(pre, i0, static_cast<uint32_t>(s0), static_cast<uint32_t>(s0) + v0 - 1, kScatter2Threads,
                 static_cast<uint32_t>(a.cs1), delta);
#pragma unroll
    for (int j = 0; j < kPer2; ++j) {
      const uint32_t p = threadIdx.x + j * kScatter2Threads;
      next[j] = p < v0 ? src[sliced ? static_cast<uint32_t>(s0) + p + delta[j] : s0 + p] : 0;
    }
  };
  if (begin < end) load_records(begin);
  // the first records are waited for here, so that at the top of every
  // step the outstanding operations are those of the previous step
  __builtin_amdgcn_s_waitcnt(wait_vmcnt(0));
  uint32_t par = 0;  // which digit-count buffer this step uses
  for (uint64_t s = begin; s < end; s += kPartStep, par ^= 1u) {
    // this step's records were loaded before the previous step's stores
    // (two per record: lo32 and block): wait for them only
    __builtin_amdgcn_s_waitcnt(wait_vmcnt(2 * kPer2));
    const uint32_t valid = static_cast<uint32_t>(end - s < kPartStep ? end - s : kPartStep);
    uint64_t r[kPer2];
    uint32_t dg[kPer2];
#pragma unroll
    for (int j = 0; j < kPer2; ++j) {
      r[j] = next[j];
      dg[j] = (rec_block(r[j]) >> cshift) & mask;
    }
    const uint64_t s_next = s + kPartStep;
    scatter_step<kScatter2Threads>(
        r, dg, valid, f2, l.stage, l.cnt[par], l.cnt[par ^ 1], l.start, l.gbase, l.room, &l.total, a.spare2,
        [&a, local_mask](uint64_t i, uint64_t v) {
          a.buf2[i] = rec_lo(v);
          a.blk2[i] = static_cast<uint16_t>(rec_block(v) & local_mask);
        },
        [cshift, mask](uint64_t v) { return (rec_block(v) >> cshift) & mask; },
        [&](uint32_t d, uint32_t c, uint64_t& gb, uint32_t& rm) {
          const uint64_t b = atomicAdd(&a.fill2[cbase + d], static_cast<unsigned long long>(c));
          gb = bucket2_base(a, cbase + d) + b;
          rm = run_room(b, c, bucket2_cap(a, cbase + d));
        },
        [&](uint64_t v) {
          uint32_t local;
          W* w = record_target<W>(a, rec_block(v), local);
          rule.add_global(w, local, rec_lo(v), a.k);
        },
        [&] {
          if (s_next < end) load_records(s_next);
        });
  }
}

// Apply: one workgroup per chunk (grid-stride).  Loads and records are
// handled four at a time per thread so that enough requests are in flight.
// Two workgroups share a CU (their chunk images take 128 KiB of its LDS),
// which takes 8 waves per SIMD: at most 64 VGPRs.
template <typename W, int S_WORDS, int K, int Z = 0>
__global__ __launch_bounds__(kApplyThreads, 8) void part_apply_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t lds_raw[kChunkBytes / 4];
  W* lds = reinterpret_cast<W*>(lds_raw);
  u32x4* lvec = reinterpret_cast<u32x4*>(lds_raw);
  const BlockRule<W, S_WORDS, K, Z> rule;
  const uint32_t blocks_per_chunk = 1u << a.chunk_shift;
  constexpr int kU = 4;
  const uint32_t split = a.apply_split > 1 ? a.apply_split : 1;
  const uint64_t nitems = a.work3 ? a.nwork3 : a.chunks * split;
  for (uint64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    uint64_t c = item;
    uint32_t si = 0, ns = 1;
    if (a.work3) {
      const PartWork w = a.work3[item];
      c = w.bucket;
      si = w.split;
      ns = w.nsplit;
    } else if (split > 1) {
      c = item / split;
      si = static_cast<uint32_t>(item % split);
      ns = split;
    }
    const uint64_t cap = bucket2_cap(a, c);
    const uint64_t filled = a.fill2[c] < cap ? a.fill2[c] : cap;
    const uint64_t rbegin = filled * si / ns;
    const uint64_t count = filled * (si + 1) / ns - rbegin;
    if (count == 0) continue;  // untouched: no traffic at all
    const uint32_t* los = a.buf2 + bucket2_base(a, c) + rbegin;
    const uint16_t* blks = a.blk2 + bucket2_base(a, c) + rbegin;
    W* words = static_cast<W*>(a.words);
    uint64_t num_blocks = a.num_blocks, local_chunk = c;
    if (a.nfilters > 1) {
      const PartFilter& f = a.filters[a.chunk_owner[c]];
      words = static_cast<W*>(f.words);
      num_blocks = f.num_blocks;
      local_chunk = c - f.chunk_base;
    }
    const uint64_t first_block = local_chunk << a.chunk_shift;
    const uint64_t nblk = num_blocks - first_block < blocks_per_chunk ? num_blocks - first_block
                                                                      : blocks_per_chunk;
    const uint32_t nbytes = static_cast<uint32_t>(nblk * S_WORDS * sizeof(W));
    const uint32_t nvec = nbytes / 16;
    const u32x4* gsrc = reinterpret_cast<const u32x4*>(words + first_block * S_WORDS);
    // The sole owner of a chunk starts from its words (copied into the
    // swizzled LDS image); one of several slices of a chunk accumulates its
    // bits only (zeroed image) and merges them with atomic OR.
    constexpr int kPer = static_cast<int>(sizeof(W) / 4);
    const uint32_t tail = nvec * 4 + threadIdx.x;  // < nbytes / 4 for at most 3 threads
    if (ns == 1) {
#pragma unroll 1
      for (int u = 0; u < kVecPerThread; ++u) {
        const uint32_t i = threadIdx.x + u * kApplyThreads;
        if (i < nvec) {
          const u32x4 v = gsrc[i];
          if constexpr (S_WORDS == 1) {
            lvec[i] = v;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) lds_raw[lds_u32<S_WORDS, kPer>(4 * i + q)] = v[q];
          }
        }
      }
      if (tail < nbytes / 4)
        lds_raw[lds_u32<S_WORDS, kPer>(tail)] = reinterpret_cast<const uint32_t*>(gsrc)[tail];
    } else {
#pragma unroll
      for (int u = 0; u < kVecPerThread; ++u) {
        const uint32_t i = threadIdx.x + u * kApplyThreads;
        if (i < nvec) lvec[i] = u32x4{0u, 0u, 0u, 0u};
      }
      if (tail < nbytes / 4) lds_raw[tail] = 0u;
    }
    __syncthreads();
    for (uint64_t i = threadIdx.x; i < count; i += kU * kApplyThreads) {
      uint32_t lo[kU], lb[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint64_t j = i + static_cast<uint64_t>(u) * kApplyThreads;
        lo[u] = j < count ? los[j] : 0;
        lb[u] = j < count ? blks[j] : 0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (i + static_cast<uint64_t>(u) * kApplyThreads < count) rule.add_lds(lds, lb[u], lo[u], a.k);
      }
    }
    __syncthreads();
    u32x4* gdst = reinterpret_cast<u32x4*>(words + first_block * S_WORDS);
    if (ns == 1) {
#pragma unroll
      for (int u = 0; u < kVecPerThread; ++u) {
        const uint32_t i = threadIdx.x + u * kApplyThreads;
        if (i < nvec) {
          if constexpr (S_WORDS == 1) {
            gdst[i] = lvec[i];
          } else {
            gdst[i] = u32x4{lds_raw[lds_u32<S_WORDS, kPer>(4 * i)], lds_raw[lds_u32<S_WORDS, kPer>(4 * i + 1)],
                            lds_raw[lds_u32<S_WORDS, kPer>(4 * i + 2)],
                            lds_raw[lds_u32<S_WORDS, kPer>(4 * i + 3)]};
          }
        }
      }
      if (tail < nbytes / 4)
        reinterpret_cast<uint32_t*>(gdst)[tail] = lds_raw[lds_u32<S_WORDS, kPer>(tail)];
    } else {  // slices of one chunk merge with atomic OR of the words they set
      uint32_t* g32 = reinterpret_cast<uint32_t*>(gdst);
      for (uint32_t i = threadIdx.x; i < nbytes / 4; i += kApplyThreads) {
        const uint32_t v = lds_raw[lds_u32<S_WORDS, kPer>(i)];
        if (v) __hip_atomic_fetch_or(g32 + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

}  // namespace bfhip
