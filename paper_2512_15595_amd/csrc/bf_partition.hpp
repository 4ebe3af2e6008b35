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
//   scatter2  records -> chunk buckets;                       [8 in, 8 out]
//   apply     per chunk: LDS load, LDS atomic OR, store;      [8 in + chunk]
// Each scatter step counting-sorts kPartStep records in LDS and reserves
// each digit's run in its bucket with one returning atomic add, so a digit
// leaves the step as one contiguous run.  Bucket capacities cover the
// expected count of uniformly hashed keys plus six standard deviations; a
// record that finds its bucket full (repeated keys can do that) is applied
// at once with direct global atomics instead, so results never depend on
// the capacities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bf_hash.hpp"
#include "bf_kernels.hpp"

namespace bfhip {

constexpr int kPartThreads = 256;
constexpr int kPartPer = 16;                        // records per thread per step
constexpr int kPartStep = kPartThreads * kPartPer;  // records per LDS-staged step
constexpr int kApplyThreads = 1024;                 // apply: 16 waves share one chunk
constexpr int kChunkBytes = 64 * 1024;              // LDS bytes owned per chunk
constexpr int kMaxDigits = 512;                     // digit fan-out limit of one pass

struct PartArgs {
  void* words;
  uint64_t num_blocks;
  uint64_t hash_init;
  uint32_t nb_lo;
  uint32_t nb_hi_mask;
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
  uint64_t* buf1;        // f1 buckets of cap1 records
  unsigned long long* fill1;
  uint64_t cap1;
  uint64_t* buf2;        // chunk buckets of cap2 records
  unsigned long long* fill2;
  uint64_t cap2;
};

__device__ __forceinline__ uint32_t rec_block(uint64_t r) { return static_cast<uint32_t>(r >> 32); }
__device__ __forceinline__ uint32_t rec_lo(uint64_t r) { return static_cast<uint32_t>(r); }

// One LDS-staged scatter step: the valid records r[] (positions p = tid +
// j * kPartThreads < valid) with digits dg[] are grouped by digit and
// written, per digit d, to bucket bucket_of(d) at a reserved offset.
// Records that do not fit their bucket go to `overflow`.
template <typename DigitOf, typename BucketOf, typename Overflow>
__device__ __forceinline__ void scatter_step(const uint64_t (&r)[kPartPer], const uint32_t (&dg)[kPartPer],
                                             uint32_t valid, uint32_t ndigits, uint64_t* stage,
                                             uint32_t* cnt, uint32_t* start, uint64_t* base,
                                             unsigned long long* fill, uint64_t cap, uint64_t* buf,
                                             DigitOf digit_of, BucketOf bucket_of, Overflow overflow) {
  uint32_t rank[kPartPer];
#pragma unroll
  for (int j = 0; j < kPartPer; ++j) {
    const uint32_t p = threadIdx.x + j * kPartThreads;
    if (p < valid) rank[j] = atomicAdd(&cnt[dg[j]], 1u);
  }
  __syncthreads();
  // reserve each digit's run in its bucket
  for (uint32_t d = threadIdx.x; d < ndigits; d += kPartThreads)
    base[d] = cnt[d] ? atomicAdd(&fill[bucket_of(d)], static_cast<unsigned long long>(cnt[d])) : 0;
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
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPartPer; ++j) {
    const uint32_t p = threadIdx.x + j * kPartThreads;
    if (p < valid) stage[start[dg[j]] + rank[j]] = r[j];
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < valid; p += kPartThreads) {
    const uint64_t v = stage[p];
    const uint32_t d = digit_of(v);
    const uint64_t pos = base[d] + (p - start[d]);
    if (pos < cap)
      buf[static_cast<uint64_t>(bucket_of(d)) * cap + pos] = v;
    else
      overflow(v);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < ndigits; d += kPartThreads) cnt[d] = 0;
  __syncthreads();
}

// First pass: hash keys and group the records by high digit.
template <typename W, int S_WORDS, int K>
__global__ __launch_bounds__(kPartThreads) void part_scatter1_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) uint64_t stage[kPartStep];
  __shared__ uint32_t cnt[kMaxDigits];
  __shared__ uint32_t start[kMaxDigits];
  __shared__ uint64_t base[kMaxDigits];
  for (uint32_t d = threadIdx.x; d < a.f1; d += kPartThreads) cnt[d] = 0;
  __syncthreads();
  const LanePatterns<W, S_WORDS, K, 1, S_WORDS> lp(0);
  W* words = static_cast<W*>(a.words);
  const uint32_t shift = a.chunk_shift + a.low_bits;
  const uint64_t begin = static_cast<uint64_t>(blockIdx.x) * a.range1;
  const uint64_t end = begin + a.range1 < a.n ? begin + a.range1 : a.n;
  for (uint64_t s = begin; s < end; s += kPartStep) {
    const uint32_t valid = static_cast<uint32_t>(end - s < kPartStep ? end - s : kPartStep);
    uint64_t key[kPartPer];
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
      const uint32_t p = threadIdx.x + j * kPartThreads;
      key[j] = p < valid ? a.keys[s + p] : 0;
    }
    uint64_t r[kPartPer];
    uint32_t dg[kPartPer];
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
      const uint64_t h = xxh64_u64(key[j], a.hash_init);
      const uint32_t blk = block_of(h, a.nb_lo, a.nb_hi_mask);
      r[j] = (static_cast<uint64_t>(blk) << 32) | static_cast<uint32_t>(h);
      dg[j] = blk >> shift;
    }
    scatter_step(
        r, dg, valid, a.f1, stage, cnt, start, base, a.fill1, a.cap1, a.buf1,
        [shift](uint64_t v) { return rec_block(v) >> shift; }, [](uint32_t d) { return d; },
        [&](uint64_t v) {
          add_block<W, S_WORDS, K, 1, S_WORDS, false>(words, rec_block(v), rec_lo(v), lp, a.k);
        });
  }
}

// Second pass: workgroup (d1, qi) groups the qi-th slice of high-digit
// bucket d1 by chunk.
template <typename W, int S_WORDS, int K>
__global__ __launch_bounds__(kPartThreads) void part_scatter2_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) uint64_t stage[kPartStep];
  __shared__ uint32_t cnt[kMaxDigits];
  __shared__ uint32_t start[kMaxDigits];
  __shared__ uint64_t base[kMaxDigits];
  for (uint32_t d = threadIdx.x; d < a.f2; d += kPartThreads) cnt[d] = 0;
  __syncthreads();
  const LanePatterns<W, S_WORDS, K, 1, S_WORDS> lp(0);
  W* words = static_cast<W*>(a.words);
  const uint32_t d1 = blockIdx.x / a.q, qi = blockIdx.x % a.q;
  const uint64_t filled = a.fill1[d1] < a.cap1 ? a.fill1[d1] : a.cap1;
  const uint64_t begin = filled * qi / a.q, end = filled * (qi + 1) / a.q;
  const uint64_t* src = a.buf1 + static_cast<uint64_t>(d1) * a.cap1;
  const uint32_t cshift = a.chunk_shift, mask = a.f2 - 1, f2 = a.f2;
  for (uint64_t s = begin; s < end; s += kPartStep) {
    const uint32_t valid = static_cast<uint32_t>(end - s < kPartStep ? end - s : kPartStep);
    uint64_t r[kPartPer];
    uint32_t dg[kPartPer];
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
      const uint32_t p = threadIdx.x + j * kPartThreads;
      r[j] = p < valid ? src[s + p] : 0;
      dg[j] = (rec_block(r[j]) >> cshift) & mask;
    }
    scatter_step(
        r, dg, valid, f2, stage, cnt, start, base, a.fill2, a.cap2, a.buf2,
        [cshift, mask](uint64_t v) { return (rec_block(v) >> cshift) & mask; },
        [d1, f2](uint32_t d) { return d1 * f2 + d; },
        [&](uint64_t v) {
          add_block<W, S_WORDS, K, 1, S_WORDS, false>(words, rec_block(v), rec_lo(v), lp, a.k);
        });
  }
}

template <typename W>
__device__ __forceinline__ void lds_or(W* p, W v) {
  if constexpr (sizeof(W) == 8)
    atomicOr(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
  else
    atomicOr(reinterpret_cast<unsigned int*>(p), static_cast<unsigned int>(v));
}

// Apply: one workgroup per chunk (grid-stride).  Loads and records are
// handled four at a time per thread so that enough requests are in flight.
template <typename W, int S_WORDS, int K>
__global__ __launch_bounds__(kApplyThreads) void part_apply_kernel(PartArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t lds_raw[kChunkBytes / 4];
  W* lds = reinterpret_cast<W*>(lds_raw);
  u32x4* lvec = reinterpret_cast<u32x4*>(lds_raw);
  W* words = static_cast<W*>(a.words);
  const LanePatterns<W, S_WORDS, K, 1, S_WORDS> lp(0);
  const uint32_t blocks_per_chunk = 1u << a.chunk_shift;
  const uint32_t local_mask = blocks_per_chunk - 1;
  constexpr int kU = 4;
  for (uint64_t c = blockIdx.x; c < a.chunks; c += gridDim.x) {
    const uint64_t count = a.fill2[c] < a.cap2 ? a.fill2[c] : a.cap2;
    if (count == 0) continue;  // untouched chunk: no traffic at all
    const uint64_t* recs = a.buf2 + c * a.cap2;
    const uint64_t first_block = c << a.chunk_shift;
    const uint64_t nblk = a.num_blocks - first_block < blocks_per_chunk ? a.num_blocks - first_block
                                                                        : blocks_per_chunk;
    const uint32_t nbytes = static_cast<uint32_t>(nblk * S_WORDS * sizeof(W));
    const uint32_t nvec = nbytes / 16;
    const u32x4* gsrc = reinterpret_cast<const u32x4*>(words + first_block * S_WORDS);
    for (uint32_t i = threadIdx.x; i < nvec; i += kU * kApplyThreads) {
      u32x4 v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i + u * kApplyThreads < nvec) v[u] = gsrc[i + u * kApplyThreads];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i + u * kApplyThreads < nvec) lvec[i + u * kApplyThreads] = v[u];
    }
    for (uint32_t i = nvec * 4 + threadIdx.x; i < nbytes / 4; i += kApplyThreads)
      lds_raw[i] = reinterpret_cast<const uint32_t*>(gsrc)[i];
    __syncthreads();
    for (uint64_t i = threadIdx.x; i < count; i += kU * kApplyThreads) {
      uint64_t r[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint64_t j = i + static_cast<uint64_t>(u) * kApplyThreads;
        r[u] = j < count ? recs[j] : 0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (i + static_cast<uint64_t>(u) * kApplyThreads < count) {
          const uint32_t lb = rec_block(r[u]) & local_mask;
          const uint32_t lo = rec_lo(r[u]);
#pragma unroll
          for (int f = 0; f < S_WORDS; ++f) {
            const W pat = lp.word(0, f, lo, a.k);
            if (pat) lds_or<W>(&lds[lb * S_WORDS + f], pat);
          }
        }
      }
    }
    __syncthreads();
    u32x4* gdst = reinterpret_cast<u32x4*>(words + first_block * S_WORDS);
    for (uint32_t i = threadIdx.x; i < nvec; i += kApplyThreads) gdst[i] = lvec[i];
    for (uint32_t i = nvec * 4 + threadIdx.x; i < nbytes / 4; i += kApplyThreads)
      reinterpret_cast<uint32_t*>(gdst)[i] = lds_raw[i];
    __syncthreads();
  }
}

}  // namespace bfhip
