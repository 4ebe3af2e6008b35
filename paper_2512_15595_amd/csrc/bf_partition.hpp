// bf_partition.hpp -- partitioned construction: bulk add without global
// atomics.
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
// reason, Sec. V-A):
//   hash     keys -> records (block << 32 | lo32), level-1 digit counts per
//            workgroup;                                       [8 B in, 8 out]
//   scan     exclusive scan of the counts (digit-major);
//   scatter1 records grouped by the high digit, LDS-staged so that each
//            digit's run is written contiguously;              [8 in, 8 out]
//   count2   low-digit counts per (high digit, slice);         [8 in]
//   scan     exclusive scan (chunk-major);
//   scatter2 records grouped by chunk;                         [8 in, 8 out]
//   apply    per chunk: LDS load, LDS atomic OR, store.  [8 in + chunk R/W]
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bf_hash.hpp"
#include "bf_kernels.hpp"

namespace bfhip {

constexpr int kPartThreads = 256;
constexpr int kPartStep = kPartThreads * 8;  // records per LDS-staged step
constexpr int kChunkBytes = 64 * 1024;       // LDS bytes owned per chunk
constexpr int kMaxDigits = 512;              // digit fan-out limit of one pass

struct PartGeometry {
  uint64_t n;            // keys
  uint32_t chunk_shift;  // log2(blocks per chunk)
  uint32_t low_bits;     // bits of the low (second-pass) digit
  uint32_t f1;           // high digits (first pass)
  uint32_t f2;           // low digits (second pass) = 1 << low_bits
  uint32_t g1;           // workgroups of the first pass
  uint32_t q;            // workgroups per high digit in the second pass
  uint64_t range1;       // keys per first-pass workgroup (multiple of kPartStep)
  uint64_t chunks;       // total chunks
};

__device__ __forceinline__ uint32_t rec_block(uint64_t r) { return static_cast<uint32_t>(r >> 32); }
__device__ __forceinline__ uint32_t rec_lo(uint64_t r) { return static_cast<uint32_t>(r); }

// ---------------------------------------------------------------------------
// apply: one workgroup per chunk (grid-stride); records of chunk c are
// recs[off2[c * q], off2[(c + 1) * q]).
// ---------------------------------------------------------------------------
template <typename W, int S_WORDS, int K>
__global__ __launch_bounds__(kPartThreads) void part_apply_kernel(W* words, uint64_t num_blocks,
                                                                  const uint64_t* recs,
                                                                  const uint64_t* off2, PartGeometry g,
                                                                  uint32_t k) {
  __shared__ __attribute__((aligned(16))) uint32_t lds_raw[kChunkBytes / 4];
  W* lds = reinterpret_cast<W*>(lds_raw);
  const LanePatterns<W, S_WORDS, K, 1, S_WORDS> lp(0);
  const uint32_t blocks_per_chunk = 1u << g.chunk_shift;
  const uint32_t local_mask = blocks_per_chunk - 1;
  for (uint64_t c = blockIdx.x; c < g.chunks; c += gridDim.x) {
    const uint64_t rb = off2[c * g.q];
    const uint64_t re = off2[(c + 1) * g.q];
    if (rb == re) continue;  // untouched chunk: no traffic at all
    const uint64_t first_block = c << g.chunk_shift;
    const uint64_t nblk = num_blocks - first_block < blocks_per_chunk ? num_blocks - first_block
                                                                      : blocks_per_chunk;
    const uint64_t nbytes = nblk * S_WORDS * sizeof(W);
    const u32x4* gsrc = reinterpret_cast<const u32x4*>(words + first_block * S_WORDS);
    u32x4* lvec = reinterpret_cast<u32x4*>(lds_raw);
    const uint32_t nvec = static_cast<uint32_t>(nbytes / 16);
    for (uint32_t i = threadIdx.x; i < nvec; i += kPartThreads) lvec[i] = gsrc[i];
    for (uint32_t i = nvec * 4 + threadIdx.x; i < nbytes / 4; i += kPartThreads)
      lds_raw[i] = reinterpret_cast<const uint32_t*>(gsrc)[i];
    __syncthreads();
    for (uint64_t i = rb + threadIdx.x; i < re; i += kPartThreads) {
      const uint64_t r = recs[i];
      const uint32_t lb = rec_block(r) & local_mask;
      const uint32_t lo = rec_lo(r);
#pragma unroll
      for (int f = 0; f < S_WORDS; ++f) {
        const W pat = lp.word(0, f, lo, k);
        if (pat) {
          if constexpr (sizeof(W) == 8)
            atomicOr(reinterpret_cast<unsigned long long*>(&lds[lb * S_WORDS + f]),
                     static_cast<unsigned long long>(pat));
          else
            atomicOr(reinterpret_cast<unsigned int*>(&lds[lb * S_WORDS + f]),
                     static_cast<unsigned int>(pat));
        }
      }
    }
    __syncthreads();
    u32x4* gdst = reinterpret_cast<u32x4*>(words + first_block * S_WORDS);
    for (uint32_t i = threadIdx.x; i < nvec; i += kPartThreads) gdst[i] = lvec[i];
    for (uint32_t i = nvec * 4 + threadIdx.x; i < nbytes / 4; i += kPartThreads)
      reinterpret_cast<uint32_t*>(gdst)[i] = lds_raw[i];
    __syncthreads();
  }
}

}  // namespace bfhip
