// bf_internal.hpp -- the filter handle, shared by the single-filter and the
// batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/bf.h"

namespace bfhip {
// Stream order of the bf.h calls on one filter (bf_api.hip: ordered_call).
// Every call records the filter's last use on its stream.  A partitioned add
// loads whole chunks into LDS and stores them back, so it first waits for
// every earlier call on every stream, and a direct add (atomic OR into the
// words) waits for the last partitioned add: adds from any streams then
// commute under every strategy, as OR does.  bf_destroy waits for the last
// uses of its filter only.
struct StreamMark {
  hipStream_t stream;
  hipEvent_t event;
};
struct FilterOrder {
  std::mutex mu;
  std::vector<StreamMark> marks;      // last use per stream
  hipEvent_t part_event = nullptr;    // recorded after the last partitioned add
  bool part_pending = false;
};
}  // namespace bfhip

struct bf_filter {
  uint64_t num_blocks;
  uint32_t s;
  uint32_t word_bits;
  uint32_t k;
  int32_t device;
  uint64_t seed;
  uint64_t nbytes;
  void* d_words;
  bf_mapping_t mapping[2];  // as set by the caller; zero fields = default
  uint32_t layout;          // BF_LAYOUT_*
  bool owns_words;          // false for bf_create_in
  uint32_t groups;          // cache-sectorized z, else 0
  uint64_t num_bits;        // nbytes * 8
  bfhip::FilterOrder order;
};

namespace bfhip {
// Partitioned construction (bf_partition.hip).
struct PartArgs;
struct PartLayout {
  uint64_t off_buf1, off_buf2, off_fill, nfill1, nfill, total;
};
struct PartKernels {
  const void* scatter1;
  const void* scatter2;
  const void* apply;
  uint32_t threads1;  // workgroup size of scatter1
};
bool partition_applicable(const bf_filter* f, uint64_t n);
// Workspace bytes a partitioned add of n keys takes from the device pool (0
// if the filter cannot be partitioned).
uint64_t partition_workspace_bytes(const bf_filter* f, uint64_t n);
bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream);
uint32_t part_chunk_shift(uint32_t words_per_block, uint32_t word_bits);
bool part_geometry(uint64_t chunks, uint32_t chunk_shift, uint64_t n, PartArgs& a, PartLayout& L);
// Switches a one-filter geometry to sliced high-digit buckets;
// records_per_key is 1, or k for the classic filter, whose a.n and a.range1
// count keys.
void part_slice(PartArgs& a, PartLayout& L, uint64_t records_per_key);
void part_bind(PartArgs& a, const PartLayout& L, void* base);
PartKernels part_kernels(const bf_filter* f);
bf_status part_launch(const PartArgs& a, const PartLayout& L, const PartKernels& k, hipStream_t stream);
dim3 part_grid1(const PartArgs& a);
dim3 part_grid2(const PartArgs& a);
dim3 part_grid3(const PartArgs& a);
__global__ void part_zero_kernel(unsigned long long* p, uint64_t n);

// Filter allocation shared by every create call (bf_api.hip): fills nbytes,
// device, d_words (zeroed, synchronously).  On error the handle is freed.
bf_status alloc_filter_words(bf_filter* f);

// Whether a bulk add of n keys takes the partitioned strategy (bf_api.hip).
bool use_partitioned(const bf_filter* f, uint64_t n, const bf_mapping_t& m);
// Whether bf_add of n keys on f takes the partitioned construction (the
// classic layout counts k records per key).
bool add_partitions(const bf_filter* f, uint64_t n);

// The classic and cache-sectorized layouts (bf_variants.hip).
bf_mapping_t variant_resolve_mapping(const bf_filter* f, int op);
bf_status variant_validate_mapping(const bf_filter* f, int op, const bf_mapping_t& m);
bf_status variant_launch(bf_filter* f, int op, const uint64_t* keys, uint64_t n, uint8_t* out,
                         hipStream_t stream);
}  // namespace bfhip
