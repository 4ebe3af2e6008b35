// bf_internal.hpp -- the filter handle, shared by the single-filter and the
// batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bf.h"

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
  void* scratch;            // partitioned-construction workspace (grow-only)
  uint64_t scratch_bytes;
};

namespace bfhip {
// Partitioned construction (bf_partition.hip).
bool partition_applicable(const bf_filter* f, uint64_t n);
bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream);
}  // namespace bfhip
