// bf_internal.hpp -- the filter handle, shared by the single-filter and the
// batched entry points.
#pragma once

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
};
