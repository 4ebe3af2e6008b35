// bf_tuned.hpp -- the measured default mapping table as compile-time data.
//
// Rows come from bf_tuned_defaults.inc (written by the autotuner from sweeps
// on gfx950): per (op, word bits, words per block, size class) the mapping
// that measured fastest.  The same table serves the runtime defaults of the
// single-filter launches and the per-size-class mappings compiled into the
// batched kernel.
#pragma once

#include <stdint.h>

namespace bfhip {

struct TunedRow {
  int op, word_bits, s, size_class;
  uint32_t theta, phi, kt, atomic_bits, max_workgroups;
};

inline constexpr TunedRow kTuned[] = {
#define BF_TUNED(op, wb, s, c, t, p, kt, ab, cap) {op, wb, s, c, t, p, kt, ab, cap},
#include "bf_tuned_defaults.inc"
#undef BF_TUNED
};

// Size class of a filter: fits one XCD's 4 MiB L2, the 256 MiB Infinity
// Cache, or only HBM.
constexpr int kNumSizeClasses = 3;
constexpr int size_class_of(uint64_t nbytes) {
  return nbytes <= (4ull << 20) ? 0 : nbytes <= (256ull << 20) ? 1 : 2;
}

struct MapSpec {
  uint32_t theta, phi, kt, atomic_bits, max_workgroups;
  bool found;
};

// Fallback for untuned layouts: one lane per 256-bit slice for lookups, one
// 64-bit atomic per lane for construction.
constexpr MapSpec fallback_map(int op, int word_bits, int s) {
  const uint32_t block_bits = static_cast<uint32_t>(s * word_bits);
  MapSpec m{1, static_cast<uint32_t>(s), 1, 32, 0, false};
  if (op == 1) {
    m.theta = block_bits > 256 ? block_bits / 256 : 1;
    m.phi = static_cast<uint32_t>(s) / m.theta;
    m.kt = 2;
    m.atomic_bits = 0;
  } else {
    m.theta = block_bits >= 64 ? block_bits / 64 : 1;
    if (m.theta > 16) m.theta = 16;
    m.phi = static_cast<uint32_t>(s) / m.theta;
    m.kt = 1;
    m.atomic_bits = (word_bits == 32 && m.phi >= 2) ? 64 : 32;
  }
  return m;
}

constexpr MapSpec tuned_map(int op, int word_bits, int s, int size_class) {
  for (const TunedRow& r : kTuned)
    if (r.op == op && r.word_bits == word_bits && r.s == s && r.size_class == size_class)
      return MapSpec{r.theta, r.phi, r.kt, op == 1 ? 0u : r.atomic_bits, r.max_workgroups, true};
  return fallback_map(op, word_bits, s);
}

}  // namespace bfhip
