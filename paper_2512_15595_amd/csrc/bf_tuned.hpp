// bf_tuned.hpp -- the measured default mapping table and the measured
// construction-strategy crossover, as compile-time data.
//
// Rows come from bf_tuned_defaults.inc (written by the autotuner from sweeps
// on gfx950).  The paper's point (Sec. IV-A, V-B to V-D) is that the best
// execution mapping depends on the operation, the block size, the memory
// regime and the GPU; here it is measured per
//   (op, word bits, words per block, size class, k, batch-size class)
// and holds lanes per key, words per lane, keys per lane, the atomic width
// of add, the grid cap and the workgroup size.  The same table serves the
// single-filter launches, the per-size-class mappings compiled into the
// batched kernel and the server's request launches.
//
// The crossover rows give, per layout, the measured cost model of the two
// constructions of an add of n keys into a filter of `bytes`:
//   partitioned ~ a + b * MiB(bytes) + c * n,   direct ~ d[size class] * n,
// so the partitioned one is taken when n * (d - c) > a + b * MiB.
#pragma once

#include <stdint.h>

namespace bfhip {

struct TunedRow {
  int op, word_bits, s, size_class, k, n_class;
  uint32_t theta, phi, kt, atomic_bits, max_workgroups, wg_threads;
};

// Per layout: kind (0 sectorized, 1 classic, 2 cache-sectorized), word
// bits, words per block, groups (cache-sectorized), k (classic: the k
// measured; others 0 = any).  a in microseconds, b in microseconds per MiB
// of filter, c and d in picoseconds per key.
struct CrossoverRow {
  int kind, word_bits, s, groups, k;
  double a_us, b_us_per_mib, c_ps, d_ps[3];
};

inline constexpr TunedRow kTuned[] = {
#define BF_TUNED(op, wb, s, c, k, nc, t, p, kt, ab, cap, wg) \
  {op, wb, s, c, k, nc, t, p, kt, ab, cap, wg},
#define BF_CROSSOVER(kind, wb, s, z, k, a, b, c, d0, d1, d2)
#include "bf_tuned_defaults.inc"
#undef BF_CROSSOVER
#undef BF_TUNED
};

inline constexpr CrossoverRow kCrossover[] = {
#define BF_TUNED(op, wb, s, c, k, nc, t, p, kt, ab, cap, wg)
#define BF_CROSSOVER(kind, wb, s, z, k, a, b, c, d0, d1, d2) \
  {kind, wb, s, z, k, a, b, c, {d0, d1, d2}},
#include "bf_tuned_defaults.inc"
#undef BF_CROSSOVER
#undef BF_TUNED
};

// Size class of a filter: fits one XCD's 4 MiB L2, the 256 MiB Infinity
// Cache, or only HBM.
constexpr int kNumSizeClasses = 3;
constexpr int size_class_of(uint64_t nbytes) {
  return nbytes <= (4ull << 20) ? 0 : nbytes <= (256ull << 20) ? 1 : 2;
}

// Batch-size class of a launch: a small batch (at most 2^16 keys, under one
// 256-key tile per CU) is latency bound, a large one throughput bound.
constexpr int kNumBatchClasses = 2;
constexpr uint64_t kSmallBatchKeys = 1ull << 16;
constexpr int n_class_of(uint64_t n) { return n <= kSmallBatchKeys ? 0 : 1; }

struct MapSpec {
  uint32_t theta, phi, kt, atomic_bits, max_workgroups, wg_threads;
  bool found;
};

// Fallback for untuned layouts: one lane per 256-bit slice for lookups, one
// 64-bit atomic per lane for construction, 256-thread workgroups.
constexpr MapSpec fallback_map(int op, int word_bits, int s) {
  const uint32_t block_bits = static_cast<uint32_t>(s * word_bits);
  MapSpec m{1, static_cast<uint32_t>(s), 1, 32, 0, 256, false};
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

// The tuned mapping of (op, word bits, s, size class, k, batch class): among
// the rows of that (op, word bits, s, size class, batch class), the one
// measured at the k nearest to k (by ratio; ties to the larger k).
// A batch class with no rows takes the other class's rows.
constexpr MapSpec tuned_map(int op, int word_bits, int s, int size_class, int k, int n_class) {
  bool have_class = false;
  for (const TunedRow& r : kTuned)
    if (r.op == op && r.word_bits == word_bits && r.s == s && r.size_class == size_class &&
        r.n_class == n_class)
      have_class = true;
  const TunedRow* best = nullptr;
  uint64_t best_ratio = 0;
  for (const TunedRow& r : kTuned) {
    if (r.op != op || r.word_bits != word_bits || r.s != s || r.size_class != size_class ||
        (have_class && r.n_class != n_class))
      continue;
    const uint64_t hi = static_cast<uint64_t>(r.k > k ? r.k : k);
    const uint64_t lo = static_cast<uint64_t>(r.k > k ? k : r.k);
    const uint64_t ratio = lo == 0 ? ~0ull : hi * 4096 / lo;
    if (best == nullptr || ratio < best_ratio || (ratio == best_ratio && r.k > best->k)) {
      best = &r;
      best_ratio = ratio;
    }
  }
  if (best == nullptr) return fallback_map(op, word_bits, s);
  return MapSpec{best->theta,          best->phi,        best->kt, op == 1 ? 0u : best->atomic_bits,
                 best->max_workgroups, best->wg_threads, true};
}

// The measured crossover row of a layout (nullptr: none measured).
inline const CrossoverRow* crossover_row(int kind, int word_bits, int s, int groups, int k) {
  const CrossoverRow* any = nullptr;
  for (const CrossoverRow& r : kCrossover) {
    if (r.kind != kind || r.word_bits != word_bits || r.s != s || r.groups != groups) continue;
    if (r.k == k) return &r;
    if (any == nullptr || r.k == 0) any = &r;
  }
  return any;
}

}  // namespace bfhip
