// bf_batch.hip -- batched plans (C ABI in include/bf_batch.h): tile list
// construction, XCD-aware ordering, HIP graph of one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/bf_batch.h"
#include "bf_batch_kernels.hpp"
#include "bf_internal.hpp"
#include "bf_registry.hpp"
#include "bf_tuned.hpp"

using namespace bfhip;

namespace {

constexpr int kXcds = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kWgPerCu = 8;       // persistent grid: 8 workgroups (32 waves) per CU

}  // namespace

struct bf_batch {
  int op;
  uint32_t nfilters;
  uint64_t nkeys;
  std::vector<bf_filter*> filters;
  std::vector<uint64_t> offsets;
  const uint64_t* d_keys;
  uint8_t* d_out;
  BatchFilter* d_filters;
  BatchTile* d_tiles;
  uint64_t ntiles;
  uint32_t grid;
  uint32_t tiles_per_class[kNumSizeClasses];
  bf_mapping_t mapping[kNumSizeClasses];
  const void* fn;
  BatchArgs args;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

MapSpec class_map(int op, const bf_filter* f, int cls) {
  if (k_index(f->k) == 0) return MapSpec{1, f->s, 1, 32, 0, true};
  return tuned_map(op, static_cast<int>(f->word_bits), static_cast<int>(f->s), cls);
}

void free_plan(bf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_filters) (void)hipFree(b->d_filters);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  delete b;
}

}  // namespace

extern "C" {

bf_status bf_batch_plan(int op, bf_filter* const* filters, uint32_t nfilters,
                        const uint64_t* d_keys, const uint64_t* h_offsets, uint8_t* d_out,
                        bf_batch** out) {
  if (out == nullptr || filters == nullptr || h_offsets == nullptr || nfilters == 0)
    return BF_EINVAL;
  if (op != BF_OP_ADD && op != BF_OP_CONTAINS) return BF_EINVAL;
  const bf_filter* f0 = filters[0];
  if (f0 == nullptr) return BF_EINVAL;
  for (uint32_t i = 0; i < nfilters; ++i) {
    const bf_filter* f = filters[i];
    if (f == nullptr || f->s != f0->s || f->word_bits != f0->word_bits || f->k != f0->k ||
        f->device != f0->device)
      return BF_EINVAL;
    if (h_offsets[i + 1] < h_offsets[i]) return BF_EINVAL;
  }
  const uint64_t nkeys = h_offsets[nfilters] - h_offsets[0];
  if (nkeys > 0 && (d_keys == nullptr || reinterpret_cast<uintptr_t>(d_keys) % 8 != 0))
    return BF_EINVAL;
  if (op == BF_OP_CONTAINS && nkeys > 0 && d_out == nullptr) return BF_EINVAL;

  ensure_registry();
  const void* fn = registry().batch_fn[batch_index(op, static_cast<int>(f0->word_bits),
                                                   static_cast<int>(f0->s), k_index(f0->k))];
  if (fn == nullptr) return BF_EUNSUPPORTED;

  bf_batch* b = new (std::nothrow) bf_batch{};
  if (b == nullptr) return BF_ENOMEM;
  b->op = op;
  b->nfilters = nfilters;
  b->nkeys = nkeys;
  b->filters.assign(filters, filters + nfilters);
  b->offsets.assign(h_offsets, h_offsets + nfilters + 1);
  b->d_keys = d_keys;
  b->d_out = d_out;
  b->fn = fn;

  // Mapping per size class (identical for all filters of a class).
  for (int c = 0; c < kNumSizeClasses; ++c) {
    const MapSpec m = class_map(op, f0, c);
    bf_mapping_t bm{};
    bm.lanes_per_key = m.theta;
    bm.words_per_lane = m.phi;
    bm.keys_per_lane = m.kt;
    bm.atomic_bits = op == BF_OP_ADD ? m.atomic_bits : 0;
    b->mapping[c] = bm;
  }

  // Filters go to XCD queues by longest-processing-time on their key counts.
  std::vector<uint32_t> order(nfilters);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    return h_offsets[x + 1] - h_offsets[x] > h_offsets[y + 1] - h_offsets[y];
  });
  std::vector<std::vector<BatchTile>> queue(kXcds);
  std::vector<uint64_t> load(kXcds, 0);
  for (uint32_t i : order) {
    const uint64_t n = h_offsets[i + 1] - h_offsets[i];
    if (n == 0) continue;
    const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += n;
    const bf_filter* f = filters[i];
    const int cls = size_class_of(f->nbytes);
    const uint32_t kt = b->mapping[cls].keys_per_lane;
    const uint64_t tile = static_cast<uint64_t>(kBlockThreads) * kt;
    for (uint64_t s = 0; s < n; s += tile) {
      const uint64_t start = h_offsets[i] + s;
      const uint32_t count = static_cast<uint32_t>(std::min<uint64_t>(tile, n - s));
      const bool vec = count == tile && (start % kt) == 0 &&
                       (reinterpret_cast<uintptr_t>(d_keys) % (8u * kt)) == 0 &&
                       (d_out == nullptr || reinterpret_cast<uintptr_t>(d_out) % kt == 0);
      BatchTile t{};
      t.key_start = start;
      t.filter = i;
      t.meta = count | (static_cast<uint32_t>(cls) << kTileClassShift) | (vec ? kTileVecBit : 0u);
      queue[x].push_back(t);
      b->tiles_per_class[cls] += 1;
    }
  }
  // Interleave: slot 8*j + x holds the j-th tile of queue x (empty if none).
  size_t longest = 0;
  for (const auto& q : queue) longest = std::max(longest, q.size());
  std::vector<BatchTile> tiles(longest * kXcds, BatchTile{0, 0, 0});
  for (int x = 0; x < kXcds; ++x)
    for (size_t j = 0; j < queue[x].size(); ++j) tiles[j * kXcds + x] = queue[x][j];
  b->ntiles = tiles.size();

  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, f0->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  uint64_t grid = static_cast<uint64_t>(cus) * kWgPerCu;
  grid = std::min<uint64_t>(grid, std::max<uint64_t>(b->ntiles, kXcds));
  grid = (grid + kXcds - 1) / kXcds * kXcds;  // a multiple of 8 keeps slots on their XCD
  b->grid = static_cast<uint32_t>(grid);

  std::vector<BatchFilter> descs(nfilters);
  for (uint32_t i = 0; i < nfilters; ++i) {
    const bf_filter* f = filters[i];
    descs[i].words = f->d_words;
    descs[i].hash_init = xxh64_u64_init(f->seed);
    descs[i].nb_lo = static_cast<uint32_t>(f->num_blocks);
    descs[i].nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
    descs[i].keys = d_keys;
    descs[i].out = d_out;
    descs[i].reserved = 0;
  }
  const size_t tiles_bytes = std::max<size_t>(1, tiles.size()) * sizeof(BatchTile);
  if (hipMalloc(&b->d_filters, descs.size() * sizeof(BatchFilter)) != hipSuccess ||
      hipMalloc(&b->d_tiles, tiles_bytes) != hipSuccess) {
    (void)hipGetLastError();
    free_plan(b);
    return BF_ENOMEM;
  }
  if (hipMemcpy(b->d_filters, descs.data(), descs.size() * sizeof(BatchFilter),
                hipMemcpyHostToDevice) != hipSuccess ||
      (!tiles.empty() && hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                                   hipMemcpyHostToDevice) != hipSuccess)) {
    free_plan(b);
    return BF_EDEVICE;
  }

  b->args.filters = b->d_filters;
  b->args.tiles = b->d_tiles;
  b->args.ntiles = b->ntiles;
  b->args.k = f0->k;

  // The graph: one kernel node, the persistent launch.
  hipKernelNodeParams p{};
  void* kargs[] = {&b->args};
  p.func = const_cast<void*>(fn);
  p.gridDim = dim3(b->grid);
  p.blockDim = dim3(kBlockThreads);
  p.sharedMemBytes = 0;
  p.kernelParams = kargs;
  p.extra = nullptr;
  hipGraphNode_t node;
  if (hipGraphCreate(&b->graph, 0) != hipSuccess ||
      hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &p) != hipSuccess ||
      hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    free_plan(b);
    return BF_EDEVICE;
  }
  *out = b;
  return BF_OK;
}

bf_status bf_batch_launch(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  if (b->ntiles == 0) return BF_OK;
  return hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? BF_OK
                                                                                  : BF_EDEVICE;
}

bf_status bf_batch_launch_direct(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  if (b->ntiles == 0) return BF_OK;
  void* kargs[] = {&b->args};
  return hipLaunchKernel(b->fn, dim3(b->grid), dim3(kBlockThreads), kargs, 0,
                         static_cast<hipStream_t>(stream)) == hipSuccess
             ? BF_OK
             : BF_EDEVICE;
}

bf_status bf_batch_launch_per_filter(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  for (uint32_t i = 0; i < b->nfilters; ++i) {
    const uint64_t n = b->offsets[i + 1] - b->offsets[i];
    if (n == 0) continue;
    const uint64_t off = b->offsets[i];
    bf_status st = b->op == BF_OP_ADD
                       ? bf_add(b->filters[i], b->d_keys + off, n, stream)
                       : bf_contains(b->filters[i], b->d_keys + off, n, b->d_out + off, stream);
    if (st != BF_OK) return st;
  }
  return BF_OK;
}

bf_status bf_batch_info(const bf_batch* b, bf_batch_info_t* out) {
  if (b == nullptr || out == nullptr) return BF_EINVAL;
  bf_batch_info_t i{};
  i.op = static_cast<uint32_t>(b->op);
  i.nfilters = b->nfilters;
  i.nkeys = b->nkeys;
  i.ntiles = b->ntiles;
  i.grid = b->grid;
  for (int c = 0; c < kNumSizeClasses; ++c) {
    i.tiles_per_class[c] = b->tiles_per_class[c];
    i.mapping[c] = b->mapping[c];
  }
  *out = i;
  return BF_OK;
}

bf_status bf_batch_destroy(bf_batch* b) {
  if (b == nullptr) return BF_OK;
  bf_status st = hipDeviceSynchronize() == hipSuccess ? BF_OK : BF_EDEVICE;
  free_plan(b);
  return st;
}

}  // extern "C"
