// bf_batch.hip -- batched plans (C ABI in include/bf_batch.h): tile list
// construction, XCD-aware ordering, HIP graph of one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <mutex>
#include <numeric>
#include <utility>
#include <vector>

#include "../../include/bf_batch.h"
#include "bf_batch_kernels.hpp"
#include "bf_internal.hpp"
#include "bf_partition.hpp"
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
  // partitioned construction over the dense filters of the plan (add only);
  // part_direct[i] marks the filters left to the tiled direct launch
  bool partitioned;
  std::vector<uint8_t> part_direct;
  PartArgs part;
  PartLayout part_layout;
  PartKernels part_k;
  void* part_scratch;
  // device memory from lib_alloc (pooled: released in stream order)
  int device;
  bool pooled_filters, pooled_tiles, pooled_scratch;
  // one event per stream the plan was launched on, recorded after its last
  // launch there: bf_batch_destroy waits for these and nothing else
  std::mutex mark_mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> marks;
  bool unmarked;  // a launch whose event could not be recorded: destroy waits for the device
};

namespace {

// The mapping the batched kernel compiles in for a size class (bf_batch_kernels.hpp:
// batch_map): the tuned rows of large batches at the filters' k.
MapSpec class_map(int op, const bf_filter* f, int cls) {
  if (k_index(f->k) == 0) return MapSpec{1, f->s, 1, 32, 0, kBlockThreads, true};
  return tuned_map(op, static_cast<int>(f->word_bits), static_cast<int>(f->s), cls,
                   static_cast<int>(f->k), 1);
}

void free_plan(bf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  lib_free(b->device, b->d_filters, b->pooled_filters);
  lib_free(b->device, b->d_tiles, b->pooled_tiles);
  lib_free(b->device, b->part_scratch, b->pooled_scratch);
  for (auto& m : b->marks) (void)hipEventDestroy(m.second);
  delete b;
}

// Records that the plan's work was enqueued on `stream` (not for a stream
// being captured: such a launch runs when the caller's graph does, which the
// caller orders against the plan's destruction).
bf_status mark_launch(bf_batch* b, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(b->mark_mu);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone) return BF_OK;
  hipEvent_t ev = nullptr;
  for (auto& m : b->marks)
    if (m.first == stream) ev = m.second;
  if (ev == nullptr && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess)
    b->marks.emplace_back(stream, ev);
  if (ev == nullptr || hipEventRecord(ev, stream) != hipSuccess) {
    (void)hipGetLastError();
    b->unmarked = true;  // the work is enqueued: destroy must still wait for it
    return BF_EDEVICE;
  }
  return BF_OK;
}

// Partitioned construction for an add plan: the filters' blocks are laid
// end to end in one global block space (each filter starting on a chunk
// boundary), so one radix partition groups every key of every filter by
// global chunk.  With the automatic strategy a filter whose keys are too
// few for its size is left to the direct launch (b->part_direct): by the
// layout's measured costs (the crossover rows of bf_tuned.hpp, without the
// fixed cost, which the plan shares), streaming its chunks would cost more
// than its keys' atomics, and its chunks then get neither records nor
// traffic.  Returns BF_OK and sets b->partitioned when taken.
bf_status plan_partitioned(bf_batch* b, bf_filter* const* filters, uint32_t nfilters,
                           const uint64_t* d_keys, const uint64_t* h_offsets) {
  const bf_filter* f0 = filters[0];
  const uint32_t strategy = f0->mapping[BF_OP_ADD].strategy;
  if (strategy == BF_STRATEGY_DIRECT) return BF_OK;
  const bool forced = strategy == BF_STRATEGY_PARTITIONED;
  uint64_t n_dense = 0, dense_chunks = 0;
  const uint32_t shift = part_chunk_shift(f0->s, f0->word_bits);
  const uint64_t bpc = 1ull << shift;
  std::vector<PartFilter> pf(nfilters);
  const CrossoverRow* xr = crossover_of(f0);
  uint64_t chunks = 0;
  for (uint32_t i = 0; i < nfilters; ++i) {
    const bf_filter* f = filters[i];
    pf[i].words = f->d_words;
    pf[i].hash_init = xxh64_u64_init(f->seed);
    pf[i].nb_lo = static_cast<uint32_t>(f->num_blocks);
    pf[i].nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
    pf[i].num_blocks = f->num_blocks;
    pf[i].chunk_base = chunks;
    pf[i].block_base = chunks * bpc;
    pf[i].key_begin = h_offsets[i] - h_offsets[0];
    pf[i].key_end = h_offsets[i + 1] - h_offsets[0];
    const uint64_t ni = pf[i].key_end - pf[i].key_begin;
    const uint64_t nc = (f->num_blocks + bpc - 1) / bpc;
    pf[i].direct = !forced && !dense_enough(xr, f->nbytes, ni, true) ? 1u : 0u;
    if (!pf[i].direct) {
      n_dense += ni;
      dense_chunks += nc;
    }
    chunks += nc;
  }
  const uint64_t n = h_offsets[nfilters] - h_offsets[0];
  if (n == 0 || chunks * bpc > (1ull << 32)) return BF_OK;  // global blocks must fit 32 bits
  if (strategy == BF_STRATEGY_AUTO && !(dense_chunks >= 512 && n_dense >= (1ull << 21))) return BF_OK;
  PartArgs a{};
  PartLayout L{};
  if (!part_geometry(chunks, shift, n, a, L)) return BF_OK;
  PartKernels k = part_kernels(f0);
  k.scatter1 = k.scatter1_multi;  // the first pass takes its key ranges from the work list
  if (k.scatter1 == nullptr || k.scatter2 == nullptr || k.apply == nullptr) return BF_OK;
  // Per-bucket capacities from each chunk's expected load: filter i's keys
  // spread uniformly over its blocks (a chunk holding part of the filter
  // expects that part's share); six standard deviations plus a margin.
  std::vector<double> load(chunks, 0.0);
  for (uint32_t i = 0; i < nfilters; ++i) {
    const double ni = static_cast<double>(pf[i].key_end - pf[i].key_begin);
    if (ni == 0 || pf[i].direct) continue;
    const uint64_t nc = (pf[i].num_blocks + bpc - 1) / bpc;
    for (uint64_t c = 0; c < nc; ++c) {
      const uint64_t blocks = std::min<uint64_t>(bpc, pf[i].num_blocks - c * bpc);
      load[pf[i].chunk_base + c] = ni * static_cast<double>(blocks) / static_cast<double>(pf[i].num_blocks);
    }
  }
  auto cap_of = [](double mean, double margin) {
    if (mean <= 0.0) return uint64_t{0};
    return static_cast<uint64_t>(std::ceil(mean + 6.0 * std::sqrt(mean) + margin));
  };
  std::vector<uint64_t> off1(a.f1 + 1, 0), off2(chunks + 1, 0);
  for (uint64_t c = 0; c < chunks; ++c) off2[c + 1] = off2[c] + cap_of(load[c], 64.0);
  for (uint32_t d = 0; d < a.f1; ++d) {
    double m = 0.0;
    for (uint64_t c = static_cast<uint64_t>(d) * a.f2; c < std::min<uint64_t>(chunks, (d + 1ull) * a.f2); ++c)
      m += load[c];
    off1[d + 1] = off1[d] + cap_of(m, 1024.0);
  }
  // buffers sized by the extents (replacing the uniform layout)
  L.off_buf1 = 0;
  a.spare1 = off1[a.f1];
  a.spare2 = off2[chunks];
  uint64_t off = (8 * (off1[a.f1] + kSpareSlots) + 255) & ~255ull;
  part_buf2(L, off, off2[chunks]);
  L.total = (L.off_fill + 8 * L.nfill + 255) & ~255ull;
  // tables after the buffers: filters, chunk owners, the first pass's work
  // items (key ranges of at most range1 keys within one dense filter; the
  // keys of direct filters are not read)
  std::vector<uint32_t> owner(chunks);
  for (uint32_t i = 0; i < nfilters; ++i) {
    const uint64_t c_end = i + 1 < nfilters ? pf[i + 1].chunk_base : chunks;
    std::fill(owner.begin() + static_cast<std::ptrdiff_t>(pf[i].chunk_base),
              owner.begin() + static_cast<std::ptrdiff_t>(c_end), i);
  }
  std::vector<PartRange> work1;
  for (uint32_t i = 0; i < nfilters; ++i) {
    if (pf[i].direct) continue;
    for (uint64_t s = pf[i].key_begin; s < pf[i].key_end; s += a.range1)
      work1.push_back(PartRange{s, std::min(s + a.range1, pf[i].key_end), i, 0});
  }
  if (work1.empty() || work1.size() > 0x7fffffffull) return BF_OK;
  // longest first: workgroups are dispatched in index order as CUs free up,
  // so the short items fill the gaps at the end
  std::stable_sort(work1.begin(), work1.end(), [](const PartRange& x, const PartRange& y) {
    return x.end - x.begin > y.end - y.begin;
  });
  const uint64_t off_pf = L.total;
  const uint64_t off_owner = (off_pf + pf.size() * sizeof(PartFilter) + 255) & ~255ull;
  const uint64_t off_first = (off_owner + owner.size() * 4 + 255) & ~255ull;
  // work lists: heavily loaded buckets are split over several workgroups
  // (~64K records per second-pass slice; ~128K per apply slice, each of
  // which then merges its whole chunk image with atomics)
  std::vector<PartWork> work2, work3;
  for (uint32_t d = 0; d < a.f1; ++d) {
    const uint64_t ns = std::clamp<uint64_t>((off1[d + 1] - off1[d] + 65535) / 65536, 1, 65535);
    for (uint64_t i = 0; i < ns; ++i)
      work2.push_back(PartWork{d, static_cast<uint16_t>(i), static_cast<uint16_t>(ns)});
  }
  for (uint64_t c = 0; c < chunks; ++c) {
    if (load[c] <= 0.0) continue;  // no records can land here: nothing to apply
    const uint64_t ns = std::clamp<uint64_t>(static_cast<uint64_t>(load[c] / 131072.0) + 1, 1, 65535);
    for (uint64_t i = 0; i < ns; ++i)
      work3.push_back(PartWork{static_cast<uint32_t>(c), static_cast<uint16_t>(i), static_cast<uint16_t>(ns)});
  }
  const uint64_t off_ext1 = (off_first + work1.size() * sizeof(PartRange) + 255) & ~255ull;
  const uint64_t off_ext2 = (off_ext1 + off1.size() * 8 + 255) & ~255ull;
  const uint64_t off_w2 = (off_ext2 + off2.size() * 8 + 255) & ~255ull;
  const uint64_t off_w3 = (off_w2 + work2.size() * sizeof(PartWork) + 255) & ~255ull;
  const uint64_t total = (off_w3 + work3.size() * sizeof(PartWork) + 255) & ~255ull;
  if (work2.size() > 0xffffffffull || work3.size() > 0xffffffffull) return BF_OK;
  b->part_scratch = lib_alloc(b->device, total, &b->pooled_scratch);
  if (b->part_scratch == nullptr) return BF_ENOMEM;
  uint8_t* base = static_cast<uint8_t*>(b->part_scratch);
  if (hipMemcpy(base + off_pf, pf.data(), pf.size() * sizeof(PartFilter), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + off_owner, owner.data(), owner.size() * 4, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + off_first, work1.data(), work1.size() * sizeof(PartRange),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + off_ext1, off1.data(), off1.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + off_ext2, off2.data(), off2.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + off_w2, work2.data(), work2.size() * sizeof(PartWork), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + off_w3, work3.data(), work3.size() * sizeof(PartWork), hipMemcpyHostToDevice) !=
          hipSuccess)
    return BF_EDEVICE;
  part_bind(a, L, b->part_scratch);
  a.off1 = reinterpret_cast<const uint64_t*>(base + off_ext1);
  a.off2 = reinterpret_cast<const uint64_t*>(base + off_ext2);
  a.work2 = reinterpret_cast<const PartWork*>(base + off_w2);
  a.nwork2 = static_cast<uint32_t>(work2.size());
  a.work3 = reinterpret_cast<const PartWork*>(base + off_w3);
  a.nwork3 = static_cast<uint32_t>(work3.size());
  a.words = pf[0].words;  // the single-filter fields mirror filter 0
  a.num_blocks = pf[0].num_blocks;
  a.hash_init = pf[0].hash_init;
  a.nb_lo = pf[0].nb_lo;
  a.nb_hi_mask = pf[0].nb_hi_mask;
  a.filters = reinterpret_cast<const PartFilter*>(base + off_pf);
  a.chunk_owner = reinterpret_cast<const uint32_t*>(base + off_owner);
  a.work1 = reinterpret_cast<const PartRange*>(base + off_first);
  a.nwork1 = static_cast<uint32_t>(work1.size());
  a.nfilters = nfilters;
  a.k = f0->k;
  a.keys = d_keys + h_offsets[0];
  b->part = a;
  b->part_layout = L;
  b->part_k = k;
  b->partitioned = true;
  b->part_direct.resize(nfilters);
  for (uint32_t i = 0; i < nfilters; ++i) b->part_direct[i] = static_cast<uint8_t>(pf[i].direct);
  return BF_OK;
}

// The plan's graph: the partitioned construction's four kernels (when
// taken), then the persistent tiled launch (when it has tiles, or when the
// plan is not partitioned).
bf_status build_graph(bf_batch* b) {
  hipGraphNode_t prev = nullptr, node = nullptr;
  if (hipGraphCreate(&b->graph, 0) != hipSuccess) return BF_EDEVICE;
  auto add_node = [&](const void* fn, dim3 grid, dim3 block, void** args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(fn);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    if (hipGraphAddKernelNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
      return false;
    prev = node;
    return true;
  };
  if (b->partitioned) {
    unsigned long long* fills = b->part.fill1;
    uint64_t nfill = b->part_layout.nfill;
    void* zargs[] = {&fills, &nfill};
    void* pargs[] = {&b->part};
    const dim3 zgrid(static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>((nfill + 255) / 256, 4096))));
    if (!add_node(reinterpret_cast<const void*>(&part_zero_kernel), zgrid, dim3(kZeroThreads), zargs) ||
        !add_node(b->part_k.scatter1, part_grid1(b->part), dim3(b->part_k.threads1), pargs) ||
        !add_node(b->part_k.scatter2, part_grid2(b->part), dim3(kScatter2Threads), pargs) ||
        !add_node(b->part_k.apply, part_grid3(b->part), dim3(kApplyThreads), pargs))
      return BF_EDEVICE;
  }
  if (!b->partitioned || b->ntiles > 0) {
    void* kargs[] = {&b->args};
    if (!add_node(b->fn, dim3(b->grid), dim3(kBlockThreads), kargs)) return BF_EDEVICE;
  }
  return hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess ? BF_OK
                                                                                     : BF_EDEVICE;
}

// The tiled direct plan: every key of the selected filters (all when
// `only` is null) in tiles of one persistent launch.  Filters go to the 8
// XCD queues by longest-processing-time on their key counts.
bf_status build_tiles(bf_batch* b, bf_filter* const* filters, uint32_t nfilters, const uint64_t* d_keys,
                      const uint64_t* h_offsets, uint8_t* d_out, const std::vector<uint8_t>* only) {
  const int op = b->op;
  const bf_filter* f0 = filters[0];
  // Mapping per size class (identical for all filters of a class).
  for (int c = 0; c < kNumSizeClasses; ++c) {
    const MapSpec m = class_map(op, f0, c);
    bf_mapping_t bm{};
    bm.lanes_per_key = m.theta;
    bm.words_per_lane = m.phi;
    bm.keys_per_lane = m.kt;
    bm.atomic_bits = op == BF_OP_ADD ? m.atomic_bits : 0;
    bm.workgroup_threads = kBlockThreads;  // tiles are planned at this size
    b->mapping[c] = bm;
  }

  std::vector<uint32_t> order(nfilters);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    return h_offsets[x + 1] - h_offsets[x] > h_offsets[y + 1] - h_offsets[y];
  });
  std::vector<std::vector<BatchTile>> queue(kXcds);
  std::vector<uint64_t> load(kXcds, 0);
  for (uint32_t i : order) {
    const uint64_t n = h_offsets[i + 1] - h_offsets[i];
    if (n == 0 || (only != nullptr && !(*only)[i])) continue;
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
  b->d_filters = static_cast<BatchFilter*>(
      lib_alloc(b->device, descs.size() * sizeof(BatchFilter), &b->pooled_filters));
  if (b->d_filters == nullptr) return BF_ENOMEM;
  b->d_tiles = static_cast<BatchTile*>(lib_alloc(b->device, tiles_bytes, &b->pooled_tiles));
  if (b->d_tiles == nullptr) return BF_ENOMEM;
  if (hipMemcpy(b->d_filters, descs.data(), descs.size() * sizeof(BatchFilter),
                hipMemcpyHostToDevice) != hipSuccess ||
      (!tiles.empty() && hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                                   hipMemcpyHostToDevice) != hipSuccess)) {
    return BF_EDEVICE;
  }

  b->args.filters = b->d_filters;
  b->args.tiles = b->d_tiles;
  b->args.ntiles = b->ntiles;
  b->args.k = f0->k;

  return BF_OK;
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
    if (f != nullptr && f->layout != BF_LAYOUT_SECTORIZED) return BF_EUNSUPPORTED;
    if (f == nullptr || f->s != f0->s || f->word_bits != f0->word_bits || f->k != f0->k ||
        f->device != f0->device || f->salts != f0->salts)
      return BF_EINVAL;
    if (h_offsets[i + 1] < h_offsets[i]) return BF_EINVAL;
  }
  const uint64_t nkeys = h_offsets[nfilters] - h_offsets[0];
  if (nkeys > 0 && (d_keys == nullptr || reinterpret_cast<uintptr_t>(d_keys) % 8 != 0))
    return BF_EINVAL;
  if (op == BF_OP_CONTAINS && nkeys > 0 && d_out == nullptr) return BF_EINVAL;

  const void* fn = kernel_table(f0->salts == kSaltsParquet).batch_fn[batch_index(op, static_cast<int>(f0->word_bits),
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
  b->device = f0->device;

  if (op == BF_OP_ADD) {
    bf_status pst = plan_partitioned(b, filters, nfilters, d_keys, h_offsets);
    if (pst != BF_OK) {
      free_plan(b);
      return pst;
    }
  }
  // The tiled direct launch: every filter, or (partitioned plan) the filters
  // left to it that have keys.
  bool tiled = !b->partitioned;
  if (b->partitioned)
    for (uint32_t i = 0; i < nfilters; ++i)
      tiled = tiled || (b->part_direct[i] && h_offsets[i + 1] > h_offsets[i]);
  if (tiled) {
    const bf_status st =
        build_tiles(b, filters, nfilters, d_keys, h_offsets, d_out, b->partitioned ? &b->part_direct : nullptr);
    if (st != BF_OK) {
      (void)hipGetLastError();
      free_plan(b);
      return st;
    }
  } else {
    b->ntiles = 0;
    b->grid = part_grid1(b->part).x;
  }
  if (build_graph(b) != BF_OK) {
    (void)hipGetLastError();
    free_plan(b);
    return BF_EDEVICE;
  }
  *out = b;
  return BF_OK;
}

bf_status bf_batch_launch(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  if (b->ntiles == 0 && !b->partitioned) return BF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return BF_EDEVICE;
  return mark_launch(b, s);
}

bf_status bf_batch_launch_direct(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->partitioned) {
    const bf_status st = part_launch(b->part, b->part_layout, b->part_k, s);
    if (st != BF_OK) return st;
  }
  if (b->ntiles > 0) {
    void* kargs[] = {&b->args};
    if (hipLaunchKernel(b->fn, dim3(b->grid), dim3(kBlockThreads), kargs, 0, s) != hipSuccess)
      return BF_EDEVICE;
  }
  return b->partitioned || b->ntiles > 0 ? mark_launch(b, s) : BF_OK;
}

bf_status bf_batch_launch_per_filter(bf_batch* b, void* stream) {
  if (b == nullptr) return BF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < b->nfilters; ++i) {
    const uint64_t n = b->offsets[i + 1] - b->offsets[i];
    if (n == 0) continue;
    const uint64_t off = b->offsets[i];
    bf_status st = b->op == BF_OP_ADD
                       ? launch_unordered(b->filters[i], BF_OP_ADD, b->d_keys + off, n, nullptr, s)
                       : launch_unordered(b->filters[i], BF_OP_CONTAINS, b->d_keys + off, n,
                                          b->d_out + off, s);
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
  i.strategy = b->partitioned ? BF_STRATEGY_PARTITIONED : BF_STRATEGY_DIRECT;
  for (int c = 0; c < kNumSizeClasses; ++c) {
    i.tiles_per_class[c] = b->tiles_per_class[c];
    i.mapping[c] = b->mapping[c];
  }
  *out = i;
  return BF_OK;
}

bf_status bf_batch_destroy(bf_batch* b) {
  if (b == nullptr) return BF_OK;
  // the host waits for the plan's own launches only (its graph is destroyed
  // next); its memory then returns to the pool in the library stream's order
  bf_status st = BF_OK;
  if (b->unmarked) {
    if (hipDeviceSynchronize() != hipSuccess) st = BF_EDEVICE;
  } else {
    for (auto& m : b->marks)
      if (hipEventSynchronize(m.second) != hipSuccess) st = BF_EDEVICE;
  }
  free_plan(b);
  return st;
}

}  // extern "C"
