// bf_internal.hpp -- the filter handle, shared by the single-filter and the
// batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/bf.h"

namespace bfhip {
// Pattern multipliers of a sectorized filter: the derived salts of
// bf_hash.hpp, or the Parquet split-block format's constants (bf_parquet.h).
constexpr uint32_t kSaltsPaper = 0;
constexpr uint32_t kSaltsParquet = 1;

// Stream order of the bf.h calls on one filter (ordered_call below).
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
  bool pooled_words;        // words from the device's filter pool (freed in stream order)
  uint32_t groups;          // cache-sectorized z, else 0
  uint32_t salts;           // sectorized pattern multipliers: bfhip::kSaltsPaper or kSaltsParquet
  uint64_t num_bits;        // nbytes * 8
  bfhip::FilterOrder order;
};

namespace bfhip {
// Partitioned construction (bf_partition.hip).
struct PartArgs;
struct PartLayout {
  uint64_t off_buf1, off_buf2, off_blk2, off_fill, nfill1, nfill, total;
  bool chunk_pass;  // one pass: the first scatter writes the chunk buckets
};
struct PartKernels {
  const void* scatter1;
  const void* scatter1_multi;  // first scatter of multi-filter plans (sectorized layout)
  const void* scatter2;
  const void* apply;
  uint32_t threads1;  // workgroup size of scatter1
  const void* scatter1_chunk = nullptr;  // first scatter into chunk buckets (one pass)
};
bool partition_applicable(const bf_filter* f, uint64_t n);
// Workspace bytes a partitioned add of n keys takes from the device pool (0
// if the filter cannot be partitioned).
uint64_t partition_workspace_bytes(const bf_filter* f, uint64_t n);
bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream);
// One partitioned pass (n keys, at most 2^28 records) over a caller-given
// workspace of ws_bytes: BF_ESCRATCH if the pass needs more, BF_EINVAL if n
// needs several passes.  Enqueues the kernels only (no allocation).
bf_status partitioned_add_in(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream,
                             void* ws, uint64_t ws_bytes);
uint32_t part_chunk_shift(uint32_t words_per_block, uint32_t word_bits);
bool part_geometry(uint64_t chunks, uint32_t chunk_shift, uint64_t n, PartArgs& a, PartLayout& L);
// Switches a one-filter geometry to sliced high-digit buckets;
// records_per_key is 1, or k for the classic filter, whose a.n and a.range1
// count keys.
void part_slice(PartArgs& a, PartLayout& L, uint64_t records_per_key);
void part_bind(PartArgs& a, const PartLayout& L, void* base);
void part_buf2(PartLayout& L, uint64_t& off, uint64_t slots);
PartKernels part_kernels(const bf_filter* f);
bf_status part_launch(const PartArgs& a, const PartLayout& L, const PartKernels& k, hipStream_t stream);
dim3 part_grid1(const PartArgs& a);
dim3 part_grid2(const PartArgs& a);
dim3 part_grid3(const PartArgs& a);
__global__ void part_zero_kernel(unsigned long long* p, uint64_t n);

// Filter allocation shared by every create call (bf_api.hip): fills nbytes,
// device, d_words (zeroed, synchronously).  On error the handle is freed.
bf_status alloc_filter_words(bf_filter* f);

// Device memory of plans and servers (bf_api.hip): taken from the stream-
// ordered pool of filter words on the library stream and complete when the
// call returns, or from hipMalloc where the device has no pool (*pooled
// false); nullptr on failure.  lib_free releases it: pooled memory in the
// library stream's order, so the caller first waits for (or orders) every
// use of it; other memory with hipFree, which waits for the whole device.
void* lib_alloc(int device, uint64_t bytes, bool* pooled);
void lib_free(int device, void* p, bool pooled);

// bf_add / bf_contains work without the per-filter stream-order bookkeeping
// (bf_api.hip), for plans and servers that order their own launches.
bf_status launch_unordered(bf_filter* f, int op, const uint64_t* keys, uint64_t n, uint8_t* out,
                           hipStream_t stream);

// The measured construction costs of f's layout (bf_tuned.hpp rows; nullptr
// if none) and the density rule built on them (bf_api.hip).
struct CrossoverRow;
const CrossoverRow* crossover_of(const bf_filter* f);
bool dense_enough(const CrossoverRow* r, uint64_t bytes, uint64_t n, bool marginal_only);

// Whether a bulk add of n keys takes the partitioned strategy (bf_api.hip).
bool use_partitioned(const bf_filter* f, uint64_t n, const bf_mapping_t& m);
// Whether bf_add of n keys on f takes the partitioned construction (the
// classic layout counts k records per key).
bool add_partitions(const bf_filter* f, uint64_t n);

// How a call touches the words, for the stream order of FilterOrder.
enum class Access {
  kUse,     // reads the words, or writes them in a way the caller orders (clear, import)
  kDirect,  // atomic OR of pattern words: commutes with other direct adds
  kOwner,   // partitioned add: loads whole chunks and stores them back
};

inline hipEvent_t new_event() {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Runs `enqueue` (which enqueues one call's work on `stream`) in the stream
// order of the filter: waits first as `access` requires, then records the
// filter's last use on `stream`.  The filter's lock is held throughout, so
// the order decided here is the order enqueued.  Work captured into a HIP
// graph is ordered by the capturing caller instead (events recorded outside
// a capture cannot be waited on inside it).
template <class F>
bf_status ordered_call(bf_filter* f, hipStream_t stream, Access access, F&& enqueue) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess) {
    (void)hipGetLastError();
    cap = hipStreamCaptureStatusNone;
  }
  if (cap != hipStreamCaptureStatusNone) return enqueue();
  FilterOrder& o = f->order;
  std::lock_guard<std::mutex> lk(o.mu);
  if (access == Access::kOwner) {
    for (const StreamMark& m : o.marks)
      if (m.stream != stream && hipStreamWaitEvent(stream, m.event, 0) != hipSuccess)
        return BF_EDEVICE;
  } else if (access == Access::kDirect && o.part_pending) {
    if (hipStreamWaitEvent(stream, o.part_event, 0) != hipSuccess) return BF_EDEVICE;
  }
  const bf_status st = enqueue();
  if (st != BF_OK) return st;
  hipEvent_t ev = nullptr;
  for (const StreamMark& m : o.marks)
    if (m.stream == stream) ev = m.event;
  if (ev == nullptr) {
    ev = new_event();
    if (ev == nullptr) return BF_EDEVICE;
    o.marks.push_back(StreamMark{stream, ev});
  }
  if (hipEventRecord(ev, stream) != hipSuccess) return BF_EDEVICE;
  if (access == Access::kOwner) {
    if (o.part_event == nullptr && (o.part_event = new_event()) == nullptr) return BF_EDEVICE;
    if (hipEventRecord(o.part_event, stream) != hipSuccess) return BF_EDEVICE;
    o.part_pending = true;
    // every other stream's last use is ordered before this add: its mark
    // on `stream` stands for them from now on
    for (const StreamMark& m : o.marks)
      if (m.stream != stream) (void)hipEventDestroy(m.event);
    o.marks.assign(1, StreamMark{stream, ev});
  }
  return BF_OK;
}

// The classic and cache-sectorized layouts (bf_variants.hip).
bf_mapping_t variant_resolve_mapping(const bf_filter* f, int op);
bf_status variant_validate_mapping(const bf_filter* f, int op, const bf_mapping_t& m);
bf_status variant_launch(bf_filter* f, int op, const uint64_t* keys, uint64_t n, uint8_t* out,
                         hipStream_t stream);
}  // namespace bfhip
