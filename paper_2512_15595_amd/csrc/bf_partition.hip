// bf_partition.hip -- host side of partitioned construction: geometry,
// bucket capacities, workspace and the launch sequence (kernels in
// bf_partition.hpp), for one filter and for a table of filters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

#include "bf_internal.hpp"
#include "bf_variant_registry.hpp"
#include "bf_partition.hpp"
#include "bf_registry.hpp"

namespace bfhip {

__global__ __launch_bounds__(kZeroThreads) void part_zero_kernel(unsigned long long* p, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kZeroThreads;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kZeroThreads + threadIdx.x; i < n; i += stride)
    p[i] = 0;
}

namespace {

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

uint32_t ceil_pow2(uint64_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Expected bucket load of uniformly hashed records plus six standard
// deviations and a fixed margin.
uint64_t capacity(double mean, uint64_t margin, uint64_t align) {
  const double c = mean + 6.0 * std::sqrt(mean) + static_cast<double>(margin);
  const uint64_t v = static_cast<uint64_t>(std::ceil(c));
  return (v + align - 1) / align * align;
}

}  // namespace

uint32_t part_chunk_shift(uint32_t words_per_block, uint32_t word_bits) {
  const uint64_t bpc = kChunkBytes / (static_cast<uint64_t>(words_per_block) * word_bits / 8);
  uint32_t shift = 0;
  while ((1ull << shift) < bpc) ++shift;
  return shift;
}

// The chunk buckets' two arrays from byte offset `off` (advanced past them):
// `slots` lo32 words and kSpareSlots spare ones, then as many 16-bit blocks.
void part_buf2(PartLayout& L, uint64_t& off, uint64_t slots) {
  L.off_buf2 = off;
  off = align256(off + 4 * (slots + kSpareSlots));
  L.off_blk2 = off;
  off = align256(off + 2 * (slots + kSpareSlots));
  L.off_fill = off;
}

bool part_geometry(uint64_t chunks, uint32_t chunk_shift, uint64_t n, PartArgs& a, PartLayout& L) {
  a.chunk_shift = chunk_shift;
  a.chunks = chunks;
  // digits balanced between the passes: f2 ~ sqrt(chunks)
  const uint64_t root = static_cast<uint64_t>(std::ceil(std::sqrt(static_cast<double>(chunks))));
  a.f2 = std::min<uint32_t>(ceil_pow2(std::max<uint64_t>(root, 1)), kMaxDigits2);
  a.low_bits = 0;
  while ((1u << a.low_bits) < a.f2) ++a.low_bits;
  const uint64_t f1 = (chunks + a.f2 - 1) / a.f2;
  if (f1 > static_cast<uint64_t>(kMaxDigits) || chunks == 0) return false;
  a.f1 = static_cast<uint32_t>(f1);
  a.n = n;
  uint64_t range = (n + 1023) / 1024;
  range = (range + kPartStep - 1) / kPartStep * kPartStep;
  a.range1 = std::max<uint64_t>(range, kPartStep);
  a.cap1 = capacity(static_cast<double>(n) / a.f1, 4 * kPartStep, 64);
  a.cap2 = capacity(static_cast<double>(n) / chunks, 64, 16);
  const uint64_t per_bucket = std::min<uint64_t>(a.cap1, n);
  a.q = static_cast<uint32_t>(std::clamp<uint64_t>((per_bucket + 65535) / 65536, 1, 32));
  // A filter of few chunks (L2 or Infinity-Cache sized) leaves too few
  // digits to fill 256 CUs: cut the second pass into more slices (at least
  // 16 Ki records each) and split every chunk's records over several apply
  // workgroups (at least 8 Ki records each), so that both grids reach about
  // a thousand or two workgroups.  Split slices merge with atomic OR.
  const uint64_t q_fill = (1024 + a.f1 - 1) / a.f1;
  a.q = static_cast<uint32_t>(std::clamp<uint64_t>(
      std::max<uint64_t>(a.q, std::min<uint64_t>(q_fill, per_bucket / 16384)), 1, 1024));
  const uint64_t split_fill = (2048 + chunks - 1) / chunks;
  a.apply_split = static_cast<uint32_t>(std::clamp<uint64_t>(
      std::min<uint64_t>(split_fill, n / chunks / 8192), 1, 1024));
  uint64_t off = 0;
  L.off_buf1 = off;
  a.spare1 = static_cast<uint64_t>(a.f1) * a.cap1;
  off = align256(off + 8ull * (a.spare1 + kSpareSlots));
  a.spare2 = chunks * a.cap2;
  part_buf2(L, off, a.spare2);
  L.nfill1 = a.f1;
  L.nfill = a.f1 + chunks;
  off = align256(off + 8ull * L.nfill);
  L.total = off;
  return true;
}

// Sliced high-digit buckets: pass-1 workgroup w owns slice (d, w) of every
// high digit d, sized for its expected share range1 * records_per_key / f1.
// Slices hold the slack (six standard deviations) that a shared bucket needs
// only once, so the first record buffer takes more address space; traffic
// is unchanged, as only filled records are written and read.
void part_slice(PartArgs& a, PartLayout& L, uint64_t records_per_key) {
  a.g1 = static_cast<uint32_t>(std::max<uint64_t>((a.n + a.range1 - 1) / a.range1, 1));
  a.q = std::min<uint32_t>(a.q, a.g1);  // every pass-2 workgroup reads a slice
  a.cs1 = capacity(static_cast<double>(a.range1 * records_per_key) / a.f1, 16, 16);
  uint64_t off = 0;
  L.off_buf1 = off;
  a.spare1 = static_cast<uint64_t>(a.f1) * a.g1 * a.cs1;
  off = align256(off + 8ull * (a.spare1 + kSpareSlots));
  a.spare2 = a.chunks * a.cap2;
  part_buf2(L, off, a.spare2);
  L.nfill1 = static_cast<uint64_t>(a.f1) * a.g1;
  L.nfill = L.nfill1 + a.chunks;
  off = align256(off + 8ull * L.nfill);
  L.total = off;
}

namespace {

// One pass for a filter of at most kChunkDigits chunks: the first scatter's
// digit is the chunk (f1 = chunks, no low digit), and it claims runs in the
// chunk buckets directly, so there is no first record buffer and no second
// pass.  A digit's run in a step is then 8192 / chunks records on average,
// down to 8 at 1024 chunks, so more of the stored lines are partial; the
// second pass it saves costs more (measured on MI355X, 2^26 keys into 16,
// 32 and 64 MiB of 256-bit blocks: 95, 103 and 102 Gkeys/s in two passes,
// 139, 133 and 120 in one).
void chunk_geometry(uint64_t chunks, uint32_t chunk_shift, uint64_t n, PartArgs& a, PartLayout& L) {
  a.chunk_shift = chunk_shift;
  a.chunks = chunks;
  a.f2 = 1;
  a.low_bits = 0;
  a.f1 = static_cast<uint32_t>(chunks);
  a.q = 1;
  a.n = n;
  uint64_t range = (n + 1023) / 1024;
  range = (range + kPartStep - 1) / kPartStep * kPartStep;
  a.range1 = std::max<uint64_t>(range, kPartStep);
  a.cap1 = 0;
  a.cs1 = 0;
  a.spare1 = 0;
  a.cap2 = capacity(static_cast<double>(n) / chunks, 64, 16);
  const uint64_t split_fill = (2048 + chunks - 1) / chunks;
  a.apply_split = static_cast<uint32_t>(std::clamp<uint64_t>(
      std::min<uint64_t>(split_fill, n / chunks / 8192), 1, 1024));
  uint64_t off = 0;
  L.off_buf1 = 0;
  a.spare2 = chunks * a.cap2;
  part_buf2(L, off, a.spare2);
  L.nfill1 = 0;
  L.nfill = chunks;
  off = align256(off + 8ull * L.nfill);
  L.total = off;
  L.chunk_pass = true;
}

}  // namespace

void part_bind(PartArgs& a, const PartLayout& L, void* base_ptr) {
  uint8_t* base = static_cast<uint8_t*>(base_ptr);
  a.buf1 = reinterpret_cast<uint64_t*>(base + L.off_buf1);
  a.buf2 = reinterpret_cast<uint32_t*>(base + L.off_buf2);
  a.blk2 = reinterpret_cast<uint16_t*>(base + L.off_blk2);
  a.fill1 = reinterpret_cast<unsigned long long*>(base + L.off_fill);
  a.fill2 = a.fill1 + L.nfill1;
}

PartKernels part_kernels(const bf_filter* f) {
  if (f->layout == BF_LAYOUT_CLASSIC) {
    ensure_variant_registry();
    const VariantRegistry& r = variant_registry();
    const bool pow2 = (f->num_bits & (f->num_bits - 1)) == 0;
    return PartKernels{r.classic_part1[k_index(f->k) * 2 + (pow2 ? 1 : 0)], nullptr, r.classic_part2,
                       r.classic_apply, kClassicThreads};
  }
  if (f->layout == BF_LAYOUT_CACHE_SECTORIZED) {
    ensure_variant_registry();
    const VariantRegistry& r = variant_registry();
    const int idx = csbf_part_index(static_cast<int>(f->word_bits), static_cast<int>(f->s),
                                    static_cast<int>(f->groups), k_index(f->k));
    return PartKernels{r.csbf_part1[idx], nullptr, r.csbf_part2[idx], r.csbf_apply[idx],
                       kScatter1Threads, r.csbf_part1_chunk[idx]};
  }
  const int idx = batch_index(0, static_cast<int>(f->word_bits), static_cast<int>(f->s),
                              k_index(f->k));
  const Registry& r = kernel_table(f->salts == kSaltsParquet);
  return PartKernels{r.part1_fn[idx], r.part1_multi_fn[idx], r.part2_fn[idx], r.apply_fn[idx],
                     kScatter1Threads, r.part1_chunk_fn[idx]};
}

bf_status part_launch(const PartArgs& a, const PartLayout& L, const PartKernels& k,
                      hipStream_t stream) {
  if (L.chunk_pass ? (k.scatter1_chunk == nullptr || k.apply == nullptr)
                   : (k.scatter1 == nullptr || k.scatter2 == nullptr || k.apply == nullptr))
    return BF_EUNSUPPORTED;
  // shared buckets' fill counters start at zero; slice counts are written
  // by their owners
  const uint64_t zbegin = a.cs1 ? L.nfill1 : 0, zn = L.nfill - zbegin;
  const uint64_t zgrid = std::min<uint64_t>((zn + kZeroThreads - 1) / kZeroThreads, 4096);
  hipLaunchKernelGGL(part_zero_kernel, dim3(static_cast<uint32_t>(std::max<uint64_t>(zgrid, 1))),
                     dim3(kZeroThreads), 0, stream, a.fill1 + zbegin, zn);
  PartArgs copy = a;
  void* args[] = {&copy};
  if (L.chunk_pass) {
    if (hipLaunchKernel(k.scatter1_chunk, part_grid1(a), dim3(kScatter1Threads), args, 0, stream) != hipSuccess ||
        hipLaunchKernel(k.apply, part_grid3(a), dim3(kApplyThreads), args, 0, stream) != hipSuccess)
      return BF_EDEVICE;
  } else if (hipLaunchKernel(k.scatter1, part_grid1(a), dim3(k.threads1), args, 0, stream) != hipSuccess ||
             hipLaunchKernel(k.scatter2, part_grid2(a), dim3(kScatter2Threads), args, 0, stream) !=
                 hipSuccess ||
             hipLaunchKernel(k.apply, part_grid3(a), dim3(kApplyThreads), args, 0, stream) != hipSuccess) {
    return BF_EDEVICE;
  }
  return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

dim3 part_grid1(const PartArgs& a) {
  if (a.work1) return dim3(a.nwork1);
  return dim3(static_cast<uint32_t>((a.n + a.range1 - 1) / a.range1));
}
dim3 part_grid2(const PartArgs& a) { return dim3(a.work2 ? a.nwork2 : a.f1 * a.q); }
dim3 part_grid3(const PartArgs& a) {
  const uint64_t items = a.work3 ? a.nwork3 : a.chunks * std::max<uint32_t>(a.apply_split, 1);
  return dim3(static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(items, 65535))));
}

namespace {

// The classic filter is partitioned as blocks of one 32-bit word, with k
// records per key; its first pass counts keys (a.n, a.range1) in whole steps
// of kClassicThreads * (kPartStep / kClassicThreads / k) keys.
bool single_geometry(const bf_filter* f, uint64_t n, PartArgs& a, PartLayout& L) {
  if (f->layout == BF_LAYOUT_CLASSIC) {
    const uint32_t shift = part_chunk_shift(1, 32);
    const uint64_t words = f->num_bits / 32;
    const uint64_t chunks = (words + (1ull << shift) - 1) >> shift;
    if (!part_geometry(chunks, shift, n * f->k, a, L)) return false;
    const uint64_t step = static_cast<uint64_t>(kClassicThreads) * (kPartStep / kClassicThreads / f->k);
    const uint64_t range = (n + 1023) / 1024;
    a.n = n;
    a.range1 = std::max<uint64_t>((range + step - 1) / step * step, step);
    part_slice(a, L, f->k);
    return true;
  }
  const uint32_t shift = part_chunk_shift(f->s, f->word_bits);
  const uint64_t chunks = (f->num_blocks + (1ull << shift) - 1) >> shift;
  if (chunks <= static_cast<uint64_t>(kChunkDigits)) {
    chunk_geometry(chunks, shift, n, a, L);
    return true;
  }
  if (!part_geometry(chunks, shift, n, a, L)) return false;
  part_slice(a, L, 1);
  return true;
}

}  // namespace

bool partition_applicable(const bf_filter* f, uint64_t n) {
  if (f->layout == BF_LAYOUT_SECTORIZED_CHAINED) return false;
  // classic records address 32-bit words by a 32-bit index (m <= 2^37) and
  // need a compiled k (at most 16 positions per key)
  if (f->layout == BF_LAYOUT_CLASSIC && (f->num_bits > (1ull << 37) || k_index(f->k) == 0))
    return false;
  PartArgs a{};
  PartLayout L{};
  return n > 0 && n < (1ull << 40) && single_geometry(f, 1, a, L);
}

namespace {

// The construction workspace comes from one stream-ordered memory pool per
// device: taken at the start of a partitioned add and returned at its end
// on the same stream, so an add never synchronizes the device and no filter
// keeps a workspace.  The pool keeps its peak size reserved (release
// threshold: never), so steady use does not remap memory.
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;

hipMemPool_t workspace_pool(int device) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pools.find(device);
  if (it != g_pools.end()) return it->second;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  hipMemPool_t pool = nullptr;
  if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  uint64_t keep = UINT64_MAX;
  (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  g_pools[device] = pool;
  return pool;
}

}  // namespace

namespace {

// One pass of a partitioned add over the workspace `ws` (at least L.total
// bytes of the geometry single_geometry gives for n): sets the arguments and
// enqueues the kernels.
bf_status partitioned_pass_in(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream,
                              PartArgs& a, const PartLayout& L, void* ws) {
  const PartKernels k = part_kernels(f);
  if (k.scatter1 == nullptr) return BF_EUNSUPPORTED;
  part_bind(a, L, ws);
  a.words = f->d_words;
  a.num_blocks = f->layout == BF_LAYOUT_CLASSIC ? f->num_bits / 32 : f->num_blocks;
  a.num_bits = f->num_bits;
  if ((f->num_bits & (f->num_bits - 1)) == 0) {
    uint32_t lg = 0;
    while ((1ull << lg) < f->num_bits) ++lg;
    a.bit_shift = 64 - lg;
  }
  a.hash_init = xxh64_u64_init(f->seed);
  a.nb_lo = static_cast<uint32_t>(f->num_blocks);
  a.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
  a.nfilters = 1;
  // the cache-sectorized rule takes the bits per selected word
  a.k = f->layout == BF_LAYOUT_CACHE_SECTORIZED ? f->k / f->groups : f->k;
  a.keys = keys;
  return part_launch(a, L, k, stream);
}

// One pass with its workspace taken from the device pool and returned at
// its end, both in stream order.
bf_status partitioned_pass(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream) {
  PartArgs a{};
  PartLayout L{};
  if (!single_geometry(f, n, a, L)) return BF_EUNSUPPORTED;
  if (part_kernels(f).scatter1 == nullptr) return BF_EUNSUPPORTED;
  hipMemPool_t pool = workspace_pool(f->device);
  if (pool == nullptr) return BF_EDEVICE;
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, L.total, pool, stream) != hipSuccess) {
    (void)hipGetLastError();
    return BF_ENOMEM;
  }
  bf_status st = partitioned_pass_in(f, keys, n, stream, a, L, ws);
  if (hipFreeAsync(ws, stream) != hipSuccess && st == BF_OK) st = BF_EDEVICE;
  return st;
}

}  // namespace

bf_status partitioned_add_in(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream,
                             void* ws, uint64_t ws_bytes) {
  const uint64_t per_key = f->layout == BF_LAYOUT_CLASSIC ? f->k : 1;
  if (n == 0 || n > std::max<uint64_t>((1ull << 28) / per_key, 1)) return BF_EINVAL;
  PartArgs a{};
  PartLayout L{};
  if (!single_geometry(f, n, a, L)) return BF_EUNSUPPORTED;
  if (L.total > ws_bytes) return BF_ESCRATCH;
  return partitioned_pass_in(f, keys, n, stream, a, L, ws);
}

// Passes of at most 2^28 records keep the workspace under ~5.5 GB; each pass
// after the first reads and writes the touched chunks once more.
bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream) {
  const uint64_t per_key = f->layout == BF_LAYOUT_CLASSIC ? f->k : 1;
  const uint64_t max_keys = std::max<uint64_t>((1ull << 28) / per_key, 1);
  for (uint64_t off = 0; off < n; off += max_keys) {
    const bf_status st = partitioned_pass(f, keys + off, std::min(max_keys, n - off), stream);
    if (st != BF_OK) return st;
  }
  return BF_OK;
}

uint64_t partition_workspace_bytes(const bf_filter* f, uint64_t n) {
  PartArgs a{};
  PartLayout L{};
  const uint64_t per_key = f->layout == BF_LAYOUT_CLASSIC ? f->k : 1;
  n = std::min(n, std::max<uint64_t>((1ull << 28) / per_key, 1));
  if (!partition_applicable(f, n) || !single_geometry(f, n, a, L)) return 0;
  return L.total;
}

}  // namespace bfhip
