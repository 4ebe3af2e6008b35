// bf_api.hip -- the C ABI declared in include/bf.h: handle, validation,
// mapping selection and kernel launch.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <new>

#include "../../include/bf.h"
#include "bf_hash.hpp"
#include "bf_kernels.hpp"
#include "bf_registry.hpp"
#include "bf_tuned.hpp"
#include "bf_internal.hpp"

namespace bfhip {

Registry& registry() {
  static Registry r{};
  return r;
}

namespace {
std::once_flag g_registry_once;
}  // namespace

void ensure_registry() {
  std::call_once(g_registry_once, [] {
    Registry& r = registry();
    register_u32_s1(r);
    register_u32_s2(r);
    register_u32_s4(r);
    register_u32_s8(r);
    register_u32_s16(r);
    register_u64_s1(r);
    register_u64_s2(r);
    register_u64_s4(r);
    register_u64_s8(r);
    register_u64_s16(r);
  });
}

namespace {

// Zero fill with 16-byte stores (a kernel rather than hipMemsetAsync so a
// captured graph holds no memset node).
__global__ __launch_bounds__(256) void clear_kernel(uint8_t* p, uint64_t nbytes) {
  const uint64_t nvec = nbytes / 16;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  u32x4* q = reinterpret_cast<u32x4*>(p);
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec;
       i += stride)
    q[i] = u32x4{0u, 0u, 0u, 0u};
  // tail (< 16 bytes; the words are 4-byte multiples)
  const uint64_t tail = nvec * 16;
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tail + 4 * t < nbytes && t < 4) reinterpret_cast<uint32_t*>(p + tail)[t] = 0u;
}

bool is_pow2(uint32_t v) { return v != 0 && (v & (v - 1)) == 0; }

}  // namespace
}  // namespace bfhip

using namespace bfhip;


namespace {

// The tuned default of one operation on f for a batch of n keys.
bf_mapping_t default_mapping(const bf_filter* f, int op, uint64_t n) {
  const MapSpec t = tuned_map(op, static_cast<int>(f->word_bits), static_cast<int>(f->s),
                              size_class_of(f->nbytes), static_cast<int>(f->k), n_class_of(n));
  bf_mapping_t m{};
  m.lanes_per_key = t.theta;
  m.words_per_lane = t.phi;
  m.keys_per_lane = t.kt;
  m.atomic_bits = op == BF_OP_ADD ? t.atomic_bits : 0;
  m.max_workgroups = t.max_workgroups;
  m.workgroup_threads = t.wg_threads;
  return m;
}

// The mapping an operation of n keys runs with: the caller's fields, and
// the tuned default for those left 0.
bf_mapping_t resolve_mapping(const bf_filter* f, int op, uint64_t n) {
  if (f->layout != BF_LAYOUT_SECTORIZED) return variant_resolve_mapping(f, op);
  bf_mapping_t m = f->mapping[op];
  const bf_mapping_t def = default_mapping(f, op, n);
  if (m.lanes_per_key == 0 && m.words_per_lane == 0 && m.keys_per_lane == 0) {
    const uint32_t cap = m.max_workgroups;
    const uint32_t ab = m.atomic_bits;
    const uint32_t strategy = m.strategy;
    const uint32_t wg = m.workgroup_threads;
    m = def;
    if (cap != 0) m.max_workgroups = cap;
    m.strategy = strategy;
    if (wg != 0) m.workgroup_threads = wg;
    if (ab != 0 && op == BF_OP_ADD && f->word_bits == 32 && m.words_per_lane >= 2) m.atomic_bits = ab;
  }
  if (m.workgroup_threads == 0) m.workgroup_threads = def.workgroup_threads;
  if (m.workgroup_threads == 0) m.workgroup_threads = kBlockThreads;
  if (m.atomic_bits == 0) m.atomic_bits = 32;
  if (k_index(f->k) == 0) {
    m.lanes_per_key = 1;
    m.words_per_lane = f->s;
    m.keys_per_lane = 1;
    if (!(f->word_bits == 32 && f->s >= 2)) m.atomic_bits = 32;
  }
  if (op == BF_OP_CONTAINS) m.atomic_bits = 0;
  return m;
}

bf_status validate_mapping(const bf_filter* f, int op, const bf_mapping_t& m) {
  if (f->layout != BF_LAYOUT_SECTORIZED) return variant_validate_mapping(f, op, m);
  if (m.strategy > BF_STRATEGY_PARTITIONED) return BF_EINVAL;
  if (op == BF_OP_CONTAINS && m.strategy != BF_STRATEGY_AUTO) return BF_EINVAL;
  if (!(m.workgroup_threads == 0 || m.workgroup_threads == 64 || m.workgroup_threads == 128 ||
        m.workgroup_threads == 256))
    return BF_EINVAL;
  if (m.lanes_per_key == 0 && m.words_per_lane == 0 && m.keys_per_lane == 0) {
    // default mapping; only the atomic width may be forced
    if (m.atomic_bits != 0 && m.atomic_bits != 32 && m.atomic_bits != 64) return BF_EINVAL;
    return BF_OK;
  }
  if (!is_pow2(m.lanes_per_key) || !is_pow2(m.words_per_lane)) return BF_EINVAL;
  if (m.lanes_per_key > 16) return BF_EINVAL;
  if (static_cast<uint64_t>(m.lanes_per_key) * m.words_per_lane > f->s) return BF_EINVAL;
  if (!(m.keys_per_lane == 1 || m.keys_per_lane == 2 || m.keys_per_lane == 4)) return BF_EINVAL;
  if (op == BF_OP_ADD) {
    if (!(m.atomic_bits == 0 || m.atomic_bits == 32 || m.atomic_bits == 64)) return BF_EINVAL;
    if (m.atomic_bits == 64 && !(f->word_bits == 32 && m.words_per_lane >= 2)) return BF_EINVAL;
  } else if (m.atomic_bits != 0) {
    return BF_EINVAL;
  }
  return BF_OK;
}

bf_status launch(bf_filter* f, int op, const uint64_t* keys, uint64_t n, uint8_t* out,
                 void* stream) {
  if (f->layout != BF_LAYOUT_SECTORIZED)
    return variant_launch(f, op, keys, n, out, static_cast<hipStream_t>(stream));
  const Registry& reg = kernel_table(f->salts == kSaltsParquet);
  bf_mapping_t m = resolve_mapping(f, op, n);
  if (op == BF_OP_ADD && add_partitions(f, n))
    return partitioned_add(f, keys, n, static_cast<hipStream_t>(stream));
  // Keys per lane needs 8*KT-byte aligned keys (and KT-byte aligned results);
  // fall back to fewer keys per lane otherwise.
  uint32_t kt = m.keys_per_lane;
  while (kt > 1 && ((reinterpret_cast<uintptr_t>(keys) % (8u * kt)) != 0 ||
                    (out != nullptr && reinterpret_cast<uintptr_t>(out) % kt != 0)))
    kt >>= 1;
  int atom64 = (op == BF_OP_ADD && m.atomic_bits == 64) ? 1 : 0;
  const int kidx = k_index(f->k);
  if (kidx == 0) {
    // k without compiled variants: one lane per key, one key per lane.
    m.lanes_per_key = 1;
    m.words_per_lane = f->s;
    kt = 1;
    if (atom64 && !(f->word_bits == 32 && f->s >= 2)) atom64 = 0;
  }
  const void* fn = reg.fn[registry_index(op, static_cast<int>(f->word_bits),
                                                static_cast<int>(f->s), kidx,
                                                static_cast<int>(m.lanes_per_key),
                                                static_cast<int>(m.words_per_lane),
                                                static_cast<int>(kt), atom64)];
  if (fn == nullptr) return BF_EUNSUPPORTED;

  const uint32_t wg = m.workgroup_threads;
  const uint64_t tile = static_cast<uint64_t>(wg) * kt;
  const uint64_t ntiles = (n + tile - 1) / tile;
  uint64_t grid = ntiles;
  const uint64_t hard_cap = 1ull << 22;  // keeps grid * 256 below 2^32
  if (grid > hard_cap) grid = hard_cap;
  if (m.max_workgroups != 0 && grid > m.max_workgroups) grid = m.max_workgroups;

  BfArgs a{};
  a.words = f->d_words;
  a.keys = keys;
  a.out = out;
  a.n = n;
  a.hash_init = xxh64_u64_init(f->seed);
  a.nb_lo = static_cast<uint32_t>(f->num_blocks);
  a.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
  a.k = f->k;
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(fn, dim3(static_cast<uint32_t>(grid)), dim3(wg), args, 0,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return BF_EDEVICE;
  return BF_OK;
}

bf_status clear_words(void* p, uint64_t nbytes, hipStream_t stream) {
  uint64_t nvec = nbytes / 16;
  uint64_t grid = (nvec + 255) / 256;
  if (grid < 1) grid = 1;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(clear_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, stream,
                     static_cast<uint8_t*>(p), nbytes);
  return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

// Releases the filter's events after either waiting for its last use on
// every stream on the host (wait_stream == nullptr) or making wait_stream
// wait for them.
bf_status drain_filter(bf_filter* f, hipStream_t wait_stream) {
  FilterOrder& o = f->order;
  std::lock_guard<std::mutex> lk(o.mu);
  bf_status st = BF_OK;
  for (const StreamMark& m : o.marks) {
    const hipError_t e = wait_stream != nullptr ? hipStreamWaitEvent(wait_stream, m.event, 0)
                                                : hipEventSynchronize(m.event);
    if (e != hipSuccess) st = BF_EDEVICE;
    (void)hipEventDestroy(m.event);
  }
  o.marks.clear();
  if (o.part_event != nullptr) (void)hipEventDestroy(o.part_event);
  o.part_event = nullptr;
  o.part_pending = false;
  return st;
}

}  // namespace

namespace {

// Per device: a memory pool for filter words and a library stream on which
// words are allocated, zeroed and released.  Pool memory is released in
// stream order (hipFreeAsync), so destroying a filter waits for nothing but
// that filter's own calls; hipFree would wait for every stream of the
// device.  The pool returns freed memory to the device at the next
// synchronization (release threshold 0).
struct WordsHome {
  hipMemPool_t pool = nullptr;
  hipStream_t stream = nullptr;
};
std::mutex g_home_mu;
std::map<int, WordsHome> g_homes;

WordsHome words_home(int device) {
  std::lock_guard<std::mutex> lk(g_home_mu);
  WordsHome& h = g_homes[device];
  if (h.stream == nullptr) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    hipStream_t stream = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      return WordsHome{};
    }
    uint64_t keep = 0;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipMemPoolDestroy(pool);
      return WordsHome{};
    }
    h.pool = pool;
    h.stream = stream;
  }
  return h;
}

}  // namespace

void* bfhip::lib_alloc(int device, uint64_t bytes, bool* pooled) {
  *pooled = false;
  void* p = nullptr;
  const WordsHome home = words_home(device);
  if (home.pool != nullptr) {
    if (hipMallocFromPoolAsync(&p, bytes, home.pool, home.stream) == hipSuccess) {
      if (hipStreamSynchronize(home.stream) == hipSuccess) {
        *pooled = true;
        return p;
      }
      (void)hipFreeAsync(p, home.stream);
      return nullptr;
    }
    (void)hipGetLastError();
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void bfhip::lib_free(int device, void* p, bool pooled) {
  if (p == nullptr) return;
  if (pooled)
    (void)hipFreeAsync(p, words_home(device).stream);
  else
    (void)hipFree(p);
}

bf_status bfhip::alloc_filter_words(bf_filter* f) {
  f->num_bits = f->nbytes * 8;
  f->owns_words = true;
  if (hipGetDevice(&f->device) != hipSuccess) {
    delete f;
    return BF_EDEVICE;
  }
  const WordsHome home = words_home(f->device);
  hipStream_t s = home.stream;
  f->pooled_words = home.pool != nullptr &&
                    hipMallocFromPoolAsync(&f->d_words, f->nbytes, home.pool, s) == hipSuccess;
  if (!f->pooled_words) {
    // no pool on this device: plain allocation, zeroed on the null stream
    (void)hipGetLastError();
    s = nullptr;
    if (hipMalloc(&f->d_words, f->nbytes) != hipSuccess) {
      (void)hipGetLastError();
      delete f;
      return BF_ENOMEM;
    }
  }
  if (clear_words(f->d_words, f->nbytes, s) != BF_OK || hipStreamSynchronize(s) != hipSuccess) {
    if (f->pooled_words) {
      (void)hipFreeAsync(f->d_words, s);
      (void)hipStreamSynchronize(s);
    } else {
      (void)hipFree(f->d_words);
    }
    delete f;
    return BF_EDEVICE;
  }
  return BF_OK;
}

// The measured cost model of the two constructions for f's layout (the
// autotuner's crossover rows; nullptr if the layout has none).
const CrossoverRow* bfhip::crossover_of(const bf_filter* f) {
  switch (f->layout) {
    case BF_LAYOUT_SECTORIZED:
      return crossover_row(0, static_cast<int>(f->word_bits), static_cast<int>(f->s), 0, 0);
    case BF_LAYOUT_CLASSIC:
      return crossover_row(1, 32, 1, 0, static_cast<int>(f->k));
    case BF_LAYOUT_CACHE_SECTORIZED:
      return crossover_row(2, static_cast<int>(f->word_bits), static_cast<int>(f->s),
                           static_cast<int>(f->groups), 0);
    default:
      return nullptr;
  }
}

// Whether n keys are dense enough in a filter of `bytes` for a partitioned
// construction, by the layout's measured costs: partitioned ~ a + b * MiB +
// c * n against direct ~ d * n (d of the filter's size class).  With
// marginal_only the fixed cost a is left out (a batched plan shares it over
// its filters).  Without a measured row: 1.5 M keys + bytes / 80 (the
// sectorized 256-bit layout's fit).
bool bfhip::dense_enough(const CrossoverRow* r, uint64_t bytes, uint64_t n, bool marginal_only) {
  if (r == nullptr) return n >= (marginal_only ? 0 : 3 * (1ull << 19)) + bytes / 80;
  const double gain = r->d_ps[size_class_of(bytes)] - r->c_ps;  // ps saved per key
  if (gain <= 0.0) return false;
  const double cost_us = (marginal_only ? 0.0 : r->a_us) +
                         r->b_us_per_mib * static_cast<double>(bytes) / (1 << 20);
  return static_cast<double>(n) * gain * 1e-6 > cost_us;
}

// Strategy of one bulk add: partitioned when asked for, or (auto) when the
// batch is dense enough for streaming the touched chunks to beat one
// memory-side atomic group per key (n counts records: k per key for the
// classic layout).
bool bfhip::use_partitioned(const bf_filter* f, uint64_t n, const bf_mapping_t& m) {
  if (m.strategy == BF_STRATEGY_DIRECT) return false;
  if (!partition_applicable(f, n)) return false;
  if (m.strategy == BF_STRATEGY_PARTITIONED) return true;
  const CrossoverRow* r = crossover_of(f);
  // the classic rows are measured in keys, the fallback rule in records
  const uint64_t units = (r != nullptr && f->layout == BF_LAYOUT_CLASSIC) ? n / f->k : n;
  return dense_enough(r, f->nbytes, units, false);
}

bool bfhip::add_partitions(const bf_filter* f, uint64_t n) {
  const uint64_t records = f->layout == BF_LAYOUT_CLASSIC ? n * f->k : n;
  return use_partitioned(f, records, f->mapping[BF_OP_ADD]);
}

// The work of one bf_add / bf_contains without the filter's stream-order
// bookkeeping, for batched plans and servers, which order their own launches
// (bf_batch.h, bf_serve.h).  Arguments are already validated.
bf_status bfhip::launch_unordered(bf_filter* f, int op, const uint64_t* keys, uint64_t n,
                                  uint8_t* out, hipStream_t stream) {
  if (n == 0) return BF_OK;
  return launch(f, op, keys, n, out, stream);
}

extern "C" {

bf_status bf_create(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits, uint32_t k,
                    uint64_t seed, bf_filter** out) {
  if (out == nullptr) return BF_EINVAL;
  const uint32_t s = words_per_block;
  if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return BF_EINVAL;
  if (!(word_bits == 32 || word_bits == 64)) return BF_EINVAL;
  if (k < s || k > static_cast<uint32_t>(kMaxK)) return BF_EINVAL;
  if (num_blocks < 1 || num_blocks > (1ull << 32)) return BF_EINVAL;

  bf_filter* f = new (std::nothrow) bf_filter{};
  if (f == nullptr) return BF_ENOMEM;
  f->layout = BF_LAYOUT_SECTORIZED;
  f->num_blocks = num_blocks;
  f->s = s;
  f->word_bits = word_bits;
  f->k = k;
  f->seed = seed;
  f->nbytes = num_blocks * s * (word_bits / 8);
  const bf_status st = alloc_filter_words(f);
  if (st != BF_OK) return st;
  *out = f;
  return BF_OK;
}

bf_status bf_create_in(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                       uint32_t k, uint64_t seed, void* d_words, uint64_t nbytes, bf_filter** out) {
  if (out == nullptr || d_words == nullptr) return BF_EINVAL;
  const uint32_t s = words_per_block;
  if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return BF_EINVAL;
  if (!(word_bits == 32 || word_bits == 64)) return BF_EINVAL;
  if (k < s || k > static_cast<uint32_t>(kMaxK)) return BF_EINVAL;
  if (num_blocks < 1 || num_blocks > (1ull << 32)) return BF_EINVAL;
  if (nbytes != num_blocks * s * (word_bits / 8)) return BF_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_words) % 256 != 0) return BF_EINVAL;
  bf_filter* f = new (std::nothrow) bf_filter{};
  if (f == nullptr) return BF_ENOMEM;
  f->layout = BF_LAYOUT_SECTORIZED;
  f->num_blocks = num_blocks;
  f->s = s;
  f->word_bits = word_bits;
  f->k = k;
  f->seed = seed;
  f->nbytes = nbytes;
  f->num_bits = nbytes * 8;
  f->d_words = d_words;
  f->owns_words = false;
  if (hipGetDevice(&f->device) != hipSuccess) {
    delete f;
    return BF_EDEVICE;
  }
  *out = f;
  return BF_OK;
}

bf_status bf_destroy(bf_filter* f) {
  if (f == nullptr) return BF_OK;
  bf_status st = BF_OK;
  if (f->owns_words && f->pooled_words) {
    // released on the library stream behind the filter's last uses; the
    // host does not wait
    hipStream_t s = words_home(f->device).stream;
    st = drain_filter(f, s);
    if (st == BF_OK && hipFreeAsync(f->d_words, s) != hipSuccess) st = BF_EDEVICE;
  } else {
    st = drain_filter(f, nullptr);
    if (f->owns_words && hipFree(f->d_words) != hipSuccess) st = BF_EDEVICE;
  }
  delete f;
  return st;
}

bf_status bf_add(bf_filter* f, const uint64_t* d_keys, uint64_t n, void* stream) {
  if (f == nullptr) return BF_EINVAL;
  if (n == 0) return BF_OK;
  if (d_keys == nullptr || reinterpret_cast<uintptr_t>(d_keys) % 8 != 0) return BF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Access access = add_partitions(f, n) ? Access::kOwner : Access::kDirect;
  return ordered_call(f, s, access, [&] { return launch(f, BF_OP_ADD, d_keys, n, nullptr, stream); });
}

bf_status bf_contains(const bf_filter* f, const uint64_t* d_keys, uint64_t n, uint8_t* d_out,
                      void* stream) {
  if (f == nullptr) return BF_EINVAL;
  if (n == 0) return BF_OK;
  if (d_keys == nullptr || d_out == nullptr || reinterpret_cast<uintptr_t>(d_keys) % 8 != 0)
    return BF_EINVAL;
  bf_filter* g = const_cast<bf_filter*>(f);
  return ordered_call(g, static_cast<hipStream_t>(stream), Access::kUse,
                      [&] { return launch(g, BF_OP_CONTAINS, d_keys, n, d_out, stream); });
}

bf_status bf_clear(bf_filter* f, void* stream) {
  if (f == nullptr) return BF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return ordered_call(f, s, Access::kUse, [&] { return clear_words(f->d_words, f->nbytes, s); });
}

bf_status bf_export_words(const bf_filter* f, void* dst, uint64_t nbytes, void* stream) {
  if (f == nullptr || dst == nullptr || nbytes < f->nbytes) return BF_EINVAL;
  bf_filter* g = const_cast<bf_filter*>(f);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return ordered_call(g, s, Access::kUse, [&] {
    return hipMemcpyAsync(dst, g->d_words, g->nbytes, hipMemcpyDefault, s) == hipSuccess
               ? BF_OK
               : BF_EDEVICE;
  });
}

bf_status bf_import_words(bf_filter* f, const void* src, uint64_t nbytes, void* stream) {
  if (f == nullptr || src == nullptr || nbytes != f->nbytes) return BF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return ordered_call(f, s, Access::kUse, [&] {
    return hipMemcpyAsync(f->d_words, src, f->nbytes, hipMemcpyDefault, s) == hipSuccess
               ? BF_OK
               : BF_EDEVICE;
  });
}

bf_status bf_info(const bf_filter* f, bf_info_t* out) {
  if (f == nullptr || out == nullptr) return BF_EINVAL;
  bf_info_t i{};
  i.num_blocks = f->num_blocks;
  i.words_per_block = f->s;
  i.word_bits = f->word_bits;
  i.k = f->k;
  i.device = f->device;
  i.seed = f->seed;
  i.size_bytes = f->nbytes;
  i.d_words = f->d_words;
  i.mapping[BF_OP_ADD] = resolve_mapping(f, BF_OP_ADD, ~0ull);
  i.mapping[BF_OP_CONTAINS] = resolve_mapping(f, BF_OP_CONTAINS, ~0ull);
  i.layout = f->salts == kSaltsParquet ? BF_LAYOUT_PARQUET : f->layout;
  i.groups = f->groups;
  i.num_bits = f->num_bits;
  *out = i;
  return BF_OK;
}

bf_status bf_add_strategy(const bf_filter* f, uint64_t n, uint32_t* out) {
  if (f == nullptr || out == nullptr) return BF_EINVAL;
  *out = add_partitions(f, n) ? BF_STRATEGY_PARTITIONED : BF_STRATEGY_DIRECT;
  return BF_OK;
}

bf_status bf_tuned_mapping(int op, uint64_t num_blocks, uint32_t words_per_block,
                           uint32_t word_bits, uint32_t k, uint64_t n, bf_mapping_t* out) {
  const uint32_t s = words_per_block;
  if (out == nullptr || (op != BF_OP_ADD && op != BF_OP_CONTAINS)) return BF_EINVAL;
  if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return BF_EINVAL;
  if (!(word_bits == 32 || word_bits == 64)) return BF_EINVAL;
  if (k < s || k > static_cast<uint32_t>(kMaxK)) return BF_EINVAL;
  if (num_blocks < 1 || num_blocks > (1ull << 32)) return BF_EINVAL;
  bf_filter f{};  // host-side description only: no words
  f.layout = BF_LAYOUT_SECTORIZED;
  f.num_blocks = num_blocks;
  f.s = s;
  f.word_bits = word_bits;
  f.k = k;
  f.nbytes = num_blocks * s * (word_bits / 8);
  f.num_bits = f.nbytes * 8;
  bf_mapping_t m = resolve_mapping(&f, op, n);
  m.strategy = op == BF_OP_ADD ? (add_partitions(&f, n) ? BF_STRATEGY_PARTITIONED
                                                          : BF_STRATEGY_DIRECT)
                               : BF_STRATEGY_AUTO;
  *out = m;
  return BF_OK;
}

bf_status bf_set_mapping_ex(bf_filter* f, int op, const bf_mapping_t* m) {
  if (f == nullptr || m == nullptr) return BF_EINVAL;
  if (op != BF_OP_ADD && op != BF_OP_CONTAINS) return BF_EINVAL;
  bf_status st = validate_mapping(f, op, *m);
  if (st != BF_OK) return st;
  f->mapping[op] = *m;
  return BF_OK;
}

bf_status bf_set_mapping(bf_filter* f, int op, uint32_t lanes_per_key, uint32_t words_per_lane,
                         uint32_t keys_per_lane) {
  bf_mapping_t m{};
  m.lanes_per_key = lanes_per_key;
  m.words_per_lane = words_per_lane;
  m.keys_per_lane = keys_per_lane;
  return bf_set_mapping_ex(f, op, &m);
}

const char* bf_strerror(bf_status s) {
  switch (s) {
    case BF_OK: return "ok";
    case BF_EINVAL: return "invalid argument";
    case BF_ENOMEM: return "device allocation failed";
    case BF_EDEVICE: return "HIP runtime or launch error";
    case BF_EUNSUPPORTED: return "no kernel for this layout and mapping";
    case BF_ESCRATCH: return "the add needs more workspace than the static scratch array holds";
    default: return "unknown status";
  }
}

}  // extern "C"
