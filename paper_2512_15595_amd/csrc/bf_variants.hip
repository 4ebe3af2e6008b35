// bf_variants.hip -- the C ABI of include/bf_variants.h (classic,
// cache-sectorized and chained-hash layouts) and their mapping selection and launch, reached
// from bf_add / bf_contains / bf_info / bf_set_mapping of bf_api.hip.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>

#include "../../include/bf.h"
#include "../../include/bf_variants.h"
#include "bf_hash.hpp"
#include "bf_internal.hpp"
#include "bf_partition.hpp"
#include "bf_variant_kernels.hpp"
#include "bf_variant_registry.hpp"

namespace bfhip {

VariantRegistry& variant_registry() {
  static VariantRegistry r{};
  return r;
}

namespace {
std::once_flag g_variant_once;

template <int K, int KT>
void register_classic_one(VariantRegistry& r) {
  const int kidx = k_index(K);
  r.classic[classic_index(kOpAdd, kidx, KT, 0)] =
      reinterpret_cast<const void*>(&classic_add_kernel<K, false, KT>);
  r.classic[classic_index(kOpAdd, kidx, KT, 1)] =
      reinterpret_cast<const void*>(&classic_add_kernel<K, true, KT>);
  r.classic[classic_index(kOpContains, kidx, KT, 0)] =
      reinterpret_cast<const void*>(&classic_contains_kernel<K, false, KT>);
  r.classic[classic_index(kOpContains, kidx, KT, 1)] =
      reinterpret_cast<const void*>(&classic_contains_kernel<K, true, KT>);
}

template <int K>
void register_classic_kt(VariantRegistry& r) {
  register_classic_one<K, 1>(r);
  register_classic_one<K, 2>(r);
  register_classic_one<K, 4>(r);
  if constexpr (K != 0) {
    r.classic_part1[k_index(K) * 2 + 0] =
        reinterpret_cast<const void*>(&part_scatter1_classic_kernel<K, false>);
    r.classic_part1[k_index(K) * 2 + 1] =
        reinterpret_cast<const void*>(&part_scatter1_classic_kernel<K, true>);
  }
}
}  // namespace

void register_classic(VariantRegistry& r) {
  r.classic_part2 = reinterpret_cast<const void*>(&part_scatter2_kernel<uint32_t, 1, 0, -1>);
  r.classic_apply = reinterpret_cast<const void*>(&part_apply_kernel<uint32_t, 1, 0, -1>);
  register_classic_kt<0>(r);
  register_classic_kt<4>(r);
  register_classic_kt<6>(r);
  register_classic_kt<8>(r);
  register_classic_kt<12>(r);
  register_classic_kt<16>(r);
}

void ensure_variant_registry() {
  std::call_once(g_variant_once, [] {
    VariantRegistry& r = variant_registry();
    register_classic(r);
    register_chained(r);
    register_csbf_u32_s1(r);
    register_csbf_u32_s2(r);
    register_csbf_u32_s4(r);
    register_csbf_u32_s8(r);
    register_csbf_u32_s16(r);
    register_csbf_u64_s1(r);
    register_csbf_u64_s2(r);
    register_csbf_u64_s4(r);
    register_csbf_u64_s8(r);
    register_csbf_u64_s16(r);
  });
}

namespace {

bool pow2_u64(uint64_t v) { return v != 0 && (v & (v - 1)) == 0; }

int log2_u64(uint64_t v) {
  int r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

// Defaults, from a measured sweep on MI355X (filters of 1 MiB .. 1 GiB,
// every layout and mapping):
//  - classic: one key per lane for add, two for contains (all k positions of
//    both keys are in flight before any is consumed);
//  - cache-sectorized add: THETA = z, so the z group updates of one key
//    leave as one instruction and merge into one request per 64-byte
//    segment (THETA = 1 issues z requests per key: up to z times slower at
//    the atomic request rate);
//  - cache-sectorized contains: the same for blocks larger than 32 bytes
//    (THETA = z, at most 4 below the HBM size class and at most 8 in it);
//    32-byte blocks below the HBM class are fastest with THETA = 1, where the
//    z loads of a key hit one line in L2 or the Infinity Cache anyway.
bf_mapping_t default_variant_mapping(const bf_filter* f, int op) {
  bf_mapping_t m{};
  m.atomic_bits = op == BF_OP_ADD ? 32 : 0;
  if (f->layout == BF_LAYOUT_CLASSIC) {
    m.lanes_per_key = 1;
    m.words_per_lane = 1;
    m.keys_per_lane = op == BF_OP_ADD ? 1 : 2;
    return m;
  }
  if (f->layout == BF_LAYOUT_SECTORIZED_CHAINED) {
    m.lanes_per_key = 1;
    m.words_per_lane = f->s;
    m.keys_per_lane = 1;
    return m;
  }
  const uint32_t z = f->groups;
  const bool hbm = f->nbytes > (256ull << 20);
  const uint32_t block_bytes = f->s * f->word_bits / 8;
  uint32_t theta = z;
  if (op == BF_OP_CONTAINS) {
    if (block_bytes <= 32 && !hbm)
      theta = 1;
    else
      theta = z < (hbm ? 8u : 4u) ? z : (hbm ? 8u : 4u);
  }
  m.lanes_per_key = theta;
  m.words_per_lane = f->s / theta;
  m.keys_per_lane = (theta == 1 && z == 1) ? 2 : 1;
  return m;
}

bool compiled_k(const bf_filter* f) { return k_index(f->k) != 0; }

}  // namespace

bf_mapping_t variant_resolve_mapping(const bf_filter* f, int op) {
  bf_mapping_t m = f->mapping[op];
  if (m.lanes_per_key == 0 && m.words_per_lane == 0 && m.keys_per_lane == 0) {
    const uint32_t cap = m.max_workgroups;
    const uint32_t strategy = m.strategy;
    m = default_variant_mapping(f, op);
    m.max_workgroups = cap;
    m.strategy = strategy;
  }
  if (f->layout == BF_LAYOUT_CACHE_SECTORIZED) {
    if (m.lanes_per_key == 0) m.lanes_per_key = 1;
    m.words_per_lane = f->s / m.lanes_per_key;
    if (!compiled_k(f)) {
      m.lanes_per_key = 1;
      m.words_per_lane = f->s;
      m.keys_per_lane = 1;
    }
  } else if (f->layout == BF_LAYOUT_SECTORIZED_CHAINED) {
    m.lanes_per_key = 1;
    m.words_per_lane = f->s;
    m.keys_per_lane = 1;
  } else {
    m.lanes_per_key = 1;
    m.words_per_lane = 1;
  }
  if (m.keys_per_lane == 0) m.keys_per_lane = 1;
  m.atomic_bits = op == BF_OP_ADD ? 32 : 0;
  m.workgroup_threads = kBlockThreads;
  // lookups have no strategy; adds that cannot be partitioned are direct
  if (op == BF_OP_CONTAINS)
    m.strategy = BF_STRATEGY_AUTO;
  else if (!partition_applicable(f, 1))
    m.strategy = BF_STRATEGY_DIRECT;
  return m;
}

bf_status variant_validate_mapping(const bf_filter* f, int op, const bf_mapping_t& m) {
  if (m.strategy > BF_STRATEGY_PARTITIONED) return BF_EINVAL;
  if (m.strategy == BF_STRATEGY_PARTITIONED && !partition_applicable(f, 1))
    return BF_EUNSUPPORTED;
  if (op == BF_OP_CONTAINS && m.strategy != BF_STRATEGY_AUTO) return BF_EINVAL;
  if (!(m.atomic_bits == 0 || (op == BF_OP_ADD && m.atomic_bits == 32))) return BF_EINVAL;
  if (!(m.workgroup_threads == 0 || m.workgroup_threads == kBlockThreads)) return BF_EINVAL;
  if (m.lanes_per_key == 0 && m.words_per_lane == 0 && m.keys_per_lane == 0) return BF_OK;
  if (f->layout == BF_LAYOUT_SECTORIZED_CHAINED) {
    if (m.lanes_per_key != 1 || (m.words_per_lane != 0 && m.words_per_lane != f->s) ||
        m.keys_per_lane > 1)
      return BF_EINVAL;
    return BF_OK;
  }
  if (f->layout == BF_LAYOUT_CLASSIC) {
    if (m.lanes_per_key != 1 || m.words_per_lane > 1) return BF_EINVAL;
    if (!(m.keys_per_lane == 1 || m.keys_per_lane == 2 || m.keys_per_lane == 4)) return BF_EINVAL;
    return BF_OK;
  }
  const uint32_t theta = m.lanes_per_key;
  if (theta == 0 || (theta & (theta - 1)) != 0 || theta > f->groups) return BF_EINVAL;
  if (m.words_per_lane != 0 && m.words_per_lane != f->s / theta) return BF_EINVAL;
  if (!(m.keys_per_lane == 1 || (m.keys_per_lane == 2 && theta == 1))) return BF_EINVAL;
  return BF_OK;
}

bf_status variant_launch(bf_filter* f, int op, const uint64_t* keys, uint64_t n, uint8_t* out,
                         hipStream_t stream) {
  ensure_variant_registry();
  if (op == BF_OP_ADD && add_partitions(f, n)) return partitioned_add(f, keys, n, stream);
  const bf_mapping_t m = variant_resolve_mapping(f, op);
  uint32_t kt = m.keys_per_lane;
  while (kt > 1 && ((reinterpret_cast<uintptr_t>(keys) % (8u * kt)) != 0 ||
                    (out != nullptr && reinterpret_cast<uintptr_t>(out) % kt != 0)))
    kt >>= 1;
  const int kidx = k_index(f->k);

  const uint64_t tile = static_cast<uint64_t>(kBlockThreads) * kt;
  uint64_t grid = (n + tile - 1) / tile;
  const uint64_t hard_cap = 1ull << 22;  // keeps grid * 256 below 2^32
  if (grid > hard_cap) grid = hard_cap;
  if (m.max_workgroups != 0 && grid > m.max_workgroups) grid = m.max_workgroups;

  hipError_t e;
  if (f->layout == BF_LAYOUT_SECTORIZED_CHAINED) {
    const void* fn = variant_registry().chained[chained_index(
        op, static_cast<int>(f->word_bits), static_cast<int>(f->s), kidx)];
    if (fn == nullptr) return BF_EUNSUPPORTED;
    BfArgs a{};
    a.words = f->d_words;
    a.keys = keys;
    a.out = out;
    a.n = n;
    a.hash_init = xxh64_u64_init(f->seed);
    a.nb_lo = static_cast<uint32_t>(f->num_blocks);
    a.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
    a.k = f->k;
    uint64_t g = (n + kBlockThreads - 1) / kBlockThreads;
    if (g > hard_cap) g = hard_cap;
    if (m.max_workgroups != 0 && g > m.max_workgroups) g = m.max_workgroups;
    void* args[] = {&a};
    e = hipLaunchKernel(fn, dim3(static_cast<uint32_t>(g)), dim3(kBlockThreads), args, 0, stream);
  } else if (f->layout == BF_LAYOUT_CLASSIC) {
    const int pow2 = pow2_u64(f->num_bits) ? 1 : 0;
    const void* fn = variant_registry().classic[classic_index(op, kidx, static_cast<int>(kt), pow2)];
    if (fn == nullptr) return BF_EUNSUPPORTED;
    ClassicArgs a{};
    a.words = static_cast<uint32_t*>(f->d_words);
    a.keys = keys;
    a.out = out;
    a.n = n;
    a.hash_init = xxh64_u64_init(f->seed);
    a.num_bits = f->num_bits;
    a.shift = pow2 ? static_cast<uint32_t>(64 - log2_u64(f->num_bits)) : 0u;
    a.k = f->k;
    void* args[] = {&a};
    e = hipLaunchKernel(fn, dim3(static_cast<uint32_t>(grid)), dim3(kBlockThreads), args, 0,
                        stream);
  } else {
    const int theta = kidx == 0 ? 1 : static_cast<int>(m.lanes_per_key);
    if (kidx == 0) kt = 1;
    const void* fn = variant_registry().csbf[csbf_index(
        op, static_cast<int>(f->word_bits), static_cast<int>(f->s), static_cast<int>(f->groups),
        kidx, theta, static_cast<int>(kt))];
    if (fn == nullptr) return BF_EUNSUPPORTED;
    BfArgs a{};
    a.words = f->d_words;
    a.keys = keys;
    a.out = out;
    a.n = n;
    a.hash_init = xxh64_u64_init(f->seed);
    a.nb_lo = static_cast<uint32_t>(f->num_blocks);
    a.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
    a.k = f->k / f->groups;  // bits per selected word
    void* args[] = {&a};
    e = hipLaunchKernel(fn, dim3(static_cast<uint32_t>(grid)), dim3(kBlockThreads), args, 0,
                        stream);
  }
  return e == hipSuccess ? BF_OK : BF_EDEVICE;
}

}  // namespace bfhip

using namespace bfhip;

extern "C" {

bf_status bf_create_classic(uint64_t num_bits, uint32_t k, uint64_t seed, bf_filter** out) {
  if (out == nullptr) return BF_EINVAL;
  if (num_bits < 64 || num_bits % 64 != 0 || num_bits > (1ull << 40)) return BF_EINVAL;
  if (k < 1 || k > static_cast<uint32_t>(kMaxK)) return BF_EINVAL;
  bf_filter* f = new (std::nothrow) bf_filter{};
  if (f == nullptr) return BF_ENOMEM;
  f->layout = BF_LAYOUT_CLASSIC;
  f->num_blocks = 0;
  f->s = 0;
  f->word_bits = 32;
  f->k = k;
  f->seed = seed;
  f->nbytes = num_bits / 8;
  const bf_status st = alloc_filter_words(f);
  if (st != BF_OK) return st;
  *out = f;
  return BF_OK;
}

bf_status bf_create_chained(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                            uint32_t k, uint64_t seed, bf_filter** out) {
  if (out == nullptr) return BF_EINVAL;
  const uint32_t s = words_per_block;
  if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return BF_EINVAL;
  if (!(word_bits == 32 || word_bits == 64)) return BF_EINVAL;
  if (k < s || k > static_cast<uint32_t>(kMaxK)) return BF_EINVAL;
  if (num_blocks < 1 || num_blocks > (1ull << 32)) return BF_EINVAL;
  bf_filter* f = new (std::nothrow) bf_filter{};
  if (f == nullptr) return BF_ENOMEM;
  f->layout = BF_LAYOUT_SECTORIZED_CHAINED;
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

bf_status bf_create_csbf(uint64_t num_blocks, uint32_t words_per_block, uint32_t word_bits,
                         uint32_t groups, uint32_t k, uint64_t seed, bf_filter** out) {
  if (out == nullptr) return BF_EINVAL;
  const uint32_t s = words_per_block, z = groups;
  if (!(s == 1 || s == 2 || s == 4 || s == 8 || s == 16)) return BF_EINVAL;
  if (!(word_bits == 32 || word_bits == 64)) return BF_EINVAL;
  if (!(z == 1 || z == 2 || z == 4 || z == 8 || z == 16) || z > s) return BF_EINVAL;
  if (k < z || k > static_cast<uint32_t>(kMaxK) || k % z != 0) return BF_EINVAL;
  if (num_blocks < 1 || num_blocks > (1ull << 32)) return BF_EINVAL;
  bf_filter* f = new (std::nothrow) bf_filter{};
  if (f == nullptr) return BF_ENOMEM;
  f->layout = BF_LAYOUT_CACHE_SECTORIZED;
  f->num_blocks = num_blocks;
  f->s = s;
  f->word_bits = word_bits;
  f->groups = z;
  f->k = k;
  f->seed = seed;
  f->nbytes = num_blocks * s * (word_bits / 8);
  const bf_status st = alloc_filter_words(f);
  if (st != BF_OK) return st;
  *out = f;
  return BF_OK;
}

}  // extern "C"
