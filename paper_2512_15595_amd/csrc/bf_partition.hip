// bf_partition.hip -- host side of partitioned construction: geometry,
// bucket capacities, workspace and the launch sequence (kernels in
// bf_partition.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bf_internal.hpp"
#include "bf_partition.hpp"
#include "bf_registry.hpp"

namespace bfhip {

namespace {

__global__ __launch_bounds__(kPartThreads) void part_zero_kernel(unsigned long long* p, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kPartThreads;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kPartThreads + threadIdx.x; i < n; i += stride)
    p[i] = 0;
}

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

struct Layout {
  PartArgs a;
  uint64_t off_buf1, off_buf2, off_fill, nfill, total;
};

bool make_layout(const bf_filter* f, uint64_t n, Layout& L) {
  const uint64_t block_bytes = static_cast<uint64_t>(f->s) * f->word_bits / 8;
  const uint64_t bpc = kChunkBytes / block_bytes;
  PartArgs a{};
  while ((1ull << a.chunk_shift) < bpc) ++a.chunk_shift;
  a.chunks = (f->num_blocks + bpc - 1) / bpc;
  a.f2 = ceil_pow2(a.chunks) < 128 ? ceil_pow2(a.chunks) : 128;
  while ((1u << a.low_bits) < a.f2) ++a.low_bits;
  const uint64_t f1 = (a.chunks + a.f2 - 1) / a.f2;
  if (f1 > static_cast<uint64_t>(kMaxDigits)) return false;
  a.f1 = static_cast<uint32_t>(f1);
  a.n = n;
  uint64_t range = (n + 1023) / 1024;
  range = (range + kPartStep - 1) / kPartStep * kPartStep;
  a.range1 = std::max<uint64_t>(range, kPartStep);
  // chunk buckets are filled uniformly (the last chunk may be partial)
  a.cap1 = capacity(static_cast<double>(n) / a.f1, 4 * kPartStep, 64);
  a.cap2 = capacity(static_cast<double>(n) / a.chunks, 64, 16);
  const uint64_t per_bucket = std::min<uint64_t>(a.cap1, n);
  uint64_t q = (per_bucket + 65535) / 65536;
  a.q = static_cast<uint32_t>(std::clamp<uint64_t>(q, 1, 32));
  L.a = a;
  uint64_t off = 0;
  L.off_buf1 = off;
  off = align256(off + 8ull * a.f1 * a.cap1);
  L.off_buf2 = off;
  off = align256(off + 8ull * a.chunks * a.cap2);
  L.off_fill = off;
  L.nfill = a.f1 + a.chunks;
  off = align256(off + 8ull * L.nfill);
  L.total = off;
  return true;
}

}  // namespace

bool partition_applicable(const bf_filter* f, uint64_t n) {
  Layout L;
  return n > 0 && n < (1ull << 40) && make_layout(f, 1, L);
}

bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream) {
  Layout L;
  if (!make_layout(f, n, L)) return BF_EUNSUPPORTED;
  ensure_registry();
  const int idx = batch_index(0, static_cast<int>(f->word_bits), static_cast<int>(f->s),
                              k_index(f->k));
  const void* k1 = registry().part1_fn[idx];
  const void* k2 = registry().part2_fn[idx];
  const void* k3 = registry().apply_fn[idx];
  if (k1 == nullptr || k2 == nullptr || k3 == nullptr) return BF_EUNSUPPORTED;
  if (f->scratch_bytes < L.total) {
    if (f->scratch != nullptr) {
      if (hipFree(f->scratch) != hipSuccess) return BF_EDEVICE;
      f->scratch = nullptr;
      f->scratch_bytes = 0;
    }
    if (hipMalloc(&f->scratch, L.total) != hipSuccess) {
      (void)hipGetLastError();
      f->scratch = nullptr;
      return BF_ENOMEM;
    }
    f->scratch_bytes = L.total;
  }
  uint8_t* base = static_cast<uint8_t*>(f->scratch);
  PartArgs a = L.a;
  a.words = f->d_words;
  a.num_blocks = f->num_blocks;
  a.hash_init = xxh64_u64_init(f->seed);
  a.nb_lo = static_cast<uint32_t>(f->num_blocks);
  a.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
  a.k = f->k;
  a.keys = keys;
  a.buf1 = reinterpret_cast<uint64_t*>(base + L.off_buf1);
  a.buf2 = reinterpret_cast<uint64_t*>(base + L.off_buf2);
  a.fill1 = reinterpret_cast<unsigned long long*>(base + L.off_fill);
  a.fill2 = a.fill1 + a.f1;

  const uint64_t zgrid = std::min<uint64_t>((L.nfill + kPartThreads - 1) / kPartThreads, 4096);
  hipLaunchKernelGGL(part_zero_kernel, dim3(static_cast<uint32_t>(std::max<uint64_t>(zgrid, 1))),
                     dim3(kPartThreads), 0, stream, a.fill1, L.nfill);
  void* args[] = {&a};
  const uint64_t g1 = (n + a.range1 - 1) / a.range1;
  const uint64_t g3 = std::min<uint64_t>(a.chunks, 65535);
  if (hipLaunchKernel(k1, dim3(static_cast<uint32_t>(g1)), dim3(kPartThreads), args, 0, stream) !=
          hipSuccess ||
      hipLaunchKernel(k2, dim3(a.f1 * a.q), dim3(kPartThreads), args, 0, stream) != hipSuccess ||
      hipLaunchKernel(k3, dim3(static_cast<uint32_t>(g3)), dim3(kApplyThreads), args, 0, stream) !=
          hipSuccess)
    return BF_EDEVICE;
  return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

}  // namespace bfhip
