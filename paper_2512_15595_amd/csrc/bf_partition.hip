// bf_partition.hip -- host side of partitioned construction: geometry,
// workspace and the launch sequence (kernels in bf_partition.hpp).
#include <hip/hip_runtime.h>

#include "bf_internal.hpp"
#include "bf_partition.hpp"
#include "bf_registry.hpp"

namespace bfhip {

// ---------------------------------------------------------------------------
// hash: records in key order and per-workgroup high-digit counts
// (hist1[d * g1 + w]).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPartThreads) void part_hash_kernel(const uint64_t* keys, uint64_t* recs,
                                                                 uint32_t* hist1, PartGeometry g,
                                                                 uint64_t hash_init, uint32_t nb_lo,
                                                                 uint32_t nb_hi_mask) {
  __shared__ uint32_t cnt[kMaxDigits];
  for (uint32_t d = threadIdx.x; d < g.f1; d += kPartThreads) cnt[d] = 0;
  __syncthreads();
  const uint64_t begin = static_cast<uint64_t>(blockIdx.x) * g.range1;
  const uint64_t end = begin + g.range1 < g.n ? begin + g.range1 : g.n;
  const uint32_t shift = g.chunk_shift + g.low_bits;
  for (uint64_t i = begin + threadIdx.x; i < end; i += kPartThreads) {
    const uint64_t h = xxh64_u64(keys[i], hash_init);
    const uint32_t blk = block_of(h, nb_lo, nb_hi_mask);
    recs[i] = (static_cast<uint64_t>(blk) << 32) | static_cast<uint32_t>(h);
    atomicAdd(&cnt[blk >> shift], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < g.f1; d += kPartThreads) hist1[d * g.g1 + blockIdx.x] = cnt[d];
}

// ---------------------------------------------------------------------------
// Exclusive scan of n counts into n + 1 offsets (one workgroup of 1024).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void part_scan_kernel(const uint32_t* in, uint64_t* out, uint64_t n,
                                                        uint64_t base) {
  __shared__ uint64_t part[1024];
  const uint64_t per = (n + 1023) / 1024;
  const uint64_t b = threadIdx.x * per;
  const uint64_t e = b + per < n ? b + per : n;
  uint64_t sum = 0;
  for (uint64_t i = b; i < e; ++i) sum += in[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint64_t v = threadIdx.x >= static_cast<unsigned>(off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t run = base + (threadIdx.x ? part[threadIdx.x - 1] : 0);
  for (uint64_t i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (threadIdx.x == 1023) out[n] = base + part[1023];
}

// ---------------------------------------------------------------------------
// LDS-staged scatter of the records [begin, end) by digit
// (rec.block >> shift) & mask into dst, the workgroup's run of digit d
// starting at base[d].  Each step of kPartStep records is counting-sorted in
// LDS so that the records of one digit leave as one contiguous run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scatter_range(const uint64_t* src, uint64_t* dst, uint64_t begin,
                                              uint64_t end, uint32_t shift, uint32_t mask,
                                              uint32_t ndigits, const uint64_t* base_global,
                                              uint64_t base_stride) {
  __shared__ __attribute__((aligned(16))) uint64_t stage[kPartStep];
  __shared__ uint32_t cnt[kMaxDigits];
  __shared__ uint32_t start[kMaxDigits];
  __shared__ uint64_t next[kMaxDigits];  // next global position per digit
  for (uint32_t d = threadIdx.x; d < ndigits; d += kPartThreads) {
    next[d] = base_global[static_cast<uint64_t>(d) * base_stride];
    cnt[d] = 0;
  }
  __syncthreads();
  for (uint64_t s = begin; s < end; s += kPartStep) {
    const uint32_t valid = static_cast<uint32_t>(end - s < kPartStep ? end - s : kPartStep);
    uint64_t r[8];
    uint32_t dg[8], rank[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t p = threadIdx.x + j * kPartThreads;
      if (p < valid) {
        r[j] = src[s + p];
        dg[j] = (rec_block(r[j]) >> shift) & mask;
        rank[j] = atomicAdd(&cnt[dg[j]], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of cnt into start (digit counts are small: serial per
    // lane over a slice, then across lanes of one wave)
    if (threadIdx.x < 64) {
      const uint32_t per = (ndigits + 63) / 64;
      const uint32_t b = threadIdx.x * per;
      uint32_t sum = 0;
      for (uint32_t d = b; d < b + per && d < ndigits; ++d) sum += cnt[d];
      uint32_t incl = sum;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (threadIdx.x >= static_cast<unsigned>(off)) incl += v;
      }
      uint32_t run = incl - sum;
      for (uint32_t d = b; d < b + per && d < ndigits; ++d) {
        start[d] = run;
        run += cnt[d];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t p = threadIdx.x + j * kPartThreads;
      if (p < valid) stage[start[dg[j]] + rank[j]] = r[j];
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < valid; p += kPartThreads) {
      const uint64_t v = stage[p];
      const uint32_t d = (rec_block(v) >> shift) & mask;
      dst[next[d] + (p - start[d])] = v;
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < ndigits; d += kPartThreads) {
      next[d] += cnt[d];
      cnt[d] = 0;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kPartThreads) void part_scatter1_kernel(const uint64_t* recs, uint64_t* out,
                                                                     const uint64_t* off1,
                                                                     PartGeometry g) {
  const uint64_t begin = static_cast<uint64_t>(blockIdx.x) * g.range1;
  const uint64_t end = begin + g.range1 < g.n ? begin + g.range1 : g.n;
  scatter_range(recs, out, begin, end, g.chunk_shift + g.low_bits, 0xffffffffu, g.f1,
                off1 + blockIdx.x, g.g1);
}

// Second pass: workgroup (d1, q) takes the q-th of g.q slices of high
// digit d1's records, as placed by the first pass (bucket1[d1] = start).
__device__ __forceinline__ void slice_of(const uint64_t* bucket1, const PartGeometry& g, uint32_t d1,
                                         uint32_t q, uint64_t& b, uint64_t& e) {
  const uint64_t lo = bucket1[static_cast<uint64_t>(d1) * g.g1];
  const uint64_t hi = d1 + 1 < g.f1 ? bucket1[static_cast<uint64_t>(d1 + 1) * g.g1] : g.n;
  const uint64_t len = hi - lo;
  b = lo + len * q / g.q;
  e = lo + len * (q + 1) / g.q;
}

__global__ __launch_bounds__(kPartThreads) void part_count2_kernel(const uint64_t* recs, const uint64_t* off1,
                                                                   uint32_t* hist2, PartGeometry g) {
  __shared__ uint32_t cnt[kMaxDigits];
  const uint32_t d1 = blockIdx.x / g.q, q = blockIdx.x % g.q;
  for (uint32_t d = threadIdx.x; d < g.f2; d += kPartThreads) cnt[d] = 0;
  __syncthreads();
  uint64_t b, e;
  slice_of(off1, g, d1, q, b, e);
  const uint32_t mask = g.f2 - 1;
  for (uint64_t i = b + threadIdx.x; i < e; i += kPartThreads)
    atomicAdd(&cnt[(rec_block(recs[i]) >> g.chunk_shift) & mask], 1u);
  __syncthreads();
  // chunk-major layout: entry (chunk c = d1 * f2 + d2, slice q)
  for (uint32_t d = threadIdx.x; d < g.f2; d += kPartThreads)
    hist2[(static_cast<uint64_t>(d1) * g.f2 + d) * g.q + q] = cnt[d];
}

__global__ __launch_bounds__(kPartThreads) void part_scatter2_kernel(const uint64_t* recs, uint64_t* out,
                                                                     const uint64_t* off1,
                                                                     const uint64_t* off2,
                                                                     PartGeometry g) {
  const uint32_t d1 = blockIdx.x / g.q, q = blockIdx.x % g.q;
  uint64_t b, e;
  slice_of(off1, g, d1, q, b, e);
  scatter_range(recs, out, b, e, g.chunk_shift, g.f2 - 1, g.f2,
                off2 + static_cast<uint64_t>(d1) * g.f2 * g.q + q, g.q);
}


namespace {

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

uint32_t ceil_pow2(uint64_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct Layout {
  PartGeometry g;
  uint64_t off_a, off_b, off_hist1, off_off1, off_hist2, off_off2, total;
};

bool make_layout(const bf_filter* f, uint64_t n, Layout& L) {
  const uint64_t block_bytes = static_cast<uint64_t>(f->s) * f->word_bits / 8;
  const uint64_t bpc = kChunkBytes / block_bytes;
  uint32_t shift = 0;
  while ((1ull << shift) < bpc) ++shift;
  PartGeometry g{};
  g.n = n;
  g.chunk_shift = shift;
  g.chunks = (f->num_blocks + bpc - 1) / bpc;
  g.f2 = ceil_pow2(g.chunks) < 128 ? ceil_pow2(g.chunks) : 128;
  g.low_bits = 0;
  while ((1u << g.low_bits) < g.f2) ++g.low_bits;
  const uint64_t f1 = (g.chunks + g.f2 - 1) / g.f2;
  if (f1 > static_cast<uint64_t>(kMaxDigits)) return false;
  g.f1 = static_cast<uint32_t>(f1);
  uint64_t range = (n + 1023) / 1024;
  range = (range + kPartStep - 1) / kPartStep * kPartStep;
  if (range < static_cast<uint64_t>(kPartStep)) range = kPartStep;
  g.range1 = range;
  g.g1 = static_cast<uint32_t>((n + range - 1) / range);
  uint64_t q = (n + static_cast<uint64_t>(g.f1) * 65536 - 1) / (static_cast<uint64_t>(g.f1) * 65536);
  g.q = static_cast<uint32_t>(q < 1 ? 1 : (q > 32 ? 32 : q));
  L.g = g;
  uint64_t off = 0;
  L.off_a = off;
  off = align256(off + 8 * n);
  L.off_b = off;
  off = align256(off + 8 * n);
  L.off_hist1 = off;
  off = align256(off + 4ull * g.f1 * g.g1);
  L.off_off1 = off;
  off = align256(off + 8ull * (static_cast<uint64_t>(g.f1) * g.g1 + 1));
  L.off_hist2 = off;
  off = align256(off + 4ull * g.f1 * g.f2 * g.q);
  L.off_off2 = off;
  off = align256(off + 8ull * (static_cast<uint64_t>(g.f1) * g.f2 * g.q + 1));
  L.total = off;
  return true;
}

}  // namespace

bool partition_applicable(const bf_filter* f, uint64_t n) {
  Layout L;
  return n > 0 && make_layout(f, 1, L) && n < (1ull << 40);
}

bf_status partitioned_add(bf_filter* f, const uint64_t* keys, uint64_t n, hipStream_t stream) {
  Layout L;
  if (!make_layout(f, n, L)) return BF_EUNSUPPORTED;
  ensure_registry();
  const void* apply = registry().apply_fn[batch_index(0, static_cast<int>(f->word_bits),
                                                      static_cast<int>(f->s), k_index(f->k))];
  if (apply == nullptr) return BF_EUNSUPPORTED;
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
  uint64_t* a = reinterpret_cast<uint64_t*>(base + L.off_a);
  uint64_t* b = reinterpret_cast<uint64_t*>(base + L.off_b);
  uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.off_hist1);
  uint64_t* off1 = reinterpret_cast<uint64_t*>(base + L.off_off1);
  uint32_t* hist2 = reinterpret_cast<uint32_t*>(base + L.off_hist2);
  uint64_t* off2 = reinterpret_cast<uint64_t*>(base + L.off_off2);
  const PartGeometry g = L.g;
  const uint64_t hash_init = xxh64_u64_init(f->seed);
  const uint32_t nb_lo = static_cast<uint32_t>(f->num_blocks);
  const uint32_t nb_hi = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
  const dim3 blk(kPartThreads);

  hipLaunchKernelGGL(part_hash_kernel, dim3(g.g1), blk, 0, stream, keys, a, hist1, g, hash_init,
                     nb_lo, nb_hi);
  hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, stream, hist1, off1,
                     static_cast<uint64_t>(g.f1) * g.g1, 0ull);
  hipLaunchKernelGGL(part_scatter1_kernel, dim3(g.g1), blk, 0, stream, a, b, off1, g);
  hipLaunchKernelGGL(part_count2_kernel, dim3(g.f1 * g.q), blk, 0, stream, b, off1, hist2, g);
  hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, stream, hist2, off2,
                     static_cast<uint64_t>(g.f1) * g.f2 * g.q, 0ull);
  hipLaunchKernelGGL(part_scatter2_kernel, dim3(g.f1 * g.q), blk, 0, stream, b, a, off1, off2, g);
  void* words = f->d_words;
  uint64_t nblocks = f->num_blocks;
  const uint64_t* recs = a;
  const uint64_t* o2 = off2;
  PartGeometry gg = g;
  uint32_t k = f->k;
  void* args[] = {&words, &nblocks, &recs, &o2, &gg, &k};
  const uint64_t grid = g.chunks < 65535 ? g.chunks : 65535;
  if (hipLaunchKernel(apply, dim3(static_cast<uint32_t>(grid)), blk, args, 0, stream) != hipSuccess)
    return BF_EDEVICE;
  return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

}  // namespace bfhip
