// gather_bench.hip -- random-access roofline microbenchmarks (C ABI in
// include/bf_bench.h).
//
// The paper measures the DRAM bound of a blocked filter with random 64-bit
// loads and stores in giga-updates per second (GUPS) and reports filter
// throughput as a fraction of it (Sec. V-B).  These kernels measure the
// same kind of bound on gfx950, at the access shapes the filter kernels use:
//   - random aligned segment reads of 4..128 bytes, addresses from an
//     in-register hash (no index stream) or from an index array (8 bytes
//     streamed per access, one result byte written per access: the shape of
//     a lookup);
//   - random aligned segment atomic ORs, the segment covered by one lane
//     (sequential 64-bit atomics) or by several lanes (one each);
//   - GUPS: random 64-bit load, xor, store;
//   - a streaming copy, used to calibrate hardware byte counters.
// Each thread performs kAccessPerThread independent accesses so that enough
// requests are in flight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bf_bench.h"

namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kAccessPerThread = 4;

// Integer mixer (a 32-bit avalanche hash); any uniform-enough hash serves.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint64_t segment_of(uint64_t i, uint32_t seed, uint32_t nseg_lo,
                                               uint32_t nseg_hi_mask) {
  const uint32_t h = mix32(static_cast<uint32_t>(i) ^ mix32(static_cast<uint32_t>(i >> 32) + seed));
  return __umulhi(h, nseg_lo) + (h & nseg_hi_mask);
}

// XOR of SEG/LANES bytes at p (16 / 8 / 4-byte loads).
template <int BYTES>
__device__ __forceinline__ uint32_t load_xor(const uint8_t* p) {
  if constexpr (BYTES >= 16) {
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < BYTES / 16; ++i) {
      u32x4 v = reinterpret_cast<const u32x4*>(p)[i];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    return acc;
  } else if constexpr (BYTES == 8) {
    u32x2 v = *reinterpret_cast<const u32x2*>(p);
    return v.x ^ v.y;
  } else {
    return *reinterpret_cast<const uint32_t*>(p);
  }
}

template <int SEG, int LANES>
__global__ __launch_bounds__(kThreads) void random_read_kernel(const uint8_t* buf, uint64_t n_access,
                                                               uint32_t nseg_lo, uint32_t nseg_hi_mask,
                                                               uint32_t seed, uint32_t* sink) {
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t group = tid / LANES;
  const uint32_t rank = threadIdx.x % LANES;
  const uint64_t groups = static_cast<uint64_t>(gridDim.x) * kThreads / LANES;
  uint32_t acc = 0;
#pragma unroll
  for (int r = 0; r < kAccessPerThread; ++r) {
    const uint64_t a = group + static_cast<uint64_t>(r) * groups;
    if (a < n_access) {
      const uint64_t seg = segment_of(a, seed, nseg_lo, nseg_hi_mask);
      acc ^= load_xor<SEG / LANES>(buf + seg * SEG + rank * (SEG / LANES));
    }
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;  // practically never; keeps the loads
}

// Eight independent 16-byte loads with an explicit cache policy, all issued
// before one wait in the same asm block (so the eight are in flight
// together, as the compiler keeps the plain loads of random_read_kernel):
// 2 = sc1 (system coherence scope), 3 = sc0 sc1, 4 = nt sc1.  Outputs are
// early-clobber, so no load overwrites an address another load still needs.
#define BFB_LOAD8_POLICY(FLAGS)                                                  \
  asm volatile("global_load_dwordx4 %0, %8, off " FLAGS "\n\t"                   \
               "global_load_dwordx4 %1, %9, off " FLAGS "\n\t"                   \
               "global_load_dwordx4 %2, %10, off " FLAGS "\n\t"                  \
               "global_load_dwordx4 %3, %11, off " FLAGS "\n\t"                  \
               "global_load_dwordx4 %4, %12, off " FLAGS "\n\t"                  \
               "global_load_dwordx4 %5, %13, off " FLAGS "\n\t"                  \
               "global_load_dwordx4 %6, %14, off " FLAGS "\n\t"                  \
               "global_load_dwordx4 %7, %15, off " FLAGS "\n\t"                  \
               "s_waitcnt vmcnt(0)"                                              \
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), \
                 "=&v"(v[5]), "=&v"(v[6]), "=&v"(v[7])                           \
               : "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3]), "v"(p[4]), "v"(p[5]), \
                 "v"(p[6]), "v"(p[7])                                            \
               : "memory")

// 1 = nontemporal hint (the compiler's own loads, scheduled freely).
template <int POL>
__device__ __forceinline__ void load8_policy(const uint8_t* const (&p)[8], u32x4 (&v)[8]) {
  if constexpr (POL == 1) {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p[i]));
  } else if constexpr (POL == 2) {
    BFB_LOAD8_POLICY("sc1");
  } else if constexpr (POL == 3) {
    BFB_LOAD8_POLICY("sc0 sc1");
  } else {
    BFB_LOAD8_POLICY("nt sc1");
  }
}

// Random SEG-byte reads (one lane per segment) with cache policy POL: the
// thread's kAccessPerThread segments are read as 16-byte pieces, eight
// pieces in flight at a time.  An access past n_access reads segment 0 (in
// bounds; its value only feeds the sink test).
template <int SEG, int POL>
__global__ __launch_bounds__(kThreads) void random_read_policy_kernel(const uint8_t* buf,
                                                                      uint64_t n_access,
                                                                      uint32_t nseg_lo,
                                                                      uint32_t nseg_hi_mask,
                                                                      uint32_t seed, uint32_t* sink) {
  static_assert(SEG % 16 == 0 && (kAccessPerThread * SEG / 16) % 8 == 0, "whole groups of 8 pieces");
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t threads = static_cast<uint64_t>(gridDim.x) * kThreads;
  const uint8_t* base[kAccessPerThread];
#pragma unroll
  for (int r = 0; r < kAccessPerThread; ++r) {
    const uint64_t a = tid + static_cast<uint64_t>(r) * threads;
    base[r] = buf + (a < n_access ? segment_of(a, seed, nseg_lo, nseg_hi_mask) : 0) * SEG;
  }
  constexpr int kPieces = SEG / 16;
  uint32_t acc = 0;
#pragma unroll
  for (int g = 0; g < kAccessPerThread * kPieces / 8; ++g) {
    const uint8_t* p[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) p[i] = base[(g * 8 + i) / kPieces] + 16 * ((g * 8 + i) % kPieces);
    u32x4 v[8];
    load8_policy<POL>(p, v);
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= v[i].x ^ v[i].y ^ v[i].z ^ v[i].w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;
}

template <int SEG>
__global__ __launch_bounds__(kThreads) void random_read_indexed_kernel(const uint8_t* buf,
                                                                       uint64_t nseg,
                                                                       const uint64_t* idx,
                                                                       uint64_t n, uint8_t* out) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
  for (uint64_t j = i; j < n; j += stride) {
    const uint64_t seg = idx[j];
    // an index outside the buffer reads nothing (result 0)
    out[j] = seg < nseg ? static_cast<uint8_t>(load_xor<SEG>(buf + seg * SEG) & 1u) : 0;
  }
}

__global__ __launch_bounds__(kThreads) void fill_index_kernel(uint64_t* idx, uint64_t n,
                                                              uint32_t nseg_lo, uint32_t nseg_hi_mask,
                                                              uint32_t seed) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
  for (uint64_t j = i; j < n; j += stride) idx[j] = segment_of(j, seed, nseg_lo, nseg_hi_mask);
}

template <int SEG, int LANES>
__global__ __launch_bounds__(kThreads) void random_atomic_kernel(uint8_t* buf, uint64_t n_access,
                                                                 uint32_t nseg_lo,
                                                                 uint32_t nseg_hi_mask,
                                                                 uint32_t seed) {
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t group = tid / LANES;
  const uint32_t rank = threadIdx.x % LANES;
  const uint64_t groups = static_cast<uint64_t>(gridDim.x) * kThreads / LANES;
  constexpr int kBytesPerLane = SEG / LANES;
#pragma unroll
  for (int r = 0; r < kAccessPerThread; ++r) {
    const uint64_t a = group + static_cast<uint64_t>(r) * groups;
    if (a < n_access) {
      const uint64_t seg = segment_of(a, seed, nseg_lo, nseg_hi_mask);
      uint8_t* p = buf + seg * SEG + rank * kBytesPerLane;
      if constexpr (kBytesPerLane == 4) {
        __hip_atomic_fetch_or(reinterpret_cast<uint32_t*>(p), 1u << (a & 31), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      } else {
#pragma unroll
        for (int w = 0; w < kBytesPerLane / 8; ++w)
          __hip_atomic_fetch_or(reinterpret_cast<uint64_t*>(p) + w, 1ull << ((a + w) & 63),
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void gups_kernel(uint64_t* buf, uint64_t n_updates,
                                                        uint32_t nword_lo, uint32_t nword_hi_mask,
                                                        uint32_t seed) {
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t threads = static_cast<uint64_t>(gridDim.x) * kThreads;
#pragma unroll
  for (int r = 0; r < kAccessPerThread; ++r) {
    const uint64_t a = tid + static_cast<uint64_t>(r) * threads;
    if (a < n_updates) {
      const uint64_t w = segment_of(a, seed, nword_lo, nword_hi_mask);
      buf[w] ^= a;
    }
  }
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): element i of stream `seed`
// is the output function applied to seed + (i + 1) * 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kThreads) void splitmix_kernel(uint64_t* out, uint64_t n, uint64_t seed,
                                                            uint64_t first) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride)
    out[i] = splitmix64_at(seed, first + i);
}

// Query i: with probability hit_q32 / 2^32 element j of the source stream
// (j uniform in [src_first, src_first + src_count)), else element
// fresh_first + i of the fresh stream; the choice and j come from element i
// of the mix stream.
__global__ __launch_bounds__(kThreads) void mixed_query_kernel(uint64_t* out, uint64_t n,
                                                               uint64_t src_seed, uint64_t src_first,
                                                               uint32_t src_count,
                                                               uint64_t fresh_seed,
                                                               uint64_t fresh_first,
                                                               uint32_t hit_q32, uint64_t mix_seed) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const uint64_t r = splitmix64_at(mix_seed, i);
    const uint32_t choose = static_cast<uint32_t>(r >> 32);
    const uint32_t pick = __umulhi(static_cast<uint32_t>(r), src_count);
    out[i] = choose < hit_q32 ? splitmix64_at(src_seed, src_first + pick)
                              : splitmix64_at(fresh_seed, fresh_first + i);
  }
}

__global__ __launch_bounds__(kThreads) void copy_kernel(u32x4* dst, const u32x4* src, uint64_t nvec) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
  for (uint64_t j = i; j < nvec; j += stride) dst[j] = src[j];
}

bool split_count(uint64_t count, uint32_t* lo, uint32_t* hi_mask) {
  if (count == 0 || count > (1ull << 32)) return false;
  *lo = static_cast<uint32_t>(count);
  *hi_mask = (count >> 32) ? 0xffffffffu : 0u;
  return true;
}

uint32_t grid_for(uint64_t threads_needed) {
  uint64_t g = (threads_needed + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > (1ull << 22)) g = 1ull << 22;
  return static_cast<uint32_t>(g);
}

template <int SEG, int LANES>
int launch_read(const void* buf, uint64_t nseg, uint64_t n_access, uint32_t seed, uint32_t* sink,
                hipStream_t s) {
  uint32_t lo, him;
  if (!split_count(nseg, &lo, &him)) return BFB_EINVAL;
  const uint64_t groups = (n_access + kAccessPerThread - 1) / kAccessPerThread;
  if (groups * LANES > (1ull << 22) * kThreads) return BFB_EINVAL;
  hipLaunchKernelGGL((random_read_kernel<SEG, LANES>), dim3(grid_for(groups * LANES)), dim3(kThreads),
                     0, s, static_cast<const uint8_t*>(buf), n_access, lo, him, seed, sink);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

template <int SEG, int LANES>
int launch_atomic(void* buf, uint64_t nseg, uint64_t n_access, uint32_t seed, hipStream_t s) {
  uint32_t lo, him;
  if (!split_count(nseg, &lo, &him)) return BFB_EINVAL;
  const uint64_t groups = (n_access + kAccessPerThread - 1) / kAccessPerThread;
  if (groups * LANES > (1ull << 22) * kThreads) return BFB_EINVAL;
  hipLaunchKernelGGL((random_atomic_kernel<SEG, LANES>), dim3(grid_for(groups * LANES)),
                     dim3(kThreads), 0, s, static_cast<uint8_t*>(buf), n_access, lo, him, seed);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

}  // namespace

extern "C" {

int bfb_random_read(const void* d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                    uint32_t lanes_per_seg, uint64_t n_access, uint32_t seed, uint32_t* d_sink,
                    void* stream) {
  if (d_buf == nullptr || d_sink == nullptr || seg_bytes == 0) return BFB_EINVAL;
  if (n_access == 0) return BFB_OK;
  const uint64_t nseg = buf_bytes / seg_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t key = (static_cast<uint64_t>(seg_bytes) << 8) | lanes_per_seg;
  switch (key) {
    case (4ull << 8) | 1: return launch_read<4, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (8ull << 8) | 1: return launch_read<8, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (16ull << 8) | 1: return launch_read<16, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (32ull << 8) | 1: return launch_read<32, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (32ull << 8) | 2: return launch_read<32, 2>(d_buf, nseg, n_access, seed, d_sink, s);
    case (64ull << 8) | 1: return launch_read<64, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (64ull << 8) | 4: return launch_read<64, 4>(d_buf, nseg, n_access, seed, d_sink, s);
    case (128ull << 8) | 1: return launch_read<128, 1>(d_buf, nseg, n_access, seed, d_sink, s);
    case (128ull << 8) | 8: return launch_read<128, 8>(d_buf, nseg, n_access, seed, d_sink, s);
    default: return BFB_EINVAL;
  }
}

int bfb_random_read_policy(const void* d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                           uint32_t policy, uint64_t n_access, uint32_t seed, uint32_t* d_sink,
                           void* stream) {
  if (d_buf == nullptr || d_sink == nullptr || (seg_bytes != 32 && seg_bytes != 128)) return BFB_EINVAL;
  if (policy < 1 || policy > 4) return BFB_EINVAL;
  if (n_access == 0) return BFB_OK;
  uint32_t lo, him;
  if (!split_count(buf_bytes / seg_bytes, &lo, &him)) return BFB_EINVAL;
  const uint64_t threads = (n_access + kAccessPerThread - 1) / kAccessPerThread;
  if (threads > (1ull << 22) * kThreads) return BFB_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(grid_for(threads)), block(kThreads);
  const uint8_t* b = static_cast<const uint8_t*>(d_buf);
  const uint32_t key = seg_bytes * 10 + policy;
  switch (key) {
    case 321: hipLaunchKernelGGL((random_read_policy_kernel<32, 1>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 322: hipLaunchKernelGGL((random_read_policy_kernel<32, 2>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 323: hipLaunchKernelGGL((random_read_policy_kernel<32, 3>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 324: hipLaunchKernelGGL((random_read_policy_kernel<32, 4>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 1281: hipLaunchKernelGGL((random_read_policy_kernel<128, 1>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 1282: hipLaunchKernelGGL((random_read_policy_kernel<128, 2>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 1283: hipLaunchKernelGGL((random_read_policy_kernel<128, 3>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    case 1284: hipLaunchKernelGGL((random_read_policy_kernel<128, 4>), grid, block, 0, s, b, n_access, lo, him, seed, d_sink); break;
    default: return BFB_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_fill_random_index(uint64_t* d_idx, uint64_t n, uint64_t nseg, uint32_t seed, void* stream) {
  uint32_t lo, him;
  if (d_idx == nullptr || !split_count(nseg, &lo, &him)) return BFB_EINVAL;
  if (n == 0) return BFB_OK;
  hipLaunchKernelGGL(fill_index_kernel, dim3(grid_for(n < (1u << 24) ? n : (1u << 24))),
                     dim3(kThreads), 0, static_cast<hipStream_t>(stream), d_idx, n, lo, him, seed);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_random_read_indexed(const void* d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                            const uint64_t* d_idx, uint64_t n, uint8_t* d_out, void* stream) {
  if (d_buf == nullptr || d_idx == nullptr || d_out == nullptr) return BFB_EINVAL;
  if (seg_bytes == 0 || buf_bytes / seg_bytes == 0) return BFB_EINVAL;
  if (n == 0) return BFB_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t grid = grid_for(n);
  const uint8_t* b = static_cast<const uint8_t*>(d_buf);
  const uint64_t ns = buf_bytes / seg_bytes;
  switch (seg_bytes) {
    case 8: hipLaunchKernelGGL(random_read_indexed_kernel<8>, dim3(grid), dim3(kThreads), 0, s, b, ns, d_idx, n, d_out); break;
    case 16: hipLaunchKernelGGL(random_read_indexed_kernel<16>, dim3(grid), dim3(kThreads), 0, s, b, ns, d_idx, n, d_out); break;
    case 32: hipLaunchKernelGGL(random_read_indexed_kernel<32>, dim3(grid), dim3(kThreads), 0, s, b, ns, d_idx, n, d_out); break;
    case 64: hipLaunchKernelGGL(random_read_indexed_kernel<64>, dim3(grid), dim3(kThreads), 0, s, b, ns, d_idx, n, d_out); break;
    case 128: hipLaunchKernelGGL(random_read_indexed_kernel<128>, dim3(grid), dim3(kThreads), 0, s, b, ns, d_idx, n, d_out); break;
    default: return BFB_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_random_atomic_or(void* d_buf, uint64_t buf_bytes, uint32_t seg_bytes,
                         uint32_t lanes_per_seg, uint64_t n_access, uint32_t seed, void* stream) {
  if (d_buf == nullptr || seg_bytes == 0) return BFB_EINVAL;
  if (n_access == 0) return BFB_OK;
  const uint64_t nseg = buf_bytes / seg_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t key = (static_cast<uint64_t>(seg_bytes) << 8) | lanes_per_seg;
  switch (key) {
    case (4ull << 8) | 1: return launch_atomic<4, 1>(d_buf, nseg, n_access, seed, s);
    case (8ull << 8) | 1: return launch_atomic<8, 1>(d_buf, nseg, n_access, seed, s);
    case (32ull << 8) | 1: return launch_atomic<32, 1>(d_buf, nseg, n_access, seed, s);
    case (32ull << 8) | 4: return launch_atomic<32, 4>(d_buf, nseg, n_access, seed, s);
    case (32ull << 8) | 8: return launch_atomic<32, 8>(d_buf, nseg, n_access, seed, s);
    case (64ull << 8) | 8: return launch_atomic<64, 8>(d_buf, nseg, n_access, seed, s);
    case (128ull << 8) | 16: return launch_atomic<128, 16>(d_buf, nseg, n_access, seed, s);
    default: return BFB_EINVAL;
  }
}

int bfb_gups(void* d_buf, uint64_t buf_bytes, uint64_t n_updates, uint32_t seed, void* stream) {
  uint32_t lo, him;
  if (d_buf == nullptr || !split_count(buf_bytes / 8, &lo, &him)) return BFB_EINVAL;
  if (n_updates == 0) return BFB_OK;
  const uint64_t threads = (n_updates + kAccessPerThread - 1) / kAccessPerThread;
  if (threads > (1ull << 22) * kThreads) return BFB_EINVAL;
  hipLaunchKernelGGL(gups_kernel, dim3(grid_for(threads)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), static_cast<uint64_t*>(d_buf), n_updates, lo,
                     him, seed);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_fill_splitmix64(uint64_t* d_out, uint64_t n, uint64_t seed, uint64_t first, void* stream) {
  if (d_out == nullptr) return BFB_EINVAL;
  if (n == 0) return BFB_OK;
  hipLaunchKernelGGL(splitmix_kernel, dim3(grid_for(n < (1u << 24) ? n : (1u << 24))), dim3(kThreads),
                     0, static_cast<hipStream_t>(stream), d_out, n, seed, first);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_fill_mixed_queries(uint64_t* d_out, uint64_t n, uint64_t src_seed, uint64_t src_first,
                           uint32_t src_count, uint64_t fresh_seed, uint64_t fresh_first,
                           uint32_t hit_q32, uint64_t mix_seed, void* stream) {
  if (d_out == nullptr || src_count == 0) return BFB_EINVAL;
  if (n == 0) return BFB_OK;
  hipLaunchKernelGGL(mixed_query_kernel, dim3(grid_for(n < (1u << 24) ? n : (1u << 24))),
                     dim3(kThreads), 0, static_cast<hipStream_t>(stream), d_out, n, src_seed,
                     src_first, src_count, fresh_seed, fresh_first, hit_q32, mix_seed);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

int bfb_copy(void* d_dst, const void* d_src, uint64_t bytes, void* stream) {
  if (d_dst == nullptr || d_src == nullptr || bytes % 16 != 0) return BFB_EINVAL;
  if (bytes == 0) return BFB_OK;
  const uint64_t nvec = bytes / 16;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(nvec < (1u << 24) ? nvec : (1u << 24))),
                     dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                     static_cast<u32x4*>(d_dst), static_cast<const u32x4*>(d_src), nvec);
  return hipGetLastError() == hipSuccess ? BFB_OK : BFB_EDEVICE;
}

}  // extern "C"
