// bf_noalloc.hip -- bf_add_noalloc (include/bf.h): bf_add whose partitioned
// construction takes its workspace from a static device array instead of
// the stream-ordered pool, for callers that cannot allocate device memory.
//
// The array lives in this translation unit only, so its device code object
// (and with it the array) is loaded on a device the first time this entry
// point runs there.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/bf.h"
#include "bf_internal.hpp"

namespace {

constexpr uint64_t kScratchBytes = uint64_t{BF_NOALLOC_SCRATCH_BYTES};

// The workspace of bf_add_noalloc; one copy per device.  Host code never
// passes this name to a kernel: it is a host-side stand-in for the device
// symbol, whose device address comes from hipGetSymbolAddress.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DeviceScratch {
  void* ptr = nullptr;        // device address of `scratch` on this device
  hipEvent_t last = nullptr;  // recorded after the last call that used it
  std::mutex mu;              // held from the wait for `last` to its new record
};

std::mutex g_mu;
std::map<int, DeviceScratch> g_scratch;

// The current device's scratch: resolves the symbol's address (and creates
// the event ordering its users) the first time a device uses it.
bf_status device_scratch(int device, DeviceScratch** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch& d = g_scratch[device];
  if (d.ptr == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return BF_EDEVICE;
    }
    hipEvent_t e = bfhip::new_event();
    if (e == nullptr) return BF_EDEVICE;
    d.ptr = p;
    d.last = e;
  }
  *out = &d;
  return BF_OK;
}

}  // namespace

extern "C" bf_status bf_add_noalloc(bf_filter* f, const uint64_t* d_keys, uint64_t n, void* stream) {
  using namespace bfhip;
  if (f == nullptr) return BF_EINVAL;
  if (n == 0) return BF_OK;
  if (d_keys == nullptr || reinterpret_cast<uintptr_t>(d_keys) % 8 != 0) return BF_EINVAL;
  // a direct add uses no workspace: it is bf_add itself
  if (!add_partitions(f, n)) return bf_add(f, d_keys, n, stream);
  // one pass whose workspace fits the array, checked before anything is
  // enqueued
  const uint64_t per_key = f->layout == BF_LAYOUT_CLASSIC ? f->k : 1;
  if (n > (uint64_t{1} << 28) / per_key || partition_workspace_bytes(f, n) > kScratchBytes)
    return BF_ESCRATCH;
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device != f->device) return BF_EINVAL;
  DeviceScratch* d = nullptr;
  bf_status st = device_scratch(device, &d);
  if (st != BF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
    (void)hipGetLastError();
    cap = hipStreamCaptureStatusNone;
  }
  const bool captured = cap != hipStreamCaptureStatusNone;
  // Calls on one device share the array: each waits for the previous one
  // (outside graph capture; captured calls are ordered by their caller).
  std::lock_guard<std::mutex> lk(d->mu);
  if (!captured && hipStreamWaitEvent(s, d->last, 0) != hipSuccess) return BF_EDEVICE;
  st = ordered_call(f, s, Access::kOwner,
                    [&] { return partitioned_add_in(f, d_keys, n, s, d->ptr, kScratchBytes); });
  if (st != BF_OK) return st;
  if (!captured && hipEventRecord(d->last, s) != hipSuccess) return BF_EDEVICE;
  return BF_OK;
}
