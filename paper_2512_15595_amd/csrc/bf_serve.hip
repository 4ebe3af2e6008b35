// bf_serve.hip -- the request loop of include/bf_serve.h: a scheduler thread
// doing FIFO admission by HBM budget and launch slots, per-filter ordering
// by events, a stream pool, and coalescing of small requests into one
// launch of the persistent batched kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/bf_serve.h"
#include "bf_batch_kernels.hpp"
#include "bf_internal.hpp"
#include "bf_registry.hpp"
#include "bf_tuned.hpp"

using namespace bfhip;

namespace {

uint64_t now_ns() {
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now().time_since_epoch())
                                   .count());
}

struct Pending {
  uint64_t id;
  bf_request_t r;
  uint64_t arrival;  // absolute steady-clock ns
  uint64_t bytes;
};

struct LaunchRec {
  hipEvent_t done;
  uint32_t index;
  uint64_t bytes;
  std::vector<uint64_t> ids;
  std::vector<uint32_t> filters;
};

struct FilterDeps {
  std::vector<hipEvent_t> adds;   // in-flight launches adding to the filter
  std::vector<hipEvent_t> reads;  // in-flight launches reading it
};

struct StreamCtx {
  hipStream_t s = nullptr;
  BatchFilter* d_desc = nullptr;
  BatchTile* d_tiles = nullptr;
  BatchFilter* h_desc = nullptr;  // pinned staging
  BatchTile* h_tiles = nullptr;
  hipEvent_t staged = nullptr;    // recorded after the last copy out of the staging
  bool staged_valid = false;
};

// Device bytes a request holds while in flight: its keys and results and,
// for an add that will take the partitioned construction, the workspace it
// takes from the device pool.
uint64_t payload_bytes(const bf_filter* f, const bf_request_t& r) {
  if (r.op == BF_OP_CONTAINS) return r.n * 9ull;
  uint64_t bytes = r.n * 8ull;
  if (add_partitions(f, r.n)) bytes += partition_workspace_bytes(f, r.n);
  return bytes;
}

}  // namespace

struct bf_server {
  std::vector<bf_filter*> filters;
  bf_server_config_t cfg{};
  int device = 0;
  int cus = 256;
  const void* batch_fn[2] = {nullptr, nullptr};
  std::vector<StreamCtx> streams;
  uint32_t next_stream = 0;

  std::thread worker;
  std::atomic<bool> stop{false};
  std::mutex mu;
  std::condition_variable cv_inbox;
  std::condition_variable cv_done;
  std::deque<Pending> inbox;                  // guarded by mu
  std::vector<bf_request_result_t> results;   // guarded by mu, indexed by id
  uint64_t submitted = 0;                     // guarded by mu
  uint64_t completed = 0;                     // guarded by mu
  bf_server_stats_t stats{};                  // guarded by mu
  uint64_t t0 = 0;

  // scheduler-thread state
  std::deque<Pending> pending;
  std::vector<LaunchRec> inflight;
  std::vector<FilterDeps> deps;
  std::vector<hipEvent_t> event_pool;
  uint64_t inflight_bytes = 0;
  uint32_t launch_counter = 0;
};

namespace {

hipEvent_t get_event(bf_server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

bool coalescable(const bf_server* s, const Pending& p) {
  return s->cfg.coalesce_max_keys > 0 && p.r.n <= s->cfg.coalesce_max_keys &&
         s->cfg.coalesce_max_requests > 1;
}

// The mapping a coalesced launch runs a request's tiles with: the batched
// kernel's (large-batch rows at the filter's k, 256-thread tiles).
MapSpec request_map(const bf_filter* f, int op) {
  if (k_index(f->k) == 0) return MapSpec{1, f->s, 1, 32, 0, kBlockThreads, true};
  return tuned_map(op, static_cast<int>(f->word_bits), static_cast<int>(f->s),
                   size_class_of(f->nbytes), static_cast<int>(f->k), 1);
}

uint64_t tiles_of(const bf_filter* f, const Pending& p) {
  const uint64_t tile = static_cast<uint64_t>(kBlockThreads) * request_map(f, p.r.op).kt;
  return (p.r.n + tile - 1) / tile;
}

void finish_request(bf_server* s, uint64_t id, uint64_t admit, uint64_t complete, uint32_t launch,
                    int32_t status, uint64_t arrival) {
  bf_request_result_t& res = s->results[id];
  res.arrival_ns = arrival;
  res.admit_ns = admit;
  res.complete_ns = complete;
  res.launch = launch;
  res.status = status;
  s->completed += 1;
}

// Enqueues one launch for a group of requests (same op; one request, or
// several coalesced ones).  Returns false if the HIP runtime refused.
bool launch_group(bf_server* s, const std::vector<Pending>& group, uint64_t group_bytes) {
  StreamCtx& sc = s->streams[s->next_stream++ % s->streams.size()];
  const int op = static_cast<int>(group[0].r.op);
  // dependencies: contains after earlier adds; add after earlier contains
  // and earlier adds (a partitioned add owns its filter while it runs)
  std::vector<hipEvent_t> waits;
  auto wait_on = [&waits](const std::vector<hipEvent_t>& src) {
    for (hipEvent_t e : src)
      if (std::find(waits.begin(), waits.end(), e) == waits.end()) waits.push_back(e);
  };
  for (const Pending& p : group) {
    const FilterDeps& d = s->deps[p.r.filter];
    wait_on(d.adds);
    if (op == BF_OP_ADD) wait_on(d.reads);
  }
  for (hipEvent_t e : waits)
    if (hipStreamWaitEvent(sc.s, e, 0) != hipSuccess) return false;

  bf_status st = BF_OK;
  if (group.size() == 1) {
    const bf_request_t& r = group[0].r;
    bf_filter* f = s->filters[r.filter];
    // the server orders its filters' work itself (the waits above)
    st = launch_unordered(f, op, r.d_keys, r.n, op == BF_OP_CONTAINS ? r.d_out : nullptr, sc.s);
  } else {
    if (sc.staged_valid && hipEventSynchronize(sc.staged) != hipSuccess) return false;
    uint64_t ntiles = 0;
    for (size_t i = 0; i < group.size(); ++i) {
      const bf_request_t& r = group[i].r;
      const bf_filter* f = s->filters[r.filter];
      BatchFilter& d = sc.h_desc[i];
      d.words = f->d_words;
      d.hash_init = xxh64_u64_init(f->seed);
      d.nb_lo = static_cast<uint32_t>(f->num_blocks);
      d.nb_hi_mask = (f->num_blocks >> 32) ? 0xffffffffu : 0u;
      d.keys = r.d_keys;
      d.out = r.d_out;
      d.reserved = 0;
      const int cls = size_class_of(f->nbytes);
      const uint32_t kt = request_map(f, op).kt;
      const uint64_t tile = static_cast<uint64_t>(kBlockThreads) * kt;
      for (uint64_t off = 0; off < r.n; off += tile) {
        const uint32_t count = static_cast<uint32_t>(std::min<uint64_t>(tile, r.n - off));
        const bool vec = count == tile &&
                         (reinterpret_cast<uintptr_t>(r.d_keys + off) % (8u * kt)) == 0 &&
                         (r.d_out == nullptr ||
                          (reinterpret_cast<uintptr_t>(r.d_out + off) % kt) == 0);
        BatchTile& t = sc.h_tiles[ntiles++];
        t.key_start = off;
        t.filter = static_cast<uint32_t>(i);
        t.meta = count | (static_cast<uint32_t>(cls) << kTileClassShift) | (vec ? kTileVecBit : 0u);
      }
    }
    if (hipMemcpyAsync(sc.d_desc, sc.h_desc, group.size() * sizeof(BatchFilter),
                       hipMemcpyHostToDevice, sc.s) != hipSuccess ||
        hipMemcpyAsync(sc.d_tiles, sc.h_tiles, ntiles * sizeof(BatchTile), hipMemcpyHostToDevice,
                       sc.s) != hipSuccess ||
        hipEventRecord(sc.staged, sc.s) != hipSuccess)
      return false;
    sc.staged_valid = true;
    BatchArgs a{};
    a.filters = sc.d_desc;
    a.tiles = sc.d_tiles;
    a.ntiles = ntiles;
    a.k = s->filters[group[0].r.filter]->k;
    void* kargs[] = {&a};
    const uint64_t grid = std::min<uint64_t>(ntiles, static_cast<uint64_t>(s->cus) * 8);
    if (hipLaunchKernel(s->batch_fn[op], dim3(static_cast<uint32_t>(grid)), dim3(kBlockThreads),
                        kargs, 0, sc.s) != hipSuccess)
      return false;
  }
  if (st != BF_OK) return false;
  hipEvent_t ev = get_event(s);
  if (ev == nullptr || hipEventRecord(ev, sc.s) != hipSuccess) return false;

  LaunchRec rec;
  rec.done = ev;
  rec.index = s->launch_counter++;
  rec.bytes = group_bytes;
  const uint64_t admit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (const Pending& p : group) {
      rec.ids.push_back(p.id);
      s->results[p.id].admit_ns = admit;
      s->results[p.id].launch = rec.index;
    }
    s->stats.launches += 1;
    if (group.size() > 1) s->stats.coalesced_launches += 1;
  }
  for (const Pending& p : group) {
    FilterDeps& d = s->deps[p.r.filter];
    std::vector<hipEvent_t>& dst = op == BF_OP_ADD ? d.adds : d.reads;
    if (std::find(dst.begin(), dst.end(), ev) == dst.end()) dst.push_back(ev);
    if (std::find(rec.filters.begin(), rec.filters.end(), p.r.filter) == rec.filters.end())
      rec.filters.push_back(p.r.filter);
  }
  s->inflight_bytes += group_bytes;
  s->inflight.push_back(std::move(rec));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.peak_inflight_bytes = std::max(s->stats.peak_inflight_bytes, s->inflight_bytes);
    s->stats.peak_inflight_launches =
        std::max<uint64_t>(s->stats.peak_inflight_launches, s->inflight.size());
  }
  return true;
}

// Retires finished launches; returns true if any finished.
bool retire(bf_server* s) {
  bool any = false;
  for (size_t i = 0; i < s->inflight.size();) {
    LaunchRec& L = s->inflight[i];
    hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    const uint64_t t = now_ns();
    const int32_t status = q == hipSuccess ? BF_OK : BF_EDEVICE;
    for (uint32_t f : L.filters) {
      FilterDeps& d = s->deps[f];
      d.adds.erase(std::remove(d.adds.begin(), d.adds.end(), L.done), d.adds.end());
      d.reads.erase(std::remove(d.reads.begin(), d.reads.end(), L.done), d.reads.end());
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (uint64_t id : L.ids) {
        bf_request_result_t& r = s->results[id];
        r.complete_ns = t;
        r.status = status;
        s->completed += 1;
      }
    }
    s->inflight_bytes -= L.bytes;
    s->event_pool.push_back(L.done);
    s->inflight.erase(s->inflight.begin() + static_cast<std::ptrdiff_t>(i));
    any = true;
  }
  if (any) s->cv_done.notify_all();
  return any;
}

bool admit(bf_server* s) {
  bool any = false;
  while (!s->pending.empty()) {
    const Pending& head = s->pending.front();
    if (head.bytes > s->cfg.hbm_budget_bytes) {  // can never fit: refuse it
      std::lock_guard<std::mutex> lk(s->mu);
      finish_request(s, head.id, now_ns(), now_ns(), 0xffffffffu, BF_ENOMEM,
                     s->results[head.id].arrival_ns);
      s->pending.pop_front();
      s->cv_done.notify_all();
      any = true;
      continue;
    }
    if (s->inflight.size() >= s->cfg.max_inflight ||
        s->inflight_bytes + head.bytes > s->cfg.hbm_budget_bytes)
      break;
    std::vector<Pending> group{head};
    uint64_t bytes = head.bytes;
    if (coalescable(s, head)) {
      uint64_t tiles = tiles_of(s->filters[head.r.filter], head);
      for (size_t j = 1; j < s->pending.size() && group.size() < s->cfg.coalesce_max_requests;
           ++j) {
        const Pending& p = s->pending[j];
        if (p.r.op != head.r.op || !coalescable(s, p)) break;
        const uint64_t t = tiles_of(s->filters[p.r.filter], p);
        if (tiles + t > s->cfg.coalesce_max_tiles ||
            s->inflight_bytes + bytes + p.bytes > s->cfg.hbm_budget_bytes)
          break;
        tiles += t;
        bytes += p.bytes;
        group.push_back(p);
      }
    }
    if (!launch_group(s, group, bytes)) {
      std::lock_guard<std::mutex> lk(s->mu);
      for (const Pending& p : group)
        finish_request(s, p.id, now_ns(), now_ns(), 0xffffffffu, BF_EDEVICE,
                       s->results[p.id].arrival_ns);
      s->cv_done.notify_all();
    }
    for (size_t j = 0; j < group.size(); ++j) s->pending.pop_front();
    any = true;
  }
  return any;
}

void worker_main(bf_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->inbox.empty() && s->pending.empty() && s->inflight.empty()) {
        if (s->stop.load()) break;
        s->cv_inbox.wait_for(lk, std::chrono::milliseconds(5));
      }
      while (!s->inbox.empty()) {
        s->pending.push_back(s->inbox.front());
        s->inbox.pop_front();
      }
    }
    const bool a = retire(s);
    const bool b = admit(s);
    if (!a && !b) std::this_thread::yield();
  }
}

bool valid_request(const bf_server* s, const bf_request_t& r) {
  if (r.op != BF_OP_ADD && r.op != BF_OP_CONTAINS) return false;
  if (r.filter >= s->filters.size() || r.n == 0 || r.d_keys == nullptr) return false;
  if (reinterpret_cast<uintptr_t>(r.d_keys) % 8 != 0) return false;
  if (r.op == BF_OP_CONTAINS && r.d_out == nullptr) return false;
  return true;
}

uint64_t submit_at(bf_server* s, const bf_request_t& r, uint64_t arrival) {
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t id = s->submitted++;
  s->results.resize(s->submitted);
  s->results[id] = bf_request_result_t{arrival, 0, 0, 0xffffffffu, BF_OK};
  s->inbox.push_back(Pending{id, r, arrival, payload_bytes(s->filters[r.filter], r)});
  s->stats.requests += 1;
  s->cv_inbox.notify_one();
  return id;
}

void wait_all(bf_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->completed == s->submitted; });
}

void destroy_streams(bf_server* s) {
  for (StreamCtx& sc : s->streams) {
    if (sc.s) (void)hipStreamSynchronize(sc.s);
    if (sc.staged) (void)hipEventDestroy(sc.staged);
    if (sc.d_desc) (void)hipFree(sc.d_desc);
    if (sc.d_tiles) (void)hipFree(sc.d_tiles);
    if (sc.h_desc) (void)hipHostFree(sc.h_desc);
    if (sc.h_tiles) (void)hipHostFree(sc.h_tiles);
    if (sc.s) (void)hipStreamDestroy(sc.s);
  }
  s->streams.clear();
}

}  // namespace

extern "C" {

bf_status bf_server_create(bf_filter* const* filters, uint32_t nfilters,
                           const bf_server_config_t* cfg, bf_server** out) {
  if (out == nullptr || filters == nullptr || nfilters == 0) return BF_EINVAL;
  const bf_filter* f0 = filters[0];
  if (f0 == nullptr) return BF_EINVAL;
  for (uint32_t i = 0; i < nfilters; ++i) {
    const bf_filter* f = filters[i];
    if (f != nullptr && f->layout != BF_LAYOUT_SECTORIZED) return BF_EUNSUPPORTED;
    if (f == nullptr || f->s != f0->s || f->word_bits != f0->word_bits || f->k != f0->k ||
        f->device != f0->device || f->salts != f0->salts)
      return BF_EINVAL;
  }
  bf_server_config_t c{};
  if (cfg != nullptr) {
    c = *cfg;
  } else {
    c.hbm_budget_bytes = 16ull << 30;
    c.max_inflight = 16;
    c.nstreams = 8;
    c.coalesce_max_keys = 65536;
    c.coalesce_max_requests = 256;
    c.coalesce_max_tiles = 16384;
  }
  if (c.hbm_budget_bytes == 0 || c.max_inflight == 0 || c.nstreams == 0 || c.nstreams > 64)
    return BF_EINVAL;
  if (c.coalesce_max_keys > 0 && (c.coalesce_max_requests == 0 || c.coalesce_max_tiles == 0))
    return BF_EINVAL;

  const Registry& reg = kernel_table(f0->salts == kSaltsParquet);
  bf_server* s = new (std::nothrow) bf_server();
  if (s == nullptr) return BF_ENOMEM;
  s->filters.assign(filters, filters + nfilters);
  s->cfg = c;
  s->device = f0->device;
  s->deps.resize(nfilters);
  for (int op = 0; op < 2; ++op)
    s->batch_fn[op] = reg.batch_fn[batch_index(op, static_cast<int>(f0->word_bits),
                                                      static_cast<int>(f0->s), k_index(f0->k))];
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, s->device) == hipSuccess && prop.multiProcessorCount > 0)
    s->cus = prop.multiProcessorCount;
  s->streams.resize(c.nstreams);
  const uint32_t nreq = std::max<uint32_t>(1, c.coalesce_max_requests);
  const uint32_t ntile = std::max<uint32_t>(1, c.coalesce_max_tiles);
  for (StreamCtx& sc : s->streams) {
    if (hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sc.staged, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&sc.d_desc, nreq * sizeof(BatchFilter)) != hipSuccess ||
        hipMalloc(&sc.d_tiles, ntile * sizeof(BatchTile)) != hipSuccess ||
        hipHostMalloc(&sc.h_desc, nreq * sizeof(BatchFilter), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&sc.h_tiles, ntile * sizeof(BatchTile), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      destroy_streams(s);
      delete s;
      return BF_ENOMEM;
    }
  }
  s->t0 = now_ns();
  s->worker = std::thread(worker_main, s);
  *out = s;
  return BF_OK;
}

bf_status bf_server_submit(bf_server* s, const bf_request_t* req, uint64_t* id) {
  if (s == nullptr || req == nullptr || id == nullptr || !valid_request(s, *req)) return BF_EINVAL;
  *id = submit_at(s, *req, now_ns());
  return BF_OK;
}

bf_status bf_server_wait(bf_server* s, const uint64_t* ids, uint64_t count,
                         bf_request_result_t* results) {
  if (s == nullptr || (count > 0 && (ids == nullptr || results == nullptr))) return BF_EINVAL;
  wait_all(s);
  std::lock_guard<std::mutex> lk(s->mu);
  for (uint64_t i = 0; i < count; ++i) {
    if (ids[i] >= s->submitted) return BF_EINVAL;
    bf_request_result_t r = s->results[ids[i]];
    r.arrival_ns -= s->t0;
    r.admit_ns = r.admit_ns ? r.admit_ns - s->t0 : 0;
    r.complete_ns = r.complete_ns ? r.complete_ns - s->t0 : 0;
    results[i] = r;
  }
  return BF_OK;
}

bf_status bf_server_replay(bf_server* s, const bf_request_t* reqs, uint64_t nreq,
                           bf_request_result_t* results) {
  if (s == nullptr || (nreq > 0 && (reqs == nullptr || results == nullptr))) return BF_EINVAL;
  for (uint64_t i = 0; i < nreq; ++i)
    if (!valid_request(s, reqs[i])) return BF_EINVAL;
  wait_all(s);  // start from an idle server
  std::vector<uint64_t> ids(nreq);
  const uint64_t start = now_ns();
  for (uint64_t i = 0; i < nreq; ++i) {
    const uint64_t due = start + reqs[i].arrival_ns;
    while (now_ns() < due) {
      // spin close to the due time, sleep when far from it
      if (due - now_ns() > 200000) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    ids[i] = submit_at(s, reqs[i], due);
  }
  wait_all(s);
  std::lock_guard<std::mutex> lk(s->mu);
  for (uint64_t i = 0; i < nreq; ++i) {
    bf_request_result_t r = s->results[ids[i]];
    r.arrival_ns -= start;
    r.admit_ns = r.admit_ns ? r.admit_ns - start : 0;
    r.complete_ns = r.complete_ns ? r.complete_ns - start : 0;
    results[i] = r;
  }
  return BF_OK;
}

bf_status bf_server_replay_serial(bf_server* s, const bf_request_t* reqs, uint64_t nreq,
                                  bf_request_result_t* results) {
  if (s == nullptr || (nreq > 0 && (reqs == nullptr || results == nullptr))) return BF_EINVAL;
  for (uint64_t i = 0; i < nreq; ++i)
    if (!valid_request(s, reqs[i])) return BF_EINVAL;
  wait_all(s);
  (void)hipSetDevice(s->device);
  hipStream_t st = s->streams[0].s;
  const uint64_t start = now_ns();
  for (uint64_t i = 0; i < nreq; ++i) {
    const bf_request_t& r = reqs[i];
    const uint64_t due = start + r.arrival_ns;
    while (now_ns() < due) {
      if (due - now_ns() > 200000) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    const uint64_t admit = now_ns();
    bf_filter* f = s->filters[r.filter];
    bf_status rc = launch_unordered(f, static_cast<int>(r.op), r.d_keys, r.n,
                                    r.op == BF_OP_CONTAINS ? r.d_out : nullptr, st);
    if (rc == BF_OK && hipStreamSynchronize(st) != hipSuccess) rc = BF_EDEVICE;
    results[i] = bf_request_result_t{r.arrival_ns, admit - start, now_ns() - start,
                                     static_cast<uint32_t>(i), rc};
  }
  return BF_OK;
}

bf_status bf_server_stats(const bf_server* s, bf_server_stats_t* out) {
  if (s == nullptr || out == nullptr) return BF_EINVAL;
  std::lock_guard<std::mutex> lk(const_cast<bf_server*>(s)->mu);
  *out = s->stats;
  return BF_OK;
}

bf_status bf_server_destroy(bf_server* s) {
  if (s == nullptr) return BF_OK;
  wait_all(s);
  s->stop.store(true);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_inbox.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  destroy_streams(s);
  delete s;
  return BF_OK;
}

}  // extern "C"
