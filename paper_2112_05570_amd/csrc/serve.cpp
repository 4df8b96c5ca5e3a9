// Request server: continuous batching of ray-walk requests over resident triangulations.
//
// Requests (a triangulation, host arrays of rays and host arrays for the results) are queued by
// server_submit. One worker thread per server runs the loop:
//   * completions: a launch slot whose event has completed hands its requests to the done queue
//     (server_poll) and returns their device memory to the pool;
//   * admission: while a slot is free, pending requests are taken in arrival order as long as
//     their device memory fits in the pool (first fit; a request that does not fit waits, and so
//     do the ones behind it) and the launch stays within max_items / max_rays; the admitted
//     requests, whatever their triangulations, go into one trace_batch launch on the slot's
//     stream, between their host-to-device and device-to-host copies.
// Requests that arrive while launches are in flight are admitted as soon as a slot and memory are
// free, so their work overlaps the launches already on the device (up to `slots` at once).
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ccsp_walk.h"
#include "walk.hpp"

namespace {

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  ccsp::set_last_error(buf);
  return code;
}

double mono_now() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Device bytes of a request of n rays: o, d, start in; prim, t, steps out.
size_t request_bytes(int64_t n) {
  const size_t m = (size_t)std::max<int64_t>(n, 1);
  return 2 * al(16 * m) + al(4 * m) + al(4 * m) + al(8 * m) + al(4 * m);
}

struct Request {
  uint64_t id = 0;
  const Triangulation* scene = nullptr;
  const double* o = nullptr;
  const double* d = nullptr;
  const int32_t* start = nullptr;
  int64_t n = 0;
  int32_t* prim = nullptr;
  double* t = nullptr;
  int32_t* steps = nullptr;
  double t_submit = 0, t_done = 0;
  int32_t status = CCSP_OK;
  size_t off = 0, bytes = 0;  // its device memory in the pool
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Request> reqs;
};

}  // namespace

struct Server {
  int device = 0;
  ServerConfig cfg{};
  unsigned char* pool = nullptr;
  std::map<size_t, size_t> free_list;  // offset -> size, disjoint and coalesced
  size_t pool_used = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::deque<Request> pending, done;
  std::thread worker;
  bool stop = false;
  uint64_t next_id = 1;
  // statistics (under mu)
  int64_t launches = 0, requests = 0, rays = 0, max_items_seen = 0, waits_for_memory = 0;
  size_t max_pool_used = 0;
  int64_t max_slots_busy = 0;
};

namespace {

bool pool_alloc(Server* s, size_t bytes, size_t* off) {
  for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
    if (it->second < bytes) continue;
    *off = it->first;
    const size_t rest = it->second - bytes, at = it->first + bytes;
    s->free_list.erase(it);
    if (rest) s->free_list.emplace(at, rest);
    s->pool_used += bytes;
    s->max_pool_used = std::max(s->max_pool_used, s->pool_used);
    return true;
  }
  return false;
}

void pool_free(Server* s, size_t off, size_t bytes) {
  auto it = s->free_list.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != s->free_list.end() && it->first + it->second == next->first) {
    it->second += next->second;
    s->free_list.erase(next);
  }
  if (it != s->free_list.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      s->free_list.erase(it);
    }
  }
  s->pool_used -= bytes;
}

// Copies in, one trace_batch over the slot's requests, copies out, completion event.
int issue(Server* s, Slot& L) {
  hipError_t e = hipSuccess;
  std::vector<TraceItem> items;
  items.reserve(L.reqs.size());
  for (Request& r : L.reqs) {
    const size_t m = (size_t)std::max<int64_t>(r.n, 1);
    unsigned char* p = s->pool + r.off;
    double* o = reinterpret_cast<double*>(p);
    double* d = reinterpret_cast<double*>(p + al(16 * m));
    int32_t* st = reinterpret_cast<int32_t*>(p + 2 * al(16 * m));
    int32_t* hp = reinterpret_cast<int32_t*>(p + 2 * al(16 * m) + al(4 * m));
    double* ht = reinterpret_cast<double*>(p + 2 * al(16 * m) + 2 * al(4 * m));
    int32_t* hs = reinterpret_cast<int32_t*>(p + 2 * al(16 * m) + 2 * al(4 * m) + al(8 * m));
    if (e == hipSuccess) e = hipMemcpyAsync(o, r.o, 16 * (size_t)r.n, hipMemcpyHostToDevice, L.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d, r.d, 16 * (size_t)r.n, hipMemcpyHostToDevice, L.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(st, r.start, 4 * (size_t)r.n, hipMemcpyHostToDevice, L.stream);
    items.push_back(TraceItem{r.scene, o, d, st, r.n, hp, ht, hs});
  }
  if (e != hipSuccess) return sfail(CCSP_E_HIP, "request upload: %s", hipGetErrorString(e));
  int rc = trace_batch(items.data(), (int32_t)items.size(), s->cfg.precision, nullptr, L.stream);
  if (rc) return sfail(rc, "trace_batch: %s", last_error());
  for (size_t k = 0; k < items.size() && e == hipSuccess; ++k) {
    const Request& r = L.reqs[k];
    const TraceItem& it = items[k];
    e = hipMemcpyAsync(r.prim, it.hit_prim, 4 * (size_t)r.n, hipMemcpyDeviceToHost, L.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r.t, it.hit_t, 8 * (size_t)r.n, hipMemcpyDeviceToHost, L.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r.steps, it.steps, 4 * (size_t)r.n, hipMemcpyDeviceToHost, L.stream);
  }
  if (e != hipSuccess) return sfail(CCSP_E_HIP, "result download: %s", hipGetErrorString(e));
  return CCSP_OK;
}

void run_worker(Server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool progress = false;
    // completions
    for (Slot& L : s->slots) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      const double now = mono_now();
      std::lock_guard<std::mutex> lk(s->mu);
      for (Request& r : L.reqs) {
        r.t_done = now;
        if (r.status == CCSP_OK && q != hipSuccess) r.status = CCSP_E_HIP;
        pool_free(s, r.off, r.bytes);
        s->done.push_back(r);
      }
      L.reqs.clear();
      L.busy = false;
      progress = true;
      s->done_cv.notify_all();
    }
    // admissions: one launch per free slot, requests in arrival order
    for (Slot& L : s->slots) {
      if (L.busy) continue;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        int64_t rays = 0;
        while (!s->pending.empty() && (int64_t)L.reqs.size() < s->cfg.max_items) {
          Request& r = s->pending.front();
          if (!L.reqs.empty() && rays + r.n > s->cfg.max_rays) break;
          size_t off = 0;
          if (!pool_alloc(s, request_bytes(r.n), &off)) {
            ++s->waits_for_memory;
            break;
          }
          r.off = off;
          r.bytes = request_bytes(r.n);
          rays += r.n;
          L.reqs.push_back(r);
          s->pending.pop_front();
        }
        if (L.reqs.empty()) break;
        ++s->launches;
        s->requests += (int64_t)L.reqs.size();
        s->rays += rays;
        s->max_items_seen = std::max<int64_t>(s->max_items_seen, (int64_t)L.reqs.size());
      }
      const int rc = issue(s, L);
      if (rc)
        for (Request& r : L.reqs) r.status = rc;
      // the event completes once everything issued above has, or at once if nothing was
      (void)hipEventRecord(L.done, L.stream);
      L.busy = true;
      progress = true;
      int64_t busy = 0;
      for (const Slot& x : s->slots) busy += x.busy;
      std::lock_guard<std::mutex> lk(s->mu);
      s->max_slots_busy = std::max(s->max_slots_busy, busy);
    }
    bool any_busy = false;
    for (const Slot& L : s->slots) any_busy |= L.busy;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->pending.empty() && !any_busy) break;
    if (!progress) {
      // poll the device often while launches are in flight, else sleep until a submission
      if (any_busy)
        s->work_cv.wait_for(lk, std::chrono::microseconds(20));
      else
        s->work_cv.wait_for(lk, std::chrono::milliseconds(5),
                            [s] { return s->stop || !s->pending.empty(); });
    }
  }
}

void release(Server* s) {
  for (Slot& L : s->slots) {
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.done) (void)hipEventDestroy(L.done);
  }
  if (s->pool) (void)hipFree(s->pool);
  delete s;
}

}  // namespace

extern "C" {

int server_create(const ServerConfig* cfg_in, Server** out) {
  ccsp::set_last_error("");
  if (!out) return sfail(CCSP_E_ARG, "null output pointer");
  *out = nullptr;
  ServerConfig cfg = cfg_in ? *cfg_in : ServerConfig{};
  if (cfg.slots == 0) cfg.slots = 4;
  if (cfg.max_items == 0) cfg.max_items = 256;
  if (cfg.max_rays == 0) cfg.max_rays = int64_t(1) << 22;
  if (cfg.memory_bytes == 0) cfg.memory_bytes = int64_t(1) << 30;
  if (cfg.slots < 1 || cfg.slots > 16) return sfail(CCSP_E_ARG, "slots %d must be 1..16", cfg.slots);
  if (cfg.max_items < 1 || cfg.max_items > 4096) return sfail(CCSP_E_ARG, "max_items %d must be 1..4096", cfg.max_items);
  if (cfg.max_rays < 1) return sfail(CCSP_E_ARG, "max_rays must be positive");
  if (cfg.memory_bytes < (int64_t(1) << 20)) return sfail(CCSP_E_ARG, "memory_bytes must be at least 1 MiB");
  const int mode = cfg.precision & CCSP_TRACE_MODE_MASK;
  if ((mode != CCSP_TRACE_FP64 && mode != CCSP_TRACE_FP32_FILTERED) || (cfg.precision & ~CCSP_TRACE_MODE_MASK))
    return sfail(CCSP_E_ARG, "precision must be a mode without flags");
  auto* s = new Server;
  s->cfg = cfg;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->pool), (size_t)cfg.memory_bytes);
  if (e != hipSuccess) {
    release(s);
    return sfail(CCSP_E_OOM, "server memory pool of %lld bytes: %s", (long long)cfg.memory_bytes,
                 hipGetErrorString(e));
  }
  s->free_list.emplace(0, (size_t)cfg.memory_bytes);
  s->slots.resize(cfg.slots);
  for (Slot& L : s->slots) {
    e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      release(s);
      return sfail(CCSP_E_HIP, "slot stream: %s", hipGetErrorString(e));
    }
  }
  s->worker = std::thread(run_worker, s);
  *out = s;
  return CCSP_OK;
}

int server_submit(Server* s, const Triangulation* scene, const double* o_xy, const double* d_xy,
                  const int32_t* start_tri, int64_t n, int32_t* hit_prim, double* hit_t,
                  int32_t* steps, uint64_t* id) {
  ccsp::set_last_error("");
  if (!s || !scene || !id) return sfail(CCSP_E_ARG, "null server, scene or id");
  if (n < 0) return sfail(CCSP_E_ARG, "negative ray count");
  if (n > 0 && (!o_xy || !d_xy || !start_tri || !hit_prim || !hit_t || !steps))
    return sfail(CCSP_E_ARG, "null ray or result array");
  if ((int64_t)request_bytes(n) > s->cfg.memory_bytes)
    return sfail(CCSP_E_ARG, "request of %lld rays needs %zu bytes, more than the server's %lld",
                 (long long)n, request_bytes(n), (long long)s->cfg.memory_bytes);
  Request r;
  r.scene = scene;
  r.o = o_xy;
  r.d = d_xy;
  r.start = start_tri;
  r.n = n;
  r.prim = hit_prim;
  r.t = hit_t;
  r.steps = steps;
  r.t_submit = mono_now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return sfail(CCSP_E_ARG, "server is shutting down");
  r.id = s->next_id++;
  *id = r.id;
  if (n == 0) {  // nothing to walk
    r.t_done = r.t_submit;
    s->done.push_back(r);
    s->done_cv.notify_all();
    return CCSP_OK;
  }
  s->pending.push_back(r);
  s->work_cv.notify_one();
  return CCSP_OK;
}

int server_poll(Server* s, int32_t max, uint64_t* ids, int32_t* status, double* t_submit,
                double* t_done, int32_t* n_out, double timeout_s) {
  ccsp::set_last_error("");
  if (!s || !n_out || max < 0 || (max > 0 && (!ids || !status || !t_submit || !t_done)))
    return sfail(CCSP_E_ARG, "bad poll arguments");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_s > 0)
    s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [s] { return !s->done.empty(); });
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    const Request& r = s->done.front();
    ids[k] = r.id;
    status[k] = r.status;
    t_submit[k] = r.t_submit;
    t_done[k] = r.t_done;
    s->done.pop_front();
    ++k;
  }
  *n_out = k;
  return CCSP_OK;
}

int server_stats(Server* s, int64_t out[8]) {
  ccsp::set_last_error("");
  if (!s || !out) return sfail(CCSP_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out[0] = s->launches;
  out[1] = s->requests;
  out[2] = s->rays;
  out[3] = s->max_items_seen;
  out[4] = (int64_t)s->max_pool_used;
  out[5] = s->waits_for_memory;
  out[6] = s->max_slots_busy;
  out[7] = (int64_t)s->pending.size();
  return CCSP_OK;
}

void server_destroy(Server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  release(s);
}

}  // extern "C"
