// C ABI of the triangulation walk: load (validate, pack, upload), trace, batch, counters.
//
// Packing for the walk (paper Sec. 5.1 needs, per visited triangle, the exit decision and the
// neighbour across the chosen edge): every (triangle, edge) slot stores the exit word and the one
// vertex the next step tests, so a step is a single dependent 16-byte (binary32) or 32-byte
// (binary64) load. Memory is traded for latency: a 4M-triangle scene takes ~0.7 GB of HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <array>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ccsp_walk.h"
#include "exact.hpp"
#include "walk.hpp"

using namespace ccsp;

struct Triangulation {
  int device = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  SceneDev dev{};
  int64_t nv = 0, nt = 0, np = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace ccsp {
void set_last_error(const char* msg) { g_err = msg; }
}  // namespace ccsp

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(CCSP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

template <class F>
void parallel_for(int64_t n, F&& f) {
  const int hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nth = n < 65536 ? 1 : hw;
  if (nth == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nth - 1) / nth;
  for (int k = 0; k < nth; ++k) {
    const int64_t a = k * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back([&f, a, b] { f(a, b); });
  }
  for (auto& t : th) t.join();
}

// host orientation: binary64 filter (Shewchuk's bound (3+16u)u for this evaluation), then exact
int orient_host(const double* a, const double* b, const double* c) {
  const double l = (b[0] - a[0]) * (c[1] - a[1]);
  const double r = (b[1] - a[1]) * (c[0] - a[0]);
  const double det = l - r, sum = std::fabs(l) + std::fabs(r);
  if (std::fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return orient_exact(a[0], a[1], b[0], b[1], c[0], c[1]);
}

// Position of (x, y) along the Hilbert curve of a 2^16 x 2^16 grid.
uint32_t hilbert16(uint32_t x, uint32_t y) {
  uint32_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = 0xffffu - x;
        y = 0xffffu - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Events of one timed trace: start of the trace, start and end of the walk kernel, end of the
// trace (after the copy of parked results, if any).
struct StageEvents {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
constexpr int kTimeSlots = 256;

struct TableSlot {
  void* p = nullptr;
  hipEvent_t free_ev = nullptr;
  bool used = false;
};
constexpr int kTableSlots = 16;

struct BatchGraph {
  hipGraphExec_t exec = nullptr;
  BatchItem* dev = nullptr;             // its item table (the upload before each replay fills it)
  unsigned long long* counter = nullptr;
  hipEvent_t done = nullptr;            // after its last replay
  hipStream_t last = nullptr;
  bool used = false;
};

struct DeviceState {
  bool init = false;
  int cus = 0;
  Workspace ws{};
  std::atomic<unsigned> next_counter{0};
  // trace_batch item tables: a ring of pinned host tables and a ring of device tables, each
  // with an event after which it may be reused (host: its upload is done; device: the launch
  // that read it is done), so that batches on different streams never share a live table
  std::mutex mu;
  std::vector<TableSlot> host_ring, dev_ring;
  int items_cap = 0;
  unsigned ring_next = 0;
  // captured batch launches, by everything the capture bakes in; each owns its device table
  // and tile counters
  std::map<std::array<int64_t, 10>, BatchGraph> graphs;
  // ray binning scratch, shared by the traces on this device
  std::mutex bin_mu;
  void* bin_ws = nullptr;
  size_t bin_ws_bytes = 0;
  hipEvent_t bin_free = nullptr;
  hipStream_t bin_last_stream = nullptr;
  // stage timing (CCSP_TRACE_TIMED): a ring of the last kTimeSlots timed traces
  std::mutex time_mu;
  std::vector<StageEvents> tev;
  int time_next = 0, time_count = 0;
  // launch parameters chosen by autotune() (or set with tune_cache_set), by workload shape
  std::mutex tune_mu;
  std::unordered_map<uint64_t, TuneParams> tuned;
};

std::mutex g_dev_mu;
DeviceState g_dev[64];

int device_state(DeviceState** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(CCSP_E_HIP, "device index %d unsupported", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceState& s = g_dev[dev];
  if (!s.init) {
    e = hipDeviceGetAttribute(&s.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    void* p = nullptr;
    const size_t bytes = sizeof(unsigned long long) * (kCounterSlots + 4) +
                         sizeof(int) * (kCounterSlots / kClaimChunks);
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(CCSP_E_OOM, "workspace allocation failed: %s", hipGetErrorString(e));
    e = hipMemset(p, 0, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMemset");
    s.ws.counters = static_cast<unsigned long long*>(p);
    s.ws.stats = s.ws.counters + kCounterSlots;
    s.ws.errflags = reinterpret_cast<int*>(s.ws.stats + 4);
    e = hipEventCreateWithFlags(&s.bin_free, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    s.init = true;
  }
  *out = &s;
  return CCSP_OK;
}

// Binning pays only when the scene does not fit the caches anyway and there are enough rays.
constexpr int64_t kBinMinRays = 1 << 16;
constexpr int64_t kBinMinTriangles = 1 << 18;

// Tile counters (and validation flag) of the next eager launch: a ring of kCounterSlots /
// kClaimChunks groups, so that launches in flight on different streams never share (captured
// graphs have their own).
unsigned long long* next_counters(DeviceState* ds, int** errflag = nullptr) {
  const unsigned groups = kCounterSlots / kClaimChunks;
  const unsigned g = ds->next_counter.fetch_add(1) % groups;
  if (errflag) *errflag = ds->ws.errflags + g;
  return ds->ws.counters + (size_t)g * kClaimChunks;
}

// Grow the per-device ray binning scratch to hold n rays (allocates only when n exceeds every
// earlier size; reserve_workspace() does it ahead of time). Caller holds ds->bin_mu.
int grow_bin_workspace(DeviceState* ds, int64_t n) {
  const size_t need = bin_workspace_bytes(n);
  if (need <= ds->bin_ws_bytes) return CCSP_OK;
  hipError_t e;
  if (ds->bin_ws) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(ds->bin_ws);
    ds->bin_ws = nullptr;
    ds->bin_ws_bytes = 0;
  }
  e = hipMalloc(&ds->bin_ws, need);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "ray binning scratch of %zu bytes: %s", need, hipGetErrorString(e));
  ds->bin_ws_bytes = need;
  return CCSP_OK;
}

// Shape of a workload for the tuning cache: item count, total rays and total triangles rounded
// up to powers of two, precision mode, graph replay, input order, and whether it is a single
// trace (trace_rays) or a batch.
uint64_t tune_key(int64_t n_items, int64_t rays, int64_t tris, int precision, bool single) {
  auto lg = [](int64_t v) {
    int b = 0;
    while (b < 62 && (int64_t(1) << b) < v) ++b;
    return (uint64_t)b;
  };
  return lg(n_items) | lg(rays) << 8 | lg(tris) << 16 |
         (uint64_t)(precision & CCSP_TRACE_MODE_MASK) << 24 |
         (uint64_t)((precision & CCSP_TRACE_GRAPH) != 0) << 32 | (uint64_t)single << 33 |
         (uint64_t)((precision & CCSP_TRACE_INPUT_ORDER) != 0) << 34;
}

bool tune_lookup(DeviceState* ds, uint64_t key, TuneParams* out) {
  std::lock_guard<std::mutex> lk(ds->tune_mu);
  auto it = ds->tuned.find(key);
  if (it == ds->tuned.end()) return false;
  *out = it->second;
  return true;
}

// The next record of the timing ring (its events are created on the first timed trace).
int timing_slot(DeviceState* ds, StageEvents** out) {
  std::lock_guard<std::mutex> lk(ds->time_mu);
  if (ds->tev.empty()) {
    std::vector<StageEvents> v(kTimeSlots);
    for (auto& s : v)
      for (auto& ev : s.ev) {
        const hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
          for (auto& s2 : v)
            for (auto& ev2 : s2.ev)
              if (ev2) (void)hipEventDestroy(ev2);
          return hip_fail(e, "hipEventCreate");
        }
      }
    ds->tev.swap(v);
  }
  *out = &ds->tev[ds->time_next];
  ds->time_next = (ds->time_next + 1) % kTimeSlots;
  ds->time_count = std::min(ds->time_count + 1, kTimeSlots);
  return CCSP_OK;
}

// Grow the trace_batch item tables to hold n_items (first call, or a batch larger than any
// before); waits for the device first, since the old tables may still be read. Caller holds
// ds->mu.
int grow_item_tables(DeviceState* ds, int n_items) {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  int cap = 256;
  while (cap < n_items) cap *= 2;
  ds->items_cap = 0;
  ds->host_ring.resize(kTableSlots);
  ds->dev_ring.resize(kTableSlots);
  for (int k = 0; k < kTableSlots; ++k) {
    TableSlot& h = ds->host_ring[k];
    TableSlot& d = ds->dev_ring[k];
    if (h.p) (void)hipHostFree(h.p);
    if (d.p) (void)hipFree(d.p);
    h.p = d.p = nullptr;
    h.used = d.used = false;
    for (TableSlot* s : {&h, &d})
      if (!s->free_ev) {
        e = hipEventCreateWithFlags(&s->free_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      }
    e = hipHostMalloc(&h.p, sizeof(BatchItem) * cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(CCSP_E_OOM, "pinned item table allocation failed");
    e = hipMalloc(&d.p, sizeof(BatchItem) * cap);
    if (e != hipSuccess) return fail(CCSP_E_OOM, "item table allocation failed");
  }
  ds->items_cap = cap;
  return CCSP_OK;
}

// Capture (reset, walk) of a batch of n_items items and `tiles` tiles into a graph with
// its own item table and tile counters.
int capture_batch_graph(DeviceState* ds, int n_items, int64_t tiles, int mode, bool count,
                        const LaunchCfg& cfg, BatchGraph* g) {
  auto cleanup = [g] {
    if (g->dev) (void)hipFree(g->dev);
    if (g->counter) (void)hipFree(g->counter);
    if (g->done) (void)hipEventDestroy(g->done);
    *g = BatchGraph{};
  };
  hipError_t e = hipMalloc(&g->dev, sizeof(BatchItem) * n_items);
  if (e == hipSuccess) e = hipMalloc(&g->counter, sizeof(unsigned long long) * kClaimChunks);
  if (e != hipSuccess) {
    cleanup();
    return fail(CCSP_E_OOM, "graph item table allocation failed");
  }
  e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipEventCreate");
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "capture stream");
  }
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  hipError_t e2 = hipSuccess, e3 = hipSuccess;
  if (e == hipSuccess) {
    e2 = launch_walk_batch(g->dev, n_items, tiles, mode, count, cfg, g->counter, ds->ws, cs);
    e3 = hipStreamEndCapture(cs, &graph);
  }
  (void)hipStreamDestroy(cs);
  if (e == hipSuccess) e = e2 != hipSuccess ? e2 : e3;
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "graph capture");
  }
  return CCSP_OK;
}

LaunchCfg make_cfg(int cus, int mode, const TuneParams* tp) {
  LaunchCfg c{};
  c.wg = (tp && tp->wg_size) ? tp->wg_size : 256;
  c.tile = (tp && tp->tile_rays) ? tp->tile_rays : (mode == 1 ? 64 : 64);
  const int wpcu = (tp && tp->waves_per_cu) ? tp->waves_per_cu : 24;
  c.refill_min = (tp && tp->refill_min) ? tp->refill_min : 16;
  c.grid = std::max(1, cus * wpcu / (c.wg / 64));
  c.chunks = (tp && tp->xcd_chunks) ? tp->xcd_chunks : kClaimChunks;
  c.group = (tp && tp->tiles_per_claim) ? tp->tiles_per_claim : 4;
  return c;
}

int check_tune(const TuneParams* tp) {
  if (!tp) return CCSP_OK;
  if (tp->wg_size < 0 || tp->tile_rays < 0 || tp->waves_per_cu < 0 || tp->refill_min < 0 ||
      tp->tiles_per_claim < 0 || tp->xcd_chunks < 0)
    return fail(CCSP_E_ARG, "negative tuning field");
  if (tp->waves_per_cu > 64) return fail(CCSP_E_ARG, "waves_per_cu %d must be at most 64", tp->waves_per_cu);
  if (tp->bin < 0 || tp->bin > 2) return fail(CCSP_E_ARG, "bin %d must be 0, 1 or 2", tp->bin);
  if (tp->step_limit < 0) return fail(CCSP_E_ARG, "negative step_limit");
  return CCSP_OK;
}

int check_cfg(const LaunchCfg& c) {
  if (c.wg < 64 || c.wg > 512 || c.wg % 64) return fail(CCSP_E_ARG, "wg_size %d must be 64..512, multiple of 64", c.wg);
  if (c.tile != 64 && c.tile != 128 && c.tile != 256) return fail(CCSP_E_ARG, "tile_rays %d must be 64, 128 or 256", c.tile);
  if (c.refill_min < 1 || c.refill_min > 64) return fail(CCSP_E_ARG, "refill_min %d must be 1..64", c.refill_min);
  if (c.group < 1 || c.group > 4096) return fail(CCSP_E_ARG, "tiles_per_claim %d must be 1..4096", c.group);
  if (c.chunks != 1 && c.chunks != kClaimChunks) return fail(CCSP_E_ARG, "xcd_chunks %d must be 1 or 8", c.chunks);
  return CCSP_OK;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

// ------------------------------------------------------------------ trace without allocation
//
// trace_rays_static keeps all of its device scratch (the tile counters of its launch and the ray
// binning records) in one file-scope device array per GPU, whose address is looked up once per
// device; it never calls hipMalloc or anything that allocates.
constexpr size_t kStaticScratchBytes = size_t(80) << 20;
constexpr size_t kStaticBinOffset = 256;  // counters (8 x 8 B) and unused stats before the bins
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

struct StaticScratch {
  bool init = false;
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  int cus = 0;
};
std::mutex g_static_mu;
StaticScratch g_static[64];

// The current device's copy of `scratch`: looked up with the device current on its first call
// (the array's host-side name is not a device address).
int static_scratch(StaticScratch** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(CCSP_E_HIP, "device index %d unsupported", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticScratch& s = g_static[dev];
  if (!s.init) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    e = hipDeviceGetAttribute(&s.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    if (bin_workspace_bytes(CCSP_STATIC_MAX_RAYS) > kStaticScratchBytes - kStaticBinOffset)
      return fail(CCSP_E_HIP, "static scratch of %zu bytes too small for %d binned rays",
                  kStaticScratchBytes, CCSP_STATIC_MAX_RAYS);
    s.ptr = static_cast<unsigned char*>(p);
    s.init = true;
  }
  *out = &s;
  return CCSP_OK;
}

}  // namespace

extern "C" {

const char* last_error(void) { return g_err.c_str(); }

int load_triangulation(const TriangulationDesc* desc, void* stream, Triangulation** out) {
  g_err.clear();
  if (!desc || !out) return fail(CCSP_E_ARG, "null descriptor or output pointer");
  *out = nullptr;
  const int64_t V = desc->n_vertices, T = desc->n_triangles, P = desc->n_prims;
  if (V < 3 || V > INT32_MAX) return fail(CCSP_E_ARG, "n_vertices %lld out of range", (long long)V);
  if (T < 1 || T >= (int64_t(1) << 29)) return fail(CCSP_E_ARG, "n_triangles %lld out of range [1, 2^29)", (long long)T);
  if (P < 0 || P > INT32_MAX - 3) return fail(CCSP_E_ARG, "n_prims %lld out of range", (long long)P);
  if (!desc->xy || !desc->tri_v || !desc->tri_nbr || !desc->tri_prim || (P > 0 && !desc->prim_seg))
    return fail(CCSP_E_ARG, "null array in descriptor");
  const double* xy = desc->xy;
  const int32_t *tv = desc->tri_v, *tn = desc->tri_nbr, *tp = desc->tri_prim;
  const double* ps = desc->prim_seg;

  // ---- validation (first failure per worker, reported in triangle order)
  const double kMax = 0x1p64;
  for (int64_t i = 0; i < 2 * V; ++i)
    if (!std::isfinite(xy[i]) || std::fabs(xy[i]) >= kMax)
      return fail(CCSP_E_BAD_TRIANGULATION, "vertex %lld: coordinate not finite or |x| >= 2^64", (long long)(i / 2));
  for (int64_t i = 0; i < 4 * P; ++i)
    if (!std::isfinite(ps[i]) || std::fabs(ps[i]) >= kMax)
      return fail(CCSP_E_BAD_TRIANGULATION, "primitive %lld: coordinate not finite or |x| >= 2^64", (long long)(i / 4));
  std::vector<int64_t> bad(64, INT64_MAX);
  std::vector<std::string> why(64);
  std::atomic<int> slot{0};
  std::vector<uint8_t> used(V, 0);
  std::atomic<int64_t> n_hull{0};
  parallel_for(T, [&](int64_t a, int64_t b) {
    const int me = slot.fetch_add(1);
    int64_t hull = 0;
    auto note = [&](int64_t t, const char* w) {
      if (t < bad[me]) { bad[me] = t; why[me] = w; }
    };
    for (int64_t t = a; t < b && bad[me] == INT64_MAX; ++t) {
      const int32_t* v = tv + 3 * t;
      bool ids_ok = true;
      for (int i = 0; i < 3; ++i)
        if (v[i] < 0 || v[i] >= V) ids_ok = false;
      if (!ids_ok) { note(t, "vertex id out of range"); break; }
      for (int i = 0; i < 3; ++i) used[v[i]] = 1;  // benign race: every writer stores 1
      if (orient_host(xy + 2 * (int64_t)v[0], xy + 2 * (int64_t)v[1], xy + 2 * (int64_t)v[2]) <= 0) {
        note(t, "triangle is not strictly counter-clockwise");
        break;
      }
      for (int i = 0; i < 3; ++i) {
        const int32_t n = tn[3 * t + i], pr = tp[3 * t + i];
        if (pr < -1 || pr >= P) { note(t, "primitive id out of range"); break; }
        const int32_t p = v[(i + 1) % 3], q = v[(i + 2) % 3];
        if (pr >= 0) {
          const double* s = ps + 4 * (int64_t)pr;
          if (orient_host(s, s + 2, xy + 2 * (int64_t)p) != 0 || orient_host(s, s + 2, xy + 2 * (int64_t)q) != 0) {
            note(t, "constrained edge is not collinear with its primitive");
            break;
          }
        }
        if (n == -1) { ++hull; continue; }
        if (n < 0 || n >= T) { note(t, "neighbour out of range"); break; }
        int back = -1, hits = 0;
        for (int j = 0; j < 3; ++j)
          if (tn[3 * (int64_t)n + j] == t) { back = j; ++hits; }
        if (hits != 1) { note(t, "adjacency is not symmetric"); break; }
        const int32_t* w = tv + 3 * (int64_t)n;
        if (w[(back + 1) % 3] != q || w[(back + 2) % 3] != p) { note(t, "shared edge does not match its neighbour"); break; }
        if (tp[3 * (int64_t)n + back] != pr) { note(t, "primitive differs across a shared edge"); break; }
      }
    }
    n_hull += hull;
  });
  int64_t first = INT64_MAX;
  std::string reason;
  for (int k = 0; k < 64; ++k)
    if (bad[k] < first) { first = bad[k]; reason = why[k]; }
  if (first != INT64_MAX)
    return fail(CCSP_E_BAD_TRIANGULATION, "triangle %lld: %s", (long long)first, reason.c_str());
  int64_t vused = 0;
  for (int64_t i = 0; i < V; ++i) vused += used[i];
  const int64_t E = (3 * T + n_hull.load()) / 2;
  if (vused - E + T != 1)
    return fail(CCSP_E_BAD_TRIANGULATION, "Euler characteristic V - E + T = %lld, expected 1 (one disk)",
                (long long)(vused - E + T));

  // ---- packing. Internal triangle order: Hilbert order of the centroids, so that ids close
  // together are triangles close together (neighbouring steps share cache lines and pages, and
  // an id range is a compact region for ray binning).
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  for (int64_t i = 0; i < V; ++i)
    for (int k = 0; k < 2; ++k) {
      lo[k] = std::min(lo[k], xy[2 * i + k]);
      hi[k] = std::max(hi[k], xy[2 * i + k]);
    }
  const double org[2] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])};
  std::vector<uint64_t> hkey(T);
  {
    const double span = std::max(hi[0] - lo[0], hi[1] - lo[1]);
    const double sc = span > 0 ? 65535.0 / span : 0.0;
    parallel_for(T, [&](int64_t a, int64_t b) {
      for (int64_t t = a; t < b; ++t) {
        double cx = 0, cy = 0;
        for (int i = 0; i < 3; ++i) {
          cx += xy[2 * (int64_t)tv[3 * t + i]];
          cy += xy[2 * (int64_t)tv[3 * t + i] + 1];
        }
        const uint32_t gx = (uint32_t)std::min(65535.0, std::max(0.0, (cx / 3.0 - lo[0]) * sc));
        const uint32_t gy = (uint32_t)std::min(65535.0, std::max(0.0, (cy / 3.0 - lo[1]) * sc));
        hkey[t] = ((uint64_t)hilbert16(gx, gy) << 32) | (uint64_t)t;
      }
    });
    std::sort(hkey.begin(), hkey.end());
  }
  std::vector<int32_t> new_of(T);
  for (int64_t r = 0; r < T; ++r) new_of[(int64_t)(hkey[r] & 0xffffffffu)] = (int32_t)r;
  // ---- point-location seeds (Sec. 5.2: points with known triangles on the centres of a regular
  // grid, from which a walk reaches any point): a G x G grid over the bounding square, about four
  // triangles per cell; each cell keeps a point strictly inside a triangle containing its centre
  const double seed_span = std::max(hi[0] - lo[0], hi[1] - lo[1]);
  const int G = (int)std::min<int64_t>(
      4096, std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)T / 4.0))));
  const double ch = seed_span > 0 ? seed_span / G : 1.0;
  std::vector<SeedCell> seeds((size_t)G * G);
  {
    std::vector<std::atomic<int32_t>> cell_tri((size_t)G * G);
    for (auto& c : cell_tri) c.store(INT32_MAX, std::memory_order_relaxed);
    auto P = [&](int64_t vtx) { return xy + 2 * vtx; };
    parallel_for(T, [&](int64_t a, int64_t b) {
      for (int64_t nt = a; nt < b; ++nt) {
        const int32_t* v = tv + 3 * (int64_t)(hkey[nt] & 0xffffffffu);
        const double *p0 = P(v[0]), *p1 = P(v[1]), *p2 = P(v[2]);
        const double x0 = std::min({p0[0], p1[0], p2[0]}), x1 = std::max({p0[0], p1[0], p2[0]});
        const double y0 = std::min({p0[1], p1[1], p2[1]}), y1 = std::max({p0[1], p1[1], p2[1]});
        const int i0 = std::max(0, (int)std::ceil((x0 - lo[0]) / ch - 0.5));
        const int i1 = std::min(G - 1, (int)std::floor((x1 - lo[0]) / ch - 0.5));
        const int j0 = std::max(0, (int)std::ceil((y0 - lo[1]) / ch - 0.5));
        const int j1 = std::min(G - 1, (int)std::floor((y1 - lo[1]) / ch - 0.5));
        for (int j = j0; j <= j1; ++j)
          for (int i = i0; i <= i1; ++i) {
            const double c[2] = {lo[0] + (i + 0.5) * ch, lo[1] + (j + 0.5) * ch};
            if (orient_host(p1, p2, c) < 0 || orient_host(p2, p0, c) < 0 || orient_host(p0, p1, c) < 0)
              continue;
            std::atomic<int32_t>& cell = cell_tri[(size_t)j * G + i];
            int32_t cur = cell.load(std::memory_order_relaxed);
            while ((int32_t)nt < cur && !cell.compare_exchange_weak(cur, (int32_t)nt)) {
            }
          }
      }
    });
    // a point strictly inside internal triangle nt (the centroid, else other interior mixes)
    auto interior = [&](int64_t nt, const double* pref, SeedCell* out) {
      const int32_t* v = tv + 3 * (int64_t)(hkey[nt] & 0xffffffffu);
      const double *p0 = P(v[0]), *p1 = P(v[1]), *p2 = P(v[2]);
      const double w[5][3] = {{1, 1, 1}, {0, 0, 0}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2}};
      for (int k = 0; k < 5; ++k) {
        double q[2];
        if (k == 1) {
          if (!pref) continue;
          q[0] = pref[0];
          q[1] = pref[1];
        } else {
          const double s = w[k][0] + w[k][1] + w[k][2];
          for (int c = 0; c < 2; ++c) q[c] = (w[k][0] * p0[c] + w[k][1] * p1[c] + w[k][2] * p2[c]) / s;
        }
        if (orient_host(p1, p2, q) > 0 && orient_host(p2, p0, q) > 0 && orient_host(p0, p1, q) > 0) {
          *out = SeedCell{q[0], q[1], (int32_t)nt, 0};
          return true;
        }
      }
      return false;
    };
    std::vector<uint8_t> have((size_t)G * G, 0);
    parallel_for((int64_t)G * G, [&](int64_t a, int64_t b) {
      for (int64_t k = a; k < b; ++k) {
        const int32_t nt = cell_tri[k].load(std::memory_order_relaxed);
        if (nt == INT32_MAX) continue;
        const double c[2] = {lo[0] + ((k % G) + 0.5) * ch, lo[1] + ((k / G) + 0.5) * ch};
        have[k] = interior(nt, c, &seeds[k]);
      }
    });
    // cells left without a seed take the nearest seeded cell's (breadth-first over the grid)
    std::queue<int64_t> bfs;
    for (int64_t k = 0; k < (int64_t)G * G; ++k)
      if (have[k]) bfs.push(k);
    if (bfs.empty()) {
      SeedCell any{};
      bool found = false;
      for (int64_t nt = 0; nt < T && !found; ++nt) found = interior(nt, nullptr, &any);
      if (!found) return fail(CCSP_E_BAD_TRIANGULATION, "no point strictly inside any triangle");
      for (auto& s : seeds) s = any;
    }
    while (!bfs.empty()) {
      const int64_t k = bfs.front();
      bfs.pop();
      const int64_t i = k % G, j = k / G;
      const int64_t nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
      for (const auto& n2 : nb) {
        if (n2[0] < 0 || n2[0] >= G || n2[1] < 0 || n2[1] >= G) continue;
        const int64_t m = n2[1] * G + n2[0];
        if (have[m]) continue;
        have[m] = 1;
        seeds[m] = seeds[k];
        bfs.push(m);
      }
    }
  }

  // primitives stay in the caller's order: the walk reads a primitive's segment at a hit, and
  // binned rays hit the primitives of one region at a time, whose lines then stay in L2
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t off_s32 = 0;
  const size_t off_s64 = align(off_s32 + sizeof(Slot32) * 3 * T);
  const size_t off_first = align(off_s64 + sizeof(Slot64) * 3 * T);
  const size_t off_tv = align(off_first + sizeof(TriFirst) * T);
  const size_t off_v = align(off_tv + sizeof(int4) * T);
  const size_t off_p = align(off_v + sizeof(double2) * V);
  const size_t off_perm = align(off_p + sizeof(PrimRec) * std::max<int64_t>(P, 1));
  const size_t off_orig = align(off_perm + sizeof(int32_t) * T);
  const size_t off_seed = align(off_orig + sizeof(int32_t) * T);
  const size_t off_pair = align(off_seed + sizeof(SeedCell) * seeds.size());
  const size_t off_pair64 = align(off_pair + sizeof(Pair32) * 3 * T);
  const size_t total = align(off_pair64 + sizeof(Pair64) * 3 * T);
  std::vector<unsigned char> host(total, 0);
  auto* s32 = reinterpret_cast<Slot32*>(host.data() + off_s32);
  auto* s64 = reinterpret_cast<Slot64*>(host.data() + off_s64);
  auto* tfirst = reinterpret_cast<TriFirst*>(host.data() + off_first);
  auto* t4 = reinterpret_cast<int4*>(host.data() + off_tv);
  std::memcpy(host.data() + off_v, xy, sizeof(double) * 2 * V);
  static_assert(sizeof(PrimRec) == 4 * sizeof(double), "primitive record = its segment");
  if (P > 0) std::memcpy(host.data() + off_p, ps, sizeof(PrimRec) * P);
  std::memcpy(host.data() + off_perm, new_of.data(), sizeof(int32_t) * T);
  {
    auto* orig = reinterpret_cast<int32_t*>(host.data() + off_orig);
    for (int64_t r = 0; r < T; ++r) orig[r] = (int32_t)(hkey[r] & 0xffffffffu);
  }
  std::memcpy(host.data() + off_seed, seeds.data(), sizeof(SeedCell) * seeds.size());
  parallel_for(T, [&](int64_t a, int64_t b) {
    for (int64_t nt = a; nt < b; ++nt) {
      const int64_t t = (int64_t)(hkey[nt] & 0xffffffffu);  // caller's id of internal triangle nt
      const int32_t* v = tv + 3 * t;
      t4[nt] = make_int4(v[0], v[1], v[2], 0);
      TriFirst& f = tfirst[t];  // the caller's order
      for (int i = 0; i < 3; ++i) {
        f.x[i] = (float)(xy[2 * (int64_t)v[i]] - org[0]);
        f.y[i] = (float)(xy[2 * (int64_t)v[i] + 1] - org[1]);
      }
      f.tri = (int32_t)nt;
      f.pad = 0;
      for (int i = 0; i < 3; ++i) {
        const int64_t k = 3 * nt + i;
        const int32_t n = tn[3 * t + i], pr = tp[3 * t + i];
        int32_t through = -1, vid = 0;
        if (n >= 0) {
          int back = 0;
          for (int j = 0; j < 3; ++j)
            if (tn[3 * (int64_t)n + j] == t) back = j;
          through = (new_of[n] << 2) | back;
          vid = tv[3 * (int64_t)n + back];
        }
        const int32_t word = pr >= 0 ? -(pr + 2) : through;
        const double vx = xy[2 * (int64_t)vid], vy = xy[2 * (int64_t)vid + 1];
        s32[k].word = word;
        // the vertex opposite the edge in this triangle, for a ray reflected at a constrained edge
        const int32_t own = v[i];
        s32[k].vid = word >= 0 ? vid : own;
        s32[k].x = word >= 0 ? (float)(vx - org[0]) : 0.0f;
        s32[k].y = word >= 0 ? (float)(vy - org[1]) : 0.0f;
        s64[k].word = word;
        s64[k].vid = vid;
        s64[k].x = through >= 0 ? vx : 0.0;
        s64[k].y = through >= 0 ? vy : 0.0;
        s64[k].through = through;
        s64[k].own = own;
      }
    }
  });
  // two-step records from the single-step slots
  auto* pr32 = reinterpret_cast<Pair32*>(host.data() + off_pair);
  parallel_for(3 * T, [&](int64_t a, int64_t b) {
    for (int64_t k = a; k < b; ++k) {
      const Slot32& sl = s32[k];
      Pair32& pr = pr32[k];
      if (sl.word < 0) {
        pr.nx = pr.ny = std::numeric_limits<float>::quiet_NaN();
        pr.w0 = sl.word;
        pr.x0 = pr.y0 = pr.x1 = pr.y1 = 0.0f;
        pr.w1 = 0;
        continue;
      }
      pr.nx = sl.x;
      pr.ny = sl.y;
      const int64_t n = sl.word >> 2;
      const int en = sl.word & 3;
      const Slot32& l = s32[3 * n + (en + 1) % 3];
      const Slot32& r = s32[3 * n + (en + 2) % 3];
      pr.w0 = l.word;
      pr.x0 = l.x;
      pr.y0 = l.y;
      pr.w1 = r.word;
      pr.x1 = r.x;
      pr.y1 = r.y;
    }
  });
  auto* pr64 = reinterpret_cast<Pair64*>(host.data() + off_pair64);
  parallel_for(3 * T, [&](int64_t a, int64_t b) {
    for (int64_t k = a; k < b; ++k) {
      const Slot64& sl = s64[k];
      Pair64& pr = pr64[k];
      pr.pad[0] = pr.pad[1] = 0;
      if (sl.word < 0) {
        pr.nx = pr.ny = std::numeric_limits<double>::quiet_NaN();
        pr.x0 = pr.y0 = pr.x1 = pr.y1 = 0.0;
        pr.w0 = sl.word;
        pr.w1 = 0;
        continue;
      }
      pr.nx = sl.x;
      pr.ny = sl.y;
      const int64_t n = sl.word >> 2;
      const int en = sl.word & 3;
      const Slot64& l = s64[3 * n + (en + 1) % 3];
      const Slot64& r = s64[3 * n + (en + 2) % 3];
      pr.x0 = l.x;
      pr.y0 = l.y;
      pr.w0 = l.word;
      pr.x1 = r.x;
      pr.y1 = r.y;
      pr.w1 = r.word;
    }
  });

  // ---- upload
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  auto* tri = new Triangulation;
  (void)hipGetDevice(&tri->device);
  hipError_t e = hipMalloc(&tri->mem, total);
  if (e != hipSuccess) {
    delete tri;
    return fail(CCSP_E_OOM, "device allocation of %zu bytes failed: %s", total, hipGetErrorString(e));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  e = hipMemcpyAsync(tri->mem, host.data(), total, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipFree(tri->mem);
    delete tri;
    return hip_fail(e, "upload");
  }
  auto* base = static_cast<unsigned char*>(tri->mem);
  tri->bytes = total;
  tri->nv = V;
  tri->nt = T;
  tri->np = P;
  tri->dev.slot32 = reinterpret_cast<const Slot32*>(base + off_s32);
  tri->dev.pair32 = reinterpret_cast<const Pair32*>(base + off_pair);
  tri->dev.pair64 = reinterpret_cast<const Pair64*>(base + off_pair64);
  tri->dev.slot64 = reinterpret_cast<const Slot64*>(base + off_s64);
  tri->dev.first = reinterpret_cast<const TriFirst*>(base + off_first);
  tri->dev.triv = reinterpret_cast<const int4*>(base + off_tv);
  tri->dev.v64 = reinterpret_cast<const double2*>(base + off_v);
  tri->dev.prim = reinterpret_cast<const PrimRec*>(base + off_p);
  tri->dev.perm = reinterpret_cast<const int32_t*>(base + off_perm);
  tri->dev.orig = reinterpret_cast<const int32_t*>(base + off_orig);
  tri->dev.seeds = reinterpret_cast<const SeedCell*>(base + off_seed);
  tri->dev.seed_x0 = lo[0];
  tri->dev.seed_y0 = lo[1];
  tri->dev.seed_inv = 1.0 / ch;
  tri->dev.seed_g = G;
  tri->dev.org_x = org[0];
  tri->dev.org_y = org[1];
  tri->dev.box_x0 = lo[0];
  tri->dev.box_y0 = lo[1];
  tri->dev.box_x1 = hi[0];
  tri->dev.box_y1 = hi[1];
  tri->dev.ntri = (int32_t)T;
  *out = tri;
  return CCSP_OK;
}

void free_triangulation(Triangulation* tri) {
  if (!tri) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(tri->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(tri->mem);
  (void)hipSetDevice(cur);
  delete tri;
}

int triangulation_info(const Triangulation* tri, int64_t out[4]) {
  if (!tri || !out) return fail(CCSP_E_ARG, "null argument");
  out[0] = tri->nt;
  out[1] = tri->nv;
  out[2] = tri->np;
  out[3] = (int64_t)tri->bytes;
  return CCSP_OK;
}

static int check_rays(const double* o, const double* d, const int32_t* s, int64_t n, int32_t* hp,
                      double* ht, int32_t* st) {
  if (n < 0) return fail(CCSP_E_ARG, "negative ray count");
  if (n == 0) return CCSP_OK;
  if (!o || !d || !s || !hp || !ht || !st) return fail(CCSP_E_ARG, "null ray or output pointer");
  if (!aligned(o, 16) || !aligned(d, 16)) return fail(CCSP_E_ARG, "o_xy and d_xy must be 16-byte aligned");
  if (!aligned(ht, 8) || !aligned(s, 4) || !aligned(hp, 4) || !aligned(st, 4))
    return fail(CCSP_E_ARG, "misaligned output or start_tri");
  return CCSP_OK;
}

static int trace_common(const Triangulation* tri, const double* o_xy, const double* d_xy,
                        const int32_t* start_tri, int64_t n, int precision, int32_t* hit_prim,
                        double* hit_t, int32_t* steps, const TuneParams* tune, void* stream,
                        int32_t* bounces, int32_t* hit_face, int32_t max_bounces) {
  g_err.clear();
  if (!tri) return fail(CCSP_E_ARG, "null triangulation");
  const int mode = precision & CCSP_TRACE_MODE_MASK;
  if (mode != CCSP_TRACE_FP64 && mode != CCSP_TRACE_FP32_FILTERED)
    return fail(CCSP_E_ARG, "unknown precision mode %d", mode);
  if (precision & ~(CCSP_TRACE_MODE_MASK | CCSP_TRACE_VALIDATE | CCSP_TRACE_COUNT | CCSP_TRACE_INPUT_ORDER |
                    CCSP_TRACE_TIMED))
    return fail(CCSP_E_ARG, "unknown precision flags 0x%x", precision);
  int rc = check_rays(o_xy, d_xy, start_tri, n, hit_prim, hit_t, steps);
  if (rc || n == 0) return rc;
  DeviceState* ds = nullptr;
  rc = device_state(&ds);
  if (rc) return rc;
  rc = check_tune(tune);
  if (rc) return rc;
  TuneParams cached;
  if (!tune && tune_lookup(ds, tune_key(1, n, tri->nt, precision, true), &cached)) tune = &cached;
  const LaunchCfg cfg = make_cfg(ds->cus, mode, tune);
  rc = check_cfg(cfg);
  if (rc) return rc;
  const bool validate = precision & CCSP_TRACE_VALIDATE;
  const bool count = precision & CCSP_TRACE_COUNT;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RaysDev io{reinterpret_cast<const double2*>(o_xy), reinterpret_cast<const double2*>(d_xy),
             start_tri, hit_prim, hit_t, steps, n, nullptr};
  io.hits = bounces;
  io.face = hit_face;
  io.max_bounces = max_bounces;
  io.max_steps = tune ? tune->step_limit : 0;
  int* errflag = nullptr;
  unsigned long long* counter = next_counters(ds, &errflag);
  hipError_t e;
  StageEvents* tev = nullptr;
  if (precision & CCSP_TRACE_TIMED) {
    rc = timing_slot(ds, &tev);
    if (rc) return rc;
    e = hipEventRecord(tev->ev[0], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  const bool bin = !(precision & CCSP_TRACE_INPUT_ORDER) && n >= kBinMinRays && n < INT32_MAX &&
                   tri->nt >= kBinMinTriangles;
  std::unique_lock<std::mutex> bin_lock(ds->bin_mu, std::defer_lock);
  if (bin) {
    bin_lock.lock();
    rc = grow_bin_workspace(ds, n);
    if (rc) return rc;
    // the shared scratch may still be in use by a trace on another stream
    if (ds->bin_last_stream != st) {
      e = hipStreamWaitEvent(st, ds->bin_free, 0);
      if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    RaysDev binned{};
    e = launch_bin_rays(tri->dev, io, (tune && tune->bin == 2) ? kBinRadix : kBinBuckets,
                        ds->bin_ws, ds->bin_ws_bytes, &binned, count ? ds->ws.stats : nullptr, st);
    io = binned;
    if (e != hipSuccess) return hip_fail(e, "ray binning");
  }
  if (validate) {
    e = hipMemsetAsync(errflag, 0, sizeof(int), st);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  }
  e = launch_walk(tri->dev, io, mode, count, validate, cfg, counter, errflag, ds->ws, st,
                  tev ? tev->ev[1] : nullptr, tev ? tev->ev[2] : nullptr);
  if (e != hipSuccess) return hip_fail(e, "walk launch");
  if (tev) {
    e = hipEventRecord(tev->ev[3], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  if (bin) {
    e = hipEventRecord(ds->bin_free, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ds->bin_last_stream = st;
    bin_lock.unlock();
  }
  if (validate) {
    int flag = 0;
    e = hipMemcpyAsync(&flag, errflag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "validation read-back");
    if (flag) return fail(CCSP_E_BAD_RAY, "a ray's origin is not strictly inside its start triangle, its start "
                                          "triangle is out of range, or its direction is zero or not finite");
  }
  return CCSP_OK;
}

int trace_rays_tuned(const Triangulation* tri, const double* o_xy, const double* d_xy,
                     const int32_t* start_tri, int64_t n, int precision, int32_t* hit_prim,
                     double* hit_t, int32_t* steps, const TuneParams* tune, void* stream) {
  return trace_common(tri, o_xy, d_xy, start_tri, n, precision, hit_prim, hit_t, steps, tune,
                      stream, nullptr, nullptr, 0);
}

int trace_bounces(const Triangulation* tri, const double* o_xy, const double* d_xy,
                  const int32_t* start_tri, int64_t n, int32_t max_bounces, int precision,
                  int32_t* hit_prim, double* hit_t, int32_t* steps, int32_t* bounces,
                  int32_t* hit_face, const TuneParams* tune, void* stream) {
  g_err.clear();
  if (max_bounces < 0) return fail(CCSP_E_ARG, "negative max_bounces");
  if (precision & CCSP_TRACE_VALIDATE) return fail(CCSP_E_ARG, "trace_bounces does not validate");
  if (n > 0 && !bounces) return fail(CCSP_E_ARG, "null bounces output");
  if (!aligned(bounces, 4) || !aligned(hit_face, 4)) return fail(CCSP_E_ARG, "misaligned output");
  return trace_common(tri, o_xy, d_xy, start_tri, n, precision, hit_prim, hit_t, steps, tune,
                      stream, n > 0 ? bounces : nullptr, hit_face, max_bounces);
}

int trace_rays(const Triangulation* tri, const double* o_xy, const double* d_xy,
               const int32_t* start_tri, int64_t n, int precision, int32_t* hit_prim,
               double* hit_t, int32_t* steps, void* stream) {
  return trace_rays_tuned(tri, o_xy, d_xy, start_tri, n, precision, hit_prim, hit_t, steps, nullptr,
                          stream);
}

int trace_batch(const TraceItem* items, int32_t n_items, int precision, const TuneParams* tune,
                void* stream) {
  g_err.clear();
  if (n_items < 0 || (n_items > 0 && !items)) return fail(CCSP_E_ARG, "bad item array");
  const int mode = precision & CCSP_TRACE_MODE_MASK;
  if (mode != CCSP_TRACE_FP64 && mode != CCSP_TRACE_FP32_FILTERED)
    return fail(CCSP_E_ARG, "unknown precision mode %d", mode);
  if (precision & ~(CCSP_TRACE_MODE_MASK | CCSP_TRACE_COUNT | CCSP_TRACE_TIMED | CCSP_TRACE_GRAPH))
    return fail(CCSP_E_ARG, "unsupported precision flags 0x%x for trace_batch", precision);
  int rc = check_tune(tune);
  if (rc) return rc;
  DeviceState* ds = nullptr;
  rc = device_state(&ds);
  if (rc) return rc;
  int64_t total_rays = 0, total_tris = 0;
  for (int i = 0; i < n_items; ++i) {
    const TraceItem& it = items[i];
    if (!it.scene) return fail(CCSP_E_ARG, "item %d: null scene", i);
    rc = check_rays(it.o_xy, it.d_xy, it.start_tri, it.n, it.hit_prim, it.hit_t, it.steps);
    if (rc) return fail(rc, "item %d: %s", i, g_err.c_str());
    total_rays += it.n;
    total_tris += it.scene->nt;
  }
  TuneParams cached;
  if (!tune && tune_lookup(ds, tune_key(n_items, total_rays, total_tris, precision, false), &cached))
    tune = &cached;
  const LaunchCfg cfg = make_cfg(ds->cus, mode, tune);
  rc = check_cfg(cfg);
  if (rc) return rc;
  const bool use_graph = precision & CCSP_TRACE_GRAPH;
  int64_t tiles = 0;
  for (int i = 0; i < n_items; ++i) tiles += (items[i].n + cfg.tile - 1) / cfg.tile;
  if (tiles == 0) return CCSP_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(ds->mu);
  hipError_t e;
  if (n_items > ds->items_cap) {
    rc = grow_item_tables(ds, n_items);
    if (rc) return rc;
  }
  const unsigned slot = ds->ring_next++ % kTableSlots;
  TableSlot& hs = ds->host_ring[slot];
  if (hs.used) {  // this pinned table's previous upload must be done before it is rewritten
    e = hipEventSynchronize(hs.free_ev);
    if (e != hipSuccess) return hip_fail(e, "staging wait");
  }
  BatchItem* host = static_cast<BatchItem*>(hs.p);
  int64_t tb = 0;
  for (int i = 0; i < n_items; ++i) {
    const TraceItem& it = items[i];
    BatchItem& b = host[i];
    b.scene = it.scene->dev;
    b.rays = RaysDev{reinterpret_cast<const double2*>(it.o_xy), reinterpret_cast<const double2*>(it.d_xy),
                     it.start_tri, it.hit_prim, it.hit_t, it.steps, it.n};
    b.rays.max_steps = tune ? tune->step_limit : 0;
    b.tile_begin = tb;
    tb += (it.n + cfg.tile - 1) / cfg.tile;
  }
  const bool count = precision & CCSP_TRACE_COUNT;
  StageEvents* tev = nullptr;
  if (precision & CCSP_TRACE_TIMED) {
    rc = timing_slot(ds, &tev);
    if (rc) return rc;
    e = hipEventRecord(tev->ev[0], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  BatchGraph* g = nullptr;
  TableSlot* dslot = nullptr;
  BatchItem* table = nullptr;
  if (use_graph) {
    // (reset, walk) captured once per key and replayed; the item table is uploaded into
    // the graph's own table before each replay
    const std::array<int64_t, 10> key{n_items, tiles,    mode,           (int64_t)count, cfg.wg,
                                      cfg.tile, cfg.grid, cfg.refill_min, cfg.chunks,     cfg.group};
    auto itg = ds->graphs.find(key);
    if (itg == ds->graphs.end()) {
      BatchGraph ng;
      rc = capture_batch_graph(ds, n_items, tiles, mode, count, cfg, &ng);
      if (rc) return rc;
      itg = ds->graphs.emplace(key, ng).first;
    }
    g = &itg->second;
    if (g->used && g->last != st) {
      e = hipStreamWaitEvent(st, g->done, 0);
      if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    table = g->dev;
  } else {
    dslot = &ds->dev_ring[slot];
    if (dslot->used) {  // the launch that last read this device table must be done
      e = hipStreamWaitEvent(st, dslot->free_ev, 0);
      if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    table = static_cast<BatchItem*>(dslot->p);
  }
  e = hipMemcpyAsync(table, host, sizeof(BatchItem) * n_items, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(hs.free_ev, st);
  if (e != hipSuccess) return hip_fail(e, "item table upload");
  hs.used = true;
  if (g) {
    if (tev) e = hipEventRecord(tev->ev[1], st);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, st);
    if (e == hipSuccess) e = hipEventRecord(g->done, st);
    if (e != hipSuccess) return hip_fail(e, "graph replay");
    g->last = st;
    g->used = true;
    if (tev) {
      e = hipEventRecord(tev->ev[2], st);
      if (e == hipSuccess) e = hipEventRecord(tev->ev[3], st);
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return CCSP_OK;
  }
  e = launch_walk_batch(table, n_items, tiles, mode, count, cfg, next_counters(ds), ds->ws, st,
                        tev ? tev->ev[1] : nullptr, tev ? tev->ev[2] : nullptr);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  e = hipEventRecord(dslot->free_ev, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  dslot->used = true;
  if (tev) {
    e = hipEventRecord(tev->ev[3], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  return CCSP_OK;
}

int trace_rays_static(const Triangulation* tri, const double* o_xy, const double* d_xy,
                      const int32_t* start_tri, int64_t n, int precision, int32_t* hit_prim,
                      double* hit_t, int32_t* steps, const TuneParams* tune, void* stream) {
  g_err.clear();
  if (!tri) return fail(CCSP_E_ARG, "null triangulation");
  const int mode = precision & CCSP_TRACE_MODE_MASK;
  if (mode != CCSP_TRACE_FP64 && mode != CCSP_TRACE_FP32_FILTERED)
    return fail(CCSP_E_ARG, "unknown precision mode %d", mode);
  if (precision & ~(CCSP_TRACE_MODE_MASK | CCSP_TRACE_INPUT_ORDER))
    return fail(CCSP_E_ARG, "trace_rays_static takes a precision mode and CCSP_TRACE_INPUT_ORDER "
                            "only (flags 0x%x)", precision);
  int rc = check_rays(o_xy, d_xy, start_tri, n, hit_prim, hit_t, steps);
  if (rc) return rc;
  if (n > CCSP_STATIC_MAX_RAYS)
    return fail(CCSP_E_ARG, "trace_rays_static traces at most %d rays per call (%lld given)",
                CCSP_STATIC_MAX_RAYS, (long long)n);
  if (n == 0) return CCSP_OK;
  rc = check_tune(tune);
  if (rc) return rc;
  StaticScratch* ss = nullptr;
  rc = static_scratch(&ss);
  if (rc) return rc;
  const LaunchCfg cfg = make_cfg(ss->cus, mode, tune);
  rc = check_cfg(cfg);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RaysDev io{reinterpret_cast<const double2*>(o_xy), reinterpret_cast<const double2*>(d_xy),
             start_tri, hit_prim, hit_t, steps, n, nullptr};
  io.max_steps = tune ? tune->step_limit : 0;
  Workspace ws{};
  ws.counters = reinterpret_cast<unsigned long long*>(ss->ptr);  // zeroed by the walk launch
  ws.stats = ws.counters + kClaimChunks;                          // not written (no counting)
  hipError_t e;
  const bool bin = !(precision & CCSP_TRACE_INPUT_ORDER) && n >= kBinMinRays &&
                   tri->nt >= kBinMinTriangles;
  if (bin) {
    RaysDev binned{};
    e = launch_bin_rays(tri->dev, io, (tune && tune->bin == 2) ? kBinRadix : kBinBuckets,
                        ss->ptr + kStaticBinOffset, kStaticScratchBytes - kStaticBinOffset, &binned,
                        nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "ray binning");
    io = binned;
  }
  e = launch_walk(tri->dev, io, mode, false, false, cfg, ws.counters, nullptr, ws, st);
  if (e != hipSuccess) return hip_fail(e, "walk launch");
  return CCSP_OK;
}

int reserve_workspace(int64_t max_rays) {
  g_err.clear();
  if (max_rays < 0 || max_rays >= INT32_MAX) return fail(CCSP_E_ARG, "max_rays out of range");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ds->bin_mu);
  return grow_bin_workspace(ds, max_rays);
}

int locate_points(const Triangulation* tri, const double* q_xy, int64_t n, int32_t* tri_out,
                  int32_t* status, void* stream) {
  g_err.clear();
  if (!tri) return fail(CCSP_E_ARG, "null triangulation");
  if (n < 0) return fail(CCSP_E_ARG, "negative point count");
  if (n == 0) return CCSP_OK;
  if (!q_xy || !tri_out || !status) return fail(CCSP_E_ARG, "null point or output pointer");
  if (!aligned(q_xy, 16) || !aligned(tri_out, 4) || !aligned(status, 4))
    return fail(CCSP_E_ARG, "q_xy must be 16-byte aligned, outputs 4-byte aligned");
  const hipError_t e = launch_locate(tri->dev, reinterpret_cast<const double2*>(q_xy), n, tri_out,
                                     status, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "locate launch");
  return CCSP_OK;
}

int tune_cache_set(int32_t n_items, int64_t total_rays, int64_t total_triangles, int precision,
                   const TuneParams* tune) {
  g_err.clear();
  if (!tune || n_items < 1 || total_rays < 0 || total_triangles < 0)
    return fail(CCSP_E_ARG, "bad tuning cache entry");
  int rc = check_tune(tune);
  if (rc) return rc;
  DeviceState* ds = nullptr;
  rc = device_state(&ds);
  if (rc) return rc;
  LaunchCfg cfg = make_cfg(ds->cus, precision & CCSP_TRACE_MODE_MASK, tune);
  rc = check_cfg(cfg);
  if (rc) return rc;
  const bool single = n_items == 1 && !(precision & CCSP_TRACE_GRAPH);
  std::lock_guard<std::mutex> lk(ds->tune_mu);
  TuneParams t = *tune;
  t.step_limit = 0;  // a limit of the walk, not a launch parameter of the shape
  ds->tuned[tune_key(n_items, total_rays, total_triangles, precision, single)] = t;
  return CCSP_OK;
}

int tune_cache_get(int32_t n_items, int64_t total_rays, int64_t total_triangles, int precision,
                   TuneParams* out) {
  g_err.clear();
  if (!out || n_items < 1 || total_rays < 0 || total_triangles < 0)
    return fail(CCSP_E_ARG, "bad tuning cache query");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  const bool single = n_items == 1 && !(precision & CCSP_TRACE_GRAPH);
  return tune_lookup(ds, tune_key(n_items, total_rays, total_triangles, precision, single), out) ? 1 : 0;
}

int autotune(const TraceItem* items, int32_t n_items, int precision, int32_t reps,
             TuneParams* best, float* best_ms, void* stream) {
  g_err.clear();
  if (!items || n_items < 1 || !best || !best_ms) return fail(CCSP_E_ARG, "null or empty argument");
  if (reps < 1 || reps > 1000) return fail(CCSP_E_ARG, "reps %d must be 1..1000", reps);
  const bool single = n_items == 1 && !(precision & CCSP_TRACE_GRAPH);
  if (precision & (CCSP_TRACE_TIMED | CCSP_TRACE_VALIDATE | CCSP_TRACE_COUNT))
    return fail(CCSP_E_ARG, "autotune takes a precision mode, CCSP_TRACE_GRAPH or CCSP_TRACE_INPUT_ORDER");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
      return fail(CCSP_E_HIP, "hipEventCreate");
    }
  auto run = [&](const TuneParams& tp) -> int {
    const TraceItem& it = items[0];
    return single ? trace_rays_tuned(it.scene, it.o_xy, it.d_xy, it.start_tri, it.n, precision,
                                     it.hit_prim, it.hit_t, it.steps, &tp, stream)
                  : trace_batch(items, n_items, precision, &tp, stream);
  };
  // mean time of `reps` calls after one untimed call (which also builds graphs and scratch)
  auto measure = [&](const TuneParams& tp, float* ms) -> int {
    int r = run(tp);
    if (r) return r;
    hipError_t e = hipEventRecord(ev[0], st);
    for (int k = 0; k < reps && e == hipSuccess && r == CCSP_OK; ++k) r = run(tp);
    if (r) return r;
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *ms /= (float)reps;
    return CCSP_OK;
  };
  // coordinate search from the defaults: each parameter in turn over its candidates, the others
  // fixed, keeping the fastest; two passes
  TuneParams cur{256, 64, 24, 16, 4, kClaimChunks, 0, 0};
  float cur_ms = 0;
  rc = measure(cur, &cur_ms);
  struct Axis {
    int32_t TuneParams::*field;
    std::vector<int32_t> values;
  };
  const Axis axes[] = {
      {&TuneParams::waves_per_cu, {8, 12, 16, 20, 24, 28}},
      {&TuneParams::refill_min, {4, 8, 16, 24, 32, 48}},
      {&TuneParams::tile_rays, {64, 128, 256}},
      {&TuneParams::wg_size, {64, 128, 256, 512}},
      {&TuneParams::tiles_per_claim, {1, 2, 4, 8, 16}},
      {&TuneParams::xcd_chunks, {1, kClaimChunks}},
  };
  for (int pass = 0; pass < 2 && rc == CCSP_OK; ++pass)
    for (const Axis& ax : axes)
      for (int32_t v : ax.values) {
        if (rc || cur.*ax.field == v) continue;
        TuneParams cand = cur;
        cand.*ax.field = v;
        float ms = 0;
        rc = measure(cand, &ms);
        if (rc == CCSP_OK && ms < cur_ms) {
          cur = cand;
          cur_ms = ms;
        }
      }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  int64_t rays = 0, tris = 0;
  for (int i = 0; i < n_items; ++i) {
    rays += items[i].n;
    tris += items[i].scene->nt;
  }
  {
    std::lock_guard<std::mutex> lk(ds->tune_mu);
    ds->tuned[tune_key(n_items, rays, tris, precision, single)] = cur;
  }
  *best = cur;
  *best_ms = cur_ms;
  return CCSP_OK;
}

int read_stage_times(int32_t max_records, float* bin_ms, float* walk_ms, float* finish_ms,
                     int32_t* n_records) {
  g_err.clear();
  if (!n_records) return fail(CCSP_E_ARG, "null n_records");
  *n_records = 0;
  if (max_records < 0) return fail(CCSP_E_ARG, "negative max_records");
  if (max_records > 0 && (!bin_ms || !walk_ms || !finish_ms)) return fail(CCSP_E_ARG, "null output array");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ds->time_mu);
  const int n = std::min(ds->time_count, (int)max_records);
  for (int i = 0; i < n; ++i) {
    const StageEvents& s = ds->tev[(ds->time_next - n + i + kTimeSlots) % kTimeSlots];
    hipError_t e = hipEventSynchronize(s.ev[3]);
    if (e == hipSuccess) e = hipEventElapsedTime(&bin_ms[i], s.ev[0], s.ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&walk_ms[i], s.ev[1], s.ev[2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&finish_ms[i], s.ev[2], s.ev[3]);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
  }
  ds->time_count = 0;
  *n_records = n;
  return CCSP_OK;
}

int read_counters(uint64_t out[4], int reset) {
  if (!out) return fail(CCSP_E_ARG, "null output");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, ds->ws.stats, sizeof(uint64_t) * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && reset) e = hipMemset(ds->ws.stats, 0, sizeof(uint64_t) * 4);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "read_counters");
  return CCSP_OK;
}

}  // extern "C"
