// Device layout of a packed triangulation and the launch interface of the walk kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ccsp {

// Exit-edge word stored per (triangle, edge) slot:
//   >= 0 : (neighbour << 2) | back, where `back` is the edge of the neighbour that leads back
//          (neighbour is an internal triangle id);
//   -1   : unconstrained hull edge (the ray leaves the triangulation);
//   <= -2: constrained edge of primitive (-word - 2), the caller's primitive id.
// Each slot also stores the vertex across the edge (the neighbour's vertex opposite `back`),
// which is exactly the one vertex the next step needs: one dependent load per step.
struct alignas(16) Slot32 {  // binary32 walk: 16 B per slot
  int32_t word;
  float x, y;                 // across vertex, relative to the scene origin, rounded to binary32
  int32_t vid;                // its vertex id (for the binary64 fallback); on a constrained edge,
                              // this triangle's vertex opposite the edge (reflected rays)
};
// Two steps of the binary32 walk in one 32-B load. For exit slot s of a triangle: the across
// vertex of the neighbour n across that edge, then the slots of n's two candidate exits, in the
// order (across vertex LEFT, RIGHT): their words and across vertices. A slot on a constrained or
// hull edge has nx = NaN and w0 = its word. Vertex ids (for the binary64 fallback) stay in Slot32.
struct alignas(32) Pair32 {
  float nx, ny;
  int32_t w0;
  float x0, y0;
  int32_t w1;
  float x1, y1;
};
// The same two steps for the binary64 walk, in one 64-B load: across vertices of n and of its two
// candidate exits (LEFT, RIGHT), and the words of those exits. A slot on a constrained or hull
// edge has nx = NaN and w0 = its word.
struct alignas(64) Pair64 {
  double nx, ny;
  double x0, y0;
  double x1, y1;
  int32_t w0, w1;
  int32_t pad[2];
};
struct alignas(32) Slot64 {  // binary64 walk: 32 B per slot
  double x, y;                // across vertex (binary64, absolute), also across constrained edges
  int32_t word;
  int32_t vid;
  int32_t through;            // (neighbour << 2) | back whatever the constraint, -1 on the hull:
                              // the word of a walk to which constraints are transparent (locate)
  int32_t own;                // this triangle's vertex opposite the edge (reflected rays)
};
// First-triangle record, in the CALLER's triangle order (rays name their start triangle by the
// caller's id): its vertices relative to the scene origin in binary32, and its internal id.
struct alignas(32) TriFirst {
  float x[3], y[3];
  int32_t tri;
  int32_t pad;
};

// A primitive, in the caller's order: its segment (t is computed from it).
struct alignas(32) PrimRec {
  double ax, ay, bx, by;
};

// Seed of point location: a point strictly inside internal triangle `tri`, per grid cell.
struct SeedCell {
  double x, y;
  int32_t tri;
  int32_t pad;
};

struct SceneDev {
  const Slot32* slot32;    // 3T
  const Pair32* pair32;    // 3T
  const Pair64* pair64;    // 3T
  const Slot64* slot64;    // 3T
  const TriFirst* first;   // T, the caller's order
  const int4* triv;      // T: v0, v1, v2, 0
  const double2* v64;    // V
  const PrimRec* prim;   // P, the caller's order
  const int32_t* perm;   // T: caller's triangle id -> internal (Hilbert-ordered) id
  const int32_t* orig;   // T: internal id -> the caller's id
  const SeedCell* seeds;  // seed_g x seed_g cells over the bounding square, row-major
  double seed_x0, seed_y0, seed_inv;  // cell = floor((p - seed_0) * seed_inv)
  int32_t seed_g;
  int32_t pad2;
  double org_x, org_y;   // origin of the binary32 coordinates
  double box_x0, box_y0, box_x1, box_y1;  // bounding box of the vertices
  int32_t ntri;
  int32_t pad;
};

// A binned ray: origin, direction, the exit slot of its first triangle (3 * internal triangle +
// exit edge; -1 if the start triangle is out of range or the origin is not inside it) and the
// caller's index of the ray.
struct alignas(16) RayRec {
  double2 o;
  double2 d;
  int32_t start;
  int32_t idx;
  int32_t pad[2];
};

// Rays in the caller's order. When `recs` is set, the ray walked at position k is recs[k] (binned
// copies, first triangle already decided); else when `order` is set it is ray order[k] (a
// permutation of 0..n-1); otherwise it is ray k.
struct RaysDev {
  const double2* o;
  const double2* d;
  const int32_t* start;
  int32_t* prim;
  double* t;
  int32_t* steps;
  int64_t n;
  const int32_t* order;
  const RayRec* recs;
  // continued rays (trace_bounces): reflections made per ray and the last hit face; hits set
  // selects the continued walk, which writes prim/t/steps itself
  int32_t* hits;
  int32_t* face;
  // rays walked in another order than the caller's (binned): 16-byte result records in the
  // caller's order, turned into prim/t/steps by a coalesced pass after the walk
  double2* park;
  int32_t max_bounces;
  // the step guard: a walk (a segment of a continued ray) that would enter one triangle more than
  // this ends with CCSP_RAY_GUARD; 0 or more than the triangle count means the triangle count
  int32_t max_steps;
};

// One item of a batched launch: the scene, its rays and where its tiles start in the
// concatenated tile sequence.
struct BatchItem {
  SceneDev scene;
  RaysDev rays;
  int64_t tile_begin;
};

struct LaunchCfg {
  int wg;          // threads per workgroup (multiple of 64)
  int tile;        // rays per wave tile (multiple of 64)
  int grid;        // workgroups
  int refill_min;  // idle lanes that trigger a refill
  int chunks;      // the tile sequence is split into this many chunks, one per XCD (1 or 8)
  int group;       // tiles claimed per atomic
};

// Per-device scratch used by the walk: tile counters and the diagnostic counters.
struct Workspace {
  unsigned long long* counters;  // ring of kCounterSlots tile counters
  unsigned long long* stats;     // 4 diagnostic counters
  int* errflags;                 // ring of kCounterSlots / kClaimChunks validation flags, one per
                                 // launch slot of the counter ring
};
constexpr int kCounterSlots = 4096;
constexpr int kClaimChunks = 8;  // tile counters per launch (one per XCD)

// Binning: *out = `in` with a cache-friendly walking order: binned records (out->recs, the
// default) or a sorted index (out->order); see bin.hip. Needs bin_workspace_bytes(n) of scratch.
// `stats`, if not null, receives the first triangles' deferred decisions (as the walk's counters).
enum { kBinBuckets = 0, kBinRadix = 2 };
size_t bin_workspace_bytes(int64_t n);
hipError_t launch_bin_rays(const SceneDev& sc, const RaysDev& in, int kind, void* workspace,
                           size_t ws_bytes, RaysDev* out, unsigned long long* stats,
                           hipStream_t stream);

// A single trace: the walk kernel, then (rays walked in another order than the caller's, i.e.
// io.park set) the copy of the parked results into the caller's arrays (finish_copy).
// `walk_begin` and `walk_end`, if not null, are recorded on `stream` right before and after the
// walk kernel itself (after the small counter reset, before the copy), so that they time it alone.
// `errflag` (validating launches only) receives 1 if a ray fails its precondition.
hipError_t launch_walk(const SceneDev& sc, const RaysDev& io, int mode, bool count, bool validate,
                       const LaunchCfg& cfg, unsigned long long* counter, int* errflag,
                       const Workspace& ws, hipStream_t stream, hipEvent_t walk_begin = nullptr,
                       hipEvent_t walk_end = nullptr);

// A batch: the walk kernel over every item's tiles (it writes every item's results).
hipError_t launch_walk_batch(const BatchItem* items_dev, int n_items, int64_t total_tiles,
                             int mode, bool count, const LaunchCfg& cfg,
                             unsigned long long* counter, const Workspace& ws, hipStream_t stream,
                             hipEvent_t walk_begin = nullptr, hipEvent_t walk_end = nullptr);

size_t walk_lds_bytes(int mode, const LaunchCfg& cfg);

// Point location (locate.hip): walk from the query's seed to each query point.
hipError_t launch_locate(const SceneDev& sc, const double2* q, int64_t n, int32_t* tri,
                         int32_t* status, hipStream_t stream);

// The message last_error() returns on the calling thread.
void set_last_error(const char* msg);

}  // namespace ccsp
