// Persistent stackless triangulation walk for gfx950 (CDNA4, wave64).
//
// Paper: Sec. 5.1 (the walk: find the exit edge, stop on scene geometry or at the hull, else
// continue in the neighbour) and Sec. 5.4 (one operation per visited triangle: choosing the exit
// edge; two candidates once the entry edge is known, three in the first triangle).
//
// Mapping to the hardware:
//  * The walk is a chain of dependent gathers with a few flops each, bound by memory latency and
//    gather bandwidth, not by MFMA or the ALUs. One step is one 16-byte load: the slot of the exit
//    edge holds the neighbour, the entry edge there and the one vertex the next decision needs.
//  * Waves are persistent. Each wave claims tiles of TPL*64 rays from a global counter, stages
//    them in its own LDS region (origin, direction and the first exit slot, computed while the
//    tile is loaded), and refills idle lanes from LDS as soon as `refill_min` of its 64 lanes have
//    finished, so that divergent ray lengths do not idle the SIMD.
//  * Decisions: the sign of D(v) = dx*(vy-oy) - dy*(vx-ox), zero counting as LEFT. In binary32 mode
//    the sign is taken from binary32 coordinates when a forward error bound proves it, otherwise
//    from the binary64 filter, otherwise from an exact expansion; all three agree with the exact
//    sign whenever they decide, so both modes give identical results.
//
// All code here is compiled with -ffp-contract=off: the filters' bounds and the hit distance
// formula assume every operation is rounded separately.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "exact.hpp"
#include "walk.hpp"

namespace ccsp {

// ------------------------------------------------------------------------------ decisions

// binary32 filter. Inputs: origin and across vertex relative to the scene origin and rounded to
// binary32 (relative error <= 2^-24 each, plus 2^-53 from the binary64 subtraction), direction
// rounded to binary32. The rounded evaluation differs from the exact D by at most
// u*|D~| + 4.02u*M, u = 2^-24, M = |dx|(|cy|+|oy|) + |dy|(|cx|+|ox|) (absolute magnitudes: input
// rounding is relative to the coordinates, not to their differences). The threshold 6u*M~ + 2^-100
// covers this with margin, also for subnormal intermediates. Returns +-1 if certain, 0 if not.
struct Ray32 {
  float ox, oy, dx, dy;
};

__device__ __forceinline__ int side32(const Ray32& r, float cx, float cy) {
  const float a = cy - r.oy;
  const float b = cx - r.ox;
  const float D = r.dx * a - r.dy * b;
  const float M = fabsf(r.dx) * (fabsf(cy) + fabsf(r.oy)) + fabsf(r.dy) * (fabsf(cx) + fabsf(r.ox));
  if (fabsf(D) > 0x1.8p-22f * M + 0x1p-100f) return D > 0.0f ? 1 : -1;
  return 0;
}

// Exact decision, kept out of line so that its expansion registers do not count against the
// occupancy of the hot loop.
__device__ __attribute__((noinline)) int side_exact_call(double ox, double oy, double dx, double dy,
                                                         double vx, double vy) {
  return side_exact(ox, oy, dx, dy, vx, vy);
}

template <bool COUNT>
__device__ __forceinline__ bool left64(double ox, double oy, double dx, double dy, double vx,
                                       double vy, unsigned& n_exact) {
  bool certain;
  int s = side_fp64_filtered(ox, oy, dx, dy, vx, vy, certain);
  if (!certain) {
    if (COUNT) ++n_exact;
    s = side_exact_call(ox, oy, dx, dy, vx, vy);
  }
  return s >= 0;
}

struct Counters {
  unsigned steps = 0, fb32 = 0, fb64 = 0, rays = 0;
};

// binary32 decision deferred to binary64 (out of line: rare).
template <bool COUNT>
__device__ __attribute__((noinline)) bool left_deferred(double2 o, double2 d, const double2* v64,
                                                        int vid, unsigned* n_exact) {
  const double2 v = v64[vid];
  unsigned n = 0;
  const bool l = left64<COUNT>(o.x, o.y, d.x, d.y, v.x, v.y, n);
  if (COUNT) *n_exact += n;
  return l;
}

__device__ __attribute__((noinline)) bool validate_ray(const SceneDev& sc, double2 o, double2 d,
                                                       int st) {
  const int4 tv = sc.triv[st];
  const double2 v[3] = {sc.v64[tv.x], sc.v64[tv.y], sc.v64[tv.z]};
  bool ok = isfinite(d.x) && isfinite(d.y) && (d.x != 0.0 || d.y != 0.0) && isfinite(o.x) &&
            isfinite(o.y);
  for (int i = 0; i < 3; ++i) {
    const double2 a = v[(i + 1) % 3], b = v[(i + 2) % 3];
    ok = ok && orient_exact(a.x, a.y, b.x, b.y, o.x, o.y) > 0;
  }
  return ok;
}

// Exit slot of the start triangle (3*st + edge), or -1 if st is out of range, no edge qualifies
// or (VALIDATE) the origin is not strictly inside / the direction is zero or not finite.
// The exit edge i is the one whose first endpoint is RIGHT of the ray and second LEFT.
template <bool COUNT>
__device__ __forceinline__ int first_exit32(const SceneDev& sc, double2 o, double2 d,
                                            const Ray32& r, int st, Counters& c) {
  const float4* p = reinterpret_cast<const float4*>(sc.trixy + st);
  const float4 a = p[0], b = p[1];
  int s0 = side32(r, a.x, a.w), s1 = side32(r, a.y, b.x), s2 = side32(r, a.z, b.y);
  if ((s0 == 0) | (s1 == 0) | (s2 == 0)) {
    const int4 tv = sc.triv[st];
    if (s0 == 0) { if (COUNT) ++c.fb32; s0 = left_deferred<COUNT>(o, d, sc.v64, tv.x, &c.fb64) ? 1 : -1; }
    if (s1 == 0) { if (COUNT) ++c.fb32; s1 = left_deferred<COUNT>(o, d, sc.v64, tv.y, &c.fb64) ? 1 : -1; }
    if (s2 == 0) { if (COUNT) ++c.fb32; s2 = left_deferred<COUNT>(o, d, sc.v64, tv.z, &c.fb64) ? 1 : -1; }
  }
  const bool L0 = s0 > 0, L1 = s1 > 0, L2 = s2 > 0;
  const int e = (!L1 && L2) ? 0 : ((!L2 && L0) ? 1 : ((!L0 && L1) ? 2 : -1));
  return e < 0 ? -1 : 3 * st + e;
}

template <bool COUNT>
__device__ __forceinline__ int first_exit64(const SceneDev& sc, double2 o, double2 d, int st,
                                            Counters& c) {
  const int4 tv = sc.triv[st];
  const double2 v0 = sc.v64[tv.x], v1 = sc.v64[tv.y], v2 = sc.v64[tv.z];
  const bool L0 = left64<COUNT>(o.x, o.y, d.x, d.y, v0.x, v0.y, c.fb64);
  const bool L1 = left64<COUNT>(o.x, o.y, d.x, d.y, v1.x, v1.y, c.fb64);
  const bool L2 = left64<COUNT>(o.x, o.y, d.x, d.y, v2.x, v2.y, c.fb64);
  const int e = (!L1 && L2) ? 0 : ((!L2 && L0) ? 1 : ((!L0 && L1) ? 2 : -1));
  return e < 0 ? -1 : 3 * st + e;
}

__device__ __forceinline__ double hit_t(const double4 g, double ox, double oy, double dx,
                                        double dy) {
  const double ex = g.z - g.x;
  const double ey = g.w - g.y;
  const double num = (g.x - ox) * ey - (g.y - oy) * ex;
  const double den = dx * ey - dy * ex;
  return num / den;
}

// ------------------------------------------------------------------------------ persistent walk

__device__ __forceinline__ int lane_rank(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ long long bcast64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ void wave_lds_fence() {
  // A wave's LDS operations execute in order; this only stops the compiler from moving the
  // reads of a freshly written tile above the writes.
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-wave LDS tile: the ray (2 x double2), its first exit slot and its index, 40 B/ray.
template <int TILE>
struct Tile {
  static constexpr int kBytes = 40 * TILE;
  double2* o;
  double2* d;
  int* s0;
  int* idx;
  __device__ explicit Tile(unsigned char* base)
      : o(reinterpret_cast<double2*>(base)),
        d(reinterpret_cast<double2*>(base + 16 * TILE)),
        s0(reinterpret_cast<int*>(base + 32 * TILE)),
        idx(reinterpret_cast<int*>(base + 36 * TILE)) {}
};

// Load rays [base, base+len) of `io` into the tile and compute their first exit slots.
template <int MODE, int TPL, bool COUNT, bool VALIDATE>
__device__ void fill_tile(const SceneDev& sc, const RaysDev& io, int64_t base, int len,
                          const Tile<TPL * 64>& tl, int lane, Counters& c, int* errflag) {
  // phase 1: all loads of the tile in flight together
  int st[TPL];
  int64_t ri[TPL];
  double2 o[TPL], d[TPL];
  const bool internal = io.recs != nullptr || io.order_start != nullptr;
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    st[q] = -1;
    ri[q] = base + k;
    if (k < len) {
      if (io.recs) {  // binned copies, read contiguously
        const RayRec* r = io.recs + base + k;
        o[q] = r->o;
        d[q] = r->d;
        const int2 si = *reinterpret_cast<const int2*>(&r->start);
        st[q] = si.x;
        ri[q] = si.y;
      } else {
        if (io.order) ri[q] = io.order[base + k];
        o[q] = io.o[ri[q]];
        d[q] = io.d[ri[q]];
        st[q] = io.order_start ? io.order_start[base + k] : io.start[ri[q]];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    if (k < len) {
      if (internal) {
        if (st[q] >= sc.ntri) st[q] = -1;  // already an internal id (binning mapped it)
      } else {
        // the caller's triangle id -> internal (Hilbert-ordered) id
        st[q] = (st[q] >= 0 && st[q] < sc.ntri) ? sc.perm[st[q]] : -1;
      }
      tl.o[k] = o[q];
      tl.d[k] = d[q];
      tl.idx[k] = (int)ri[q];
      if (VALIDATE && (st[q] < 0 || !validate_ray(sc, o[q], d[q], st[q]))) {
        atomicOr(errflag, 1);
        st[q] = -1;
      }
    }
  }
  // phase 2: first triangle of each ray
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    if (k < len) {
      int s0 = -1;
      if (st[q] >= 0) {
        if (MODE == 1) {
          const Ray32 rr{(float)(o[q].x - sc.org_x), (float)(o[q].y - sc.org_y), (float)d[q].x,
                         (float)d[q].y};
          s0 = first_exit32<COUNT>(sc, o[q], d[q], rr, st[q], c);
        } else {
          s0 = first_exit64<COUNT>(sc, o[q], d[q], st[q], c);
        }
      }
      tl.s0[k] = s0;
    }
  }
  wave_lds_fence();
}

// Scene access in a batched launch.
struct ItemRef {
  const BatchItem* items;
  int n_items;
  const int64_t* lds_tile_begin;  // tile_begin of the first n_lds items, staged in LDS
  int n_lds;
};

// Claim the next tile of [0, total): the sequence is split into `chunks` contiguous chunks with a
// counter each; a workgroup starts in chunk blockIdx.x % chunks (workgroups are dispatched to the
// XCDs round-robin, so with 8 chunks each XCD walks its own part of the binned rays and keeps its
// own region of the scene in its L2) and moves on to the next chunk once one is exhausted.
// Returns -1 when every chunk is exhausted. Wave-uniform.
__device__ __forceinline__ long long claim_tile(unsigned long long* counter, int chunks,
                                                long long total, int& cur, int& tried, int lane) {
  while (tried < chunks) {
    const long long c0 = total * cur / chunks, c1 = total * (cur + 1) / chunks;
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(counter + cur, 1ull);
    const long long t = c0 + bcast64(b);
    if (t < c1) return t;
    cur = cur + 1 == chunks ? 0 : cur + 1;
    ++tried;
  }
  return -1;
}

template <int MODE, int TPL, bool COUNT, bool VALIDATE, bool BATCH>
__global__ void __launch_bounds__(512)
walk_persistent(SceneDev sc_arg, RaysDev io_arg, ItemRef batch, int64_t total_tiles,
                unsigned long long* __restrict__ counter, int refill_min, int chunks,
                unsigned long long* __restrict__ stats, int* __restrict__ errflag) {
  constexpr int TILE = TPL * 64;
  extern __shared__ unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  unsigned char* tile_mem = lds;
  if (BATCH) {
    // stage the items' first tiles in LDS for the tile -> item search
    int64_t* tb = reinterpret_cast<int64_t*>(lds);
    for (int i = threadIdx.x; i < batch.n_lds; i += blockDim.x) tb[i] = batch.items[i].tile_begin;
    __syncthreads();
    batch.lds_tile_begin = tb;
    tile_mem = lds + (size_t)((batch.n_lds + 1) & ~1) * 8;
  }
  const Tile<TILE> tl(tile_mem + (size_t)wave * Tile<TILE>::kBytes);

  Counters c;
  // lane state: IDLE (no ray), WALK (s is the exit slot to load), FIN (hit primitive p to load)
  enum : int { IDLE = 0, WALK = 1, FIN = 2 };
  int state = IDLE;
  Ray32 r32{0, 0, 0, 0};                  // binary32 mode
  double ox = 0, oy = 0, dx = 0, dy = 0;  // the ray in binary64
  int s = 0, steps = 0;
  int64_t ray = 0;
  int item = 0;
  // per-lane scene in a batch, kernel argument otherwise
  const Slot32* slot32 = sc_arg.slot32;
  const Slot64* slot64 = sc_arg.slot64;
  int ntri = sc_arg.ntri;

  // wave-uniform tile state
  int64_t tbase = 0;
  int tlen = 0, thead = 0, titem = 0;
  bool drained = false;
  bool io_order = io_arg.order != nullptr || io_arg.recs != nullptr;
  int chunk_cur = (int)(blockIdx.x % (unsigned)chunks), chunk_tried = 0;

  for (;;) {
    const unsigned long long idle = __ballot(state == IDLE);
    const int nidle = __popcll(idle);
    if (drained && nidle == 64) break;
    if (!drained && nidle >= refill_min) {
      const int rank = lane_rank(idle);
      int served = 0;
      while (served < nidle) {
        if (thead == tlen) {
          const long long claim = claim_tile(counter, chunks, total_tiles, chunk_cur, chunk_tried, lane);
          if (claim < 0) {
            drained = true;
            break;
          }
          if (BATCH) {
            // item owning tile `claim`: the last item whose tile_begin <= claim
            int lo = 0, hi = batch.n_items - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              const int64_t tbm = mid < batch.n_lds ? batch.lds_tile_begin[mid]
                                                    : batch.items[mid].tile_begin;
              if (tbm <= claim) lo = mid;
              else hi = mid - 1;
            }
            titem = __builtin_amdgcn_readfirstlane(lo);
            const BatchItem& it = batch.items[titem];
            tbase = (claim - it.tile_begin) * TILE;
            tlen = (int)min((int64_t)TILE, it.rays.n - tbase);
            thead = 0;
            io_order = it.rays.order != nullptr || it.rays.recs != nullptr;
            fill_tile<MODE, TPL, COUNT, false>(it.scene, it.rays, tbase, tlen, tl, lane, c, errflag);
          } else {
            tbase = claim * TILE;
            tlen = (int)min((int64_t)TILE, io_arg.n - tbase);
            thead = 0;
            fill_tile<MODE, TPL, COUNT, VALIDATE>(sc_arg, io_arg, tbase, tlen, tl, lane, c, errflag);
          }
        }
        const int take = min(nidle - served, tlen - thead);
        if (state == IDLE && rank >= served && rank < served + take) {
          const int k = thead + (rank - served);
          {
            const double2 o = tl.o[k], d = tl.d[k];
            ox = o.x; oy = o.y; dx = d.x; dy = d.y;
          }
          s = tl.s0[k];
          ray = io_order ? (int64_t)tl.idx[k] : tbase + k;
          steps = 1;
          state = WALK;
          double org_x = sc_arg.org_x, org_y = sc_arg.org_y;
          if (BATCH) {
            item = titem;
            const SceneDev& sc = batch.items[item].scene;
            slot32 = sc.slot32;
            slot64 = sc.slot64;
            ntri = sc.ntri;
            org_x = sc.org_x;
            org_y = sc.org_y;
          }
          if (MODE == 1) r32 = Ray32{(float)(ox - org_x), (float)(oy - org_y), (float)dx, (float)dy};
          if (s < 0) {  // bad ray: out-of-range start, no exit edge, or failed validation
            const RaysDev& io = BATCH ? batch.items[item].rays : io_arg;
            io.prim[ray] = -3;
            io.t[ray] = INFINITY;
            io.steps[ray] = 0;
            state = IDLE;
          }
        }
        served += take;
        thead += take;
      }
    }
    // Issue this iteration's loads before using any: a walking lane loads its exit slot, a
    // finishing lane its hit primitive, so both share one memory round trip.
    const int st_now = state;
    int4 q = make_int4(0, 0, 0, 0);
    double2 xy64 = make_double2(0.0, 0.0);
    double2 ga = make_double2(0.0, 0.0), gb = make_double2(0.0, 0.0);
    int gid = 0;
    if (st_now == WALK) {
      if (MODE == 1) {
        q = *reinterpret_cast<const int4*>(slot32 + s);
        // Keep the slot one 16-byte load: without this the compiler loads the exit word alone,
        // branches on it and only then loads the vertex, a second dependent round trip.
        __asm__ volatile("" ::"v"(q.x), "v"(q.y), "v"(q.z), "v"(q.w));
      } else {
        xy64 = *reinterpret_cast<const double2*>(slot64 + s);
        q.x = *reinterpret_cast<const int*>(&slot64[s].word);
        __asm__ volatile("" ::"v"(xy64.x), "v"(xy64.y), "v"(q.x));
      }
    } else if (st_now == FIN) {
      const PrimRec* prim = BATCH ? batch.items[item].scene.prim : sc_arg.prim;
      const PrimRec* g = prim + s;
      ga = *reinterpret_cast<const double2*>(&g->ax);
      gb = *reinterpret_cast<const double2*>(&g->bx);
      gid = g->id;
      __asm__ volatile("" ::"v"(ga.x), "v"(ga.y), "v"(gb.x), "v"(gb.y), "v"(gid));
    }
    if (st_now == WALK) {
      const int word = q.x;
      bool left = false;
      if (word >= 0) {
        if (MODE == 1) {
          const int sg = side32(r32, __int_as_float(q.y), __int_as_float(q.z));
          if (sg != 0) {
            left = sg > 0;
          } else {
            if (COUNT) ++c.fb32;
            const double2* v64 = BATCH ? batch.items[item].scene.v64 : sc_arg.v64;
            left = left_deferred<COUNT>(make_double2(ox, oy), make_double2(dx, dy), v64, q.w, &c.fb64);
          }
        } else {
          left = left64<COUNT>(ox, oy, dx, dy, xy64.x, xy64.y, c.fb64);
        }
      }
      if (word >= 0 && steps < ntri) {
        ++steps;
        int e = (word & 3) + (left ? 1 : 2);
        e = e >= 3 ? e - 3 : e;
        s = 3 * (word >> 2) + e;
      } else if (word <= -2) {
        s = -word - 2;  // constrained edge: hit; its primitive is loaded next iteration
        state = FIN;
      } else {
        // hull edge (miss) or the step guard
        const RaysDev& io = BATCH ? batch.items[item].rays : io_arg;
        io.prim[ray] = word >= 0 ? -2 : -1;
        io.t[ray] = INFINITY;
        io.steps[ray] = steps;
        if (COUNT) {
          c.steps += steps;
          ++c.rays;
        }
        state = IDLE;
      }
    } else if (st_now == FIN) {
      const RaysDev& io = BATCH ? batch.items[item].rays : io_arg;
      io.prim[ray] = gid;
      io.t[ray] = hit_t(make_double4(ga.x, ga.y, gb.x, gb.y), ox, oy, dx, dy);
      io.steps[ray] = steps;
      if (COUNT) {
        c.steps += steps;
        ++c.rays;
      }
      state = IDLE;
    }
  }
  if (COUNT) {
    if (c.steps) atomicAdd(&stats[0], (unsigned long long)c.steps);
    if (c.fb32) atomicAdd(&stats[1], (unsigned long long)c.fb32);
    if (c.fb64) atomicAdd(&stats[2], (unsigned long long)c.fb64);
    if (c.rays) atomicAdd(&stats[3], (unsigned long long)c.rays);
  }
}

__global__ void reset_counters(unsigned long long* counter) {
  if (threadIdx.x < kClaimChunks) counter[threadIdx.x] = 0ull;
}

// ------------------------------------------------------------------------------ launchers

size_t walk_lds_bytes(int mode, const LaunchCfg& cfg) {
  (void)mode;
  return (size_t)(cfg.wg / 64) * cfg.tile * 40;
}

template <int MODE, int TPL, bool COUNT, bool VALIDATE, bool BATCH>
static hipError_t go(const SceneDev& sc, const RaysDev& io, ItemRef br, int64_t total_tiles,
                     const LaunchCfg& cfg, size_t lds, unsigned long long* counter,
                     const Workspace& ws, hipStream_t stream) {
  hipLaunchKernelGGL((walk_persistent<MODE, TPL, COUNT, VALIDATE, BATCH>), dim3(cfg.grid),
                     dim3(cfg.wg), lds, stream, sc, io, br, total_tiles, counter, cfg.refill_min,
                     cfg.chunks, ws.stats, ws.errflag);
  return hipGetLastError();
}

template <int MODE, bool COUNT, bool VALIDATE, bool BATCH>
static hipError_t pick_tile(const SceneDev& sc, const RaysDev& io, ItemRef br, int64_t total_tiles,
                            const LaunchCfg& cfg, size_t lds, unsigned long long* counter,
                            const Workspace& ws, hipStream_t stream) {
  switch (cfg.tile) {
    case 64: return go<MODE, 1, COUNT, VALIDATE, BATCH>(sc, io, br, total_tiles, cfg, lds, counter, ws, stream);
    case 128: return go<MODE, 2, COUNT, VALIDATE, BATCH>(sc, io, br, total_tiles, cfg, lds, counter, ws, stream);
    case 256: return go<MODE, 4, COUNT, VALIDATE, BATCH>(sc, io, br, total_tiles, cfg, lds, counter, ws, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_walk(const SceneDev& sc, const RaysDev& io, int mode, bool count, bool validate,
                       const LaunchCfg& cfg, unsigned long long* counter, const Workspace& ws,
                       hipStream_t stream) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counter);
  const size_t lds = walk_lds_bytes(mode, cfg);
  const ItemRef none{nullptr, 0, nullptr, 0};
  const int64_t tiles = (io.n + cfg.tile - 1) / cfg.tile;
#define CCSP_CASE(M, C, V) \
  if (mode == M && count == C && validate == V) \
    return pick_tile<M, C, V, false>(sc, io, none, tiles, cfg, lds, counter, ws, stream);
  CCSP_CASE(0, false, false) CCSP_CASE(0, true, false) CCSP_CASE(0, false, true) CCSP_CASE(0, true, true)
  CCSP_CASE(1, false, false) CCSP_CASE(1, true, false) CCSP_CASE(1, false, true) CCSP_CASE(1, true, true)
#undef CCSP_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_walk_batch(const BatchItem* items_dev, int n_items, int64_t total_tiles,
                             int mode, bool count, const LaunchCfg& cfg,
                             unsigned long long* counter, const Workspace& ws, hipStream_t stream) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counter);
  const int n_lds = n_items < 1024 ? n_items : 1024;
  const size_t lds = walk_lds_bytes(mode, cfg) + (size_t)((n_lds + 1) & ~1) * 8;
  const ItemRef br{items_dev, n_items, nullptr, n_lds};
  const SceneDev nosc{};
  const RaysDev noio{};
  if (mode == 0 && !count) return pick_tile<0, false, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, stream);
  if (mode == 0 && count) return pick_tile<0, true, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, stream);
  if (mode == 1 && !count) return pick_tile<1, false, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, stream);
  if (mode == 1 && count) return pick_tile<1, true, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, stream);
  return hipErrorInvalidValue;
}

}  // namespace ccsp
