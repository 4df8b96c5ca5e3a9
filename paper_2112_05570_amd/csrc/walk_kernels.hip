// Persistent stackless triangulation walk for gfx950 (CDNA4, wave64).
//
// Paper: Sec. 5.1 (the walk: find the exit edge, stop on scene geometry or at the hull, else
// continue in the neighbour), Sec. 5.4 (one operation per visited triangle: choosing the exit
// edge) and the footnote of Sec. 7.2 (two candidates once the entry edge is known, three in the
// first triangle).
//
// Mapping to the hardware:
//  * The walk is a chain of dependent gathers with a few flops each, bound by memory latency and
//    gather bandwidth, not by MFMA or the ALUs. One step is one 16-byte load: the slot of the exit
//    edge holds the neighbour, the entry edge there and the one vertex the next decision needs.
//  * Waves are persistent. Each wave claims tiles of TPL*64 rays from global counters (one per
//    XCD), stages them in its own LDS region (origin, direction, and the start triangle or, for
//    binned rays, the first exit slot) and refills idle lanes from LDS as soon as `refill_min` of
//    its 64 lanes have finished, so that divergent ray lengths do not idle the SIMD.
//  * A trace finishes in a second kernel, in input order with coalesced accesses, because the
//    caller's three result arrays would take three scattered stores per ray from the walk.
//    Binned rays (walked in another order than the caller's): a hit frees the lane at once, but
//    the lane keeps the ray and the primitive as a pending hit, fetches the primitive's segment in
//    the next iteration's load round (which the wave makes anyway, for its other lanes or the
//    lane's next ray), computes t and parks a 16-byte record (t, primitive, steps) per ray;
//    binned rays hit the primitives of one region at a time, so that fetch mostly hits in L2.
//    finish_copy then copies the records into the caller's arrays. Rays walked in input order
//    (batches, unbinned traces) park only (primitive, steps) in the ray's 8-byte hit_t slot and
//    finish_rays / finish_batch compute t there, since their hits gather primitives at random
//    either way.
//  * Decisions: the sign of D(v) = dx*(vy-oy) - dy*(vx-ox), zero counting as LEFT. In binary32 mode
//    the sign is taken from binary32 coordinates when a forward error bound proves it, otherwise
//    from the binary64 filter, otherwise from an exact expansion; all three agree with the exact
//    sign whenever they decide, so both modes give identical results.
//
// All code here is compiled with -ffp-contract=off: the filters' bounds and the hit distance
// formula assume every operation is rounded separately.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "decide.hpp"
#include "exact.hpp"
#include "walk.hpp"

namespace ccsp {

// Exact check of a ray's precondition: finite nonzero direction, finite origin strictly inside
// internal triangle `st`.
static __device__ __attribute__((noinline)) bool validate_ray(const SceneDev& sc, double2 o,
                                                              double2 d, int st) {
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

// ------------------------------------------------------------------------------ persistent walk

// Result of a ray walked in input order, as left for finish_rays / finish_batch: x = the caller's
// primitive id (>= 0) or a CCSP_RAY_* code, y = steps; stored in the ray's hit_t slot (8 bytes),
// non-temporally: it is read back once, by the finishing pass.
__device__ __forceinline__ void park_result(const RaysDev& io, int64_t ray, int code, int steps) {
  __builtin_nontemporal_store(((unsigned long long)(unsigned)steps << 32) | (unsigned)code,
                              reinterpret_cast<unsigned long long*>(io.t) + ray);
}

// Result of a binned ray, t included, as left for finish_copy: one 16-byte record at io.park[ray].
__device__ __forceinline__ void park_record(const RaysDev& io, int64_t ray, int code, double t,
                                            int steps) {
  typedef long long vl2 __attribute__((ext_vector_type(2)));
  vl2 v;
  v.x = __double_as_longlong(t);
  v.y = (long long)(((unsigned long long)(unsigned)steps << 32) | (unsigned)code);
  __builtin_nontemporal_store(v, reinterpret_cast<vl2*>(io.park) + ray);
}

// A ray that ends without a hit (a CCSP_RAY_* code).
__device__ __forceinline__ void park_code(const RaysDev& io, int64_t ray, int code, int steps) {
  if (io.park)
    park_record(io, ray, code, INFINITY, steps);
  else
    park_result(io, ray, code, steps);
}

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

// Per-wave LDS tile: the ray (2 x double2), its internal start triangle and its index, 40 B/ray.
template <int TILE>
struct Tile {
  static constexpr int kBytes = 40 * TILE;
  double2* o;
  double2* d;
  int* st;
  int* idx;
  __device__ explicit Tile(unsigned char* base)
      : o(reinterpret_cast<double2*>(base)),
        d(reinterpret_cast<double2*>(base + 16 * TILE)),
        st(reinterpret_cast<int*>(base + 32 * TILE)),
        idx(reinterpret_cast<int*>(base + 36 * TILE)) {}
};

// Load rays [base, base+len) of `io` into the tile, one round of loads. A binned tile (io.recs)
// holds each ray's first exit slot (binning decided the first triangle), any other tile the
// caller's start triangle, whose first triangle the walk loop decides; -1 marks a bad ray.
template <int TPL, bool VALIDATE>
__device__ void fill_tile(const SceneDev& sc, const RaysDev& io, int64_t base, int len,
                          const Tile<TPL * 64>& tl, int lane, int* errflag) {
  int st[TPL];
  int64_t ri[TPL];
  double2 o[TPL], d[TPL];
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
        st[q] = io.start[ri[q]];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    if (k < len) {
      if (io.recs) {
        if (st[q] >= 3 * sc.ntri) st[q] = -1;
      } else if (st[q] >= sc.ntri) {
        st[q] = -1;
      }
      if (VALIDATE && (st[q] < 0 ||
                       !validate_ray(sc, o[q], d[q], io.recs ? st[q] / 3 : sc.first[st[q]].tri))) {
        atomicOr(errflag, 1);
        st[q] = -1;
      }
      tl.o[k] = o[q];
      tl.d[k] = d[q];
      tl.st[k] = st[q];
      tl.idx[k] = (int)ri[q];
    }
  }
  wave_lds_fence();
}

// Results of a continued (reflecting) ray, written directly: its last segment's primitive or
// code, t, the triangles visited over all segments, the reflections made, the last hit face.
__device__ __forceinline__ void bounce_result(const RaysDev& io, int64_t ray, int code, double t,
                                              int steps, int hits, int face) {
  io.prim[ray] = code;
  io.t[ray] = t;
  io.steps[ray] = steps;
  io.hits[ray] = hits;
  if (io.face) io.face[ray] = face;
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

// Each lane is a small state machine that issues exactly one round of loads per iteration:
//   FIRST: the start triangle's first-triangle record (then three decisions, the first
//          step of Sec. 7.2's footnote; rays of binned tiles skip it: binning decided their first triangle),
//   WALK:  the two-step record of the exit edge (Pair32 or Pair64: then one decision for the
//          neighbour across that edge and, unless its exit ends the walk, one for the triangle
//          after it; the one-step slots are read only for rare fallbacks and at hits),
// so lanes in different states share one memory round trip, and a refilled lane starts walking
// in the next iteration without a separate gather phase.
// BOUNCE: rays continue by specular reflection at hits (up to io.max_bounces times): a fourth
// state loads the hit primitive and the hit triangle's vertex opposite the hit edge, computes t
// and either reflects the ray, which then enters the same triangle through the hit edge (Sec.
// 5.2: the final triangle of a traversal starts the secondary ray), or writes the results.
template <int MODE, int TPL, bool COUNT, bool VALIDATE, bool BATCH, bool BOUNCE>
__global__ void __launch_bounds__(512)
walk_persistent(SceneDev sc_arg, RaysDev io_arg, ItemRef batch, int64_t total_tiles,
                unsigned long long* __restrict__ counter, int refill_min, int chunks, int group,
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
  enum : int { IDLE = 0, FIRST = 1, WALK = 2, BNC = 3 };
  int state = IDLE;
  Ray32 r32{0, 0, 0, 0};                  // binary32 mode
  double ox = 0, oy = 0, dx = 0, dy = 0;  // the ray in binary64
  int s = 0, steps = 0;                   // s: start triangle (FIRST), exit slot (WALK), prim (BNC)
  int nb = 0, seg = 0, hs = 0, cv = 0;    // BOUNCE: reflections, steps of this segment, hit slot,
                                          // vertex opposite the hit edge
  int64_t ray = 0;
  int item = 0;
  // a binned ray's hit waiting for its primitive's segment: ray, primitive, steps and the ray
  // itself (a refill in the same iteration replaces ox..dy)
  constexpr bool PEND = !BOUNCE && !BATCH;
  const bool parked = PEND && io_arg.park != nullptr;
  int64_t pray = -1;
  int pprim = 0, psteps = 0;
  double pox = 0, poy = 0, pdx = 0, pdy = 0;
  // per-lane scene in a batch, kernel argument otherwise
  const Slot32* slot32 = sc_arg.slot32;
  const Pair32* pair32 = sc_arg.pair32;
  const Pair64* pair64 = sc_arg.pair64;
  // the step guard's limit: the triangle count, or the caller's smaller limit
  int ntri = sc_arg.ntri;
  if (!BATCH && io_arg.max_steps > 0 && io_arg.max_steps < ntri) ntri = io_arg.max_steps;

  // wave-uniform tile state
  int64_t tbase = 0;
  int tlen = 0, thead = 0, titem = 0;
  bool drained = false;
  bool io_order = io_arg.order != nullptr || io_arg.recs != nullptr;
  // rays of binned tiles start walking at once: binning decided their first triangle
  const bool binned = !BATCH && io_arg.recs != nullptr;
  int chunk_cur = (int)(blockIdx.x % (unsigned)chunks), chunk_tried = 0;
  // tiles are claimed `group` at a time (one global atomic per group): same-address atomics
  // from thousands of waves serialise, and one per tile would stall every refill
  const long long total_groups = (total_tiles + group - 1) / group;
  long long grp_next = 0, grp_end = 0;

  for (;;) {
    const unsigned long long idle = __ballot(state == IDLE);
    const int nidle = __popcll(idle);
    if (drained && nidle == 64 && (!PEND || __ballot(pray >= 0) == 0)) break;
    if (!drained && nidle >= refill_min) {
      const int rank = lane_rank(idle);
      int served = 0;
      while (served < nidle) {
        if (thead == tlen) {
          if (grp_next == grp_end) {
            const long long g = claim_tile(counter, chunks, total_groups, chunk_cur, chunk_tried, lane);
            if (g < 0) {
              drained = true;
              break;
            }
            grp_next = g * group;
            grp_end = min(grp_next + group, (long long)total_tiles);
          }
          const long long claim = grp_next++;
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
            fill_tile<TPL, false>(it.scene, it.rays, tbase, tlen, tl, lane, errflag);
          } else {
            tbase = claim * TILE;
            tlen = (int)min((int64_t)TILE, io_arg.n - tbase);
            thead = 0;
            fill_tile<TPL, VALIDATE>(sc_arg, io_arg, tbase, tlen, tl, lane, errflag);
          }
        }
        const int take = min(nidle - served, tlen - thead);
        if (state == IDLE && rank >= served && rank < served + take) {
          const int k = thead + (rank - served);
          {
            const double2 o = tl.o[k], d = tl.d[k];
            ox = o.x; oy = o.y; dx = d.x; dy = d.y;
          }
          s = tl.st[k];
          ray = io_order ? (int64_t)tl.idx[k] : tbase + k;
          steps = 1;
          if (BOUNCE) {
            nb = 0;
            seg = 1;
          }
          state = binned ? WALK : FIRST;
          double org_x = sc_arg.org_x, org_y = sc_arg.org_y;
          if (BATCH) {
            item = titem;
            const SceneDev& sc = batch.items[item].scene;
            slot32 = sc.slot32;
            pair32 = sc.pair32;
            pair64 = sc.pair64;
            ntri = sc.ntri;
            const int lim = batch.items[item].rays.max_steps;
            if (lim > 0 && lim < ntri) ntri = lim;
            org_x = sc.org_x;
            org_y = sc.org_y;
          }
          if (MODE == 1 || !binned) r32 = ray32(ox, oy, dx, dy, org_x, org_y);
          if (s < 0) {  // bad ray: out-of-range start or failed validation
            if (BOUNCE)
              bounce_result(io_arg, ray, -3, INFINITY, 0, 0, -1);
            else
              park_code(BATCH ? batch.items[item].rays : io_arg, ray, -3, 0);
            state = IDLE;
          }
        }
        served += take;
        thead += take;
      }
    }
    // ---- issue: one round of loads for every busy lane, whatever its state
    const int st_now = state;
    int4 R0 = make_int4(0, 0, 0, 0), R1 = R0, R2 = R0, RW = R0;
    int R3 = 0;
    if (st_now == WALK) {
      if (MODE == 1) {
        const int4* p = reinterpret_cast<const int4*>(pair32 + s);
        R0 = p[0];
        R1 = p[1];
      } else {
        const int4* p = reinterpret_cast<const int4*>(pair64 + s);
        R0 = p[0];
        R1 = p[1];
        R2 = p[2];
        RW = p[3];
      }
    } else if (st_now == FIRST) {
      const int4* p = reinterpret_cast<const int4*>((BATCH ? batch.items[item].scene.first : sc_arg.first) + s);
      R0 = p[0];
      R1 = p[1];
    } else if (BOUNCE && st_now == BNC) {
      const int4* p = reinterpret_cast<const int4*>(sc_arg.prim + s);
      R0 = p[0];
      R1 = p[1];
      R2 = *reinterpret_cast<const int4*>(sc_arg.v64 + cv);
      if (nb >= io_arg.max_bounces && io_arg.face) R3 = sc_arg.orig[hs / 3];
    }
    int4 P0 = make_int4(0, 0, 0, 0), P1 = P0;  // the pending hit's primitive record
    if (PEND && pray >= 0) {
      const int4* p = reinterpret_cast<const int4*>(sc_arg.prim + pprim);
      P0 = p[0];
      P1 = p[1];
    }
    // every load above is issued before any result is used (and none is split per field)
    __asm__ volatile("" ::"v"(R0.x), "v"(R0.y), "v"(R0.z), "v"(R0.w), "v"(R1.x), "v"(R1.y),
                     "v"(R1.z), "v"(R1.w));
    if (PEND)
      __asm__ volatile("" ::"v"(P0.x), "v"(P0.y), "v"(P0.z), "v"(P0.w), "v"(P1.x), "v"(P1.y),
                       "v"(P1.z), "v"(P1.w));
    if (BOUNCE || MODE == 0)
      __asm__ volatile("" ::"v"(R2.x), "v"(R2.y), "v"(R2.z), "v"(R2.w), "v"(R3));
    if (MODE == 0) __asm__ volatile("" ::"v"(RW.x), "v"(RW.y));
    // ---- process
    if (PEND && pray >= 0) {  // the pending hit: t from the primitive's own segment
      const double th = hit_t(make_double4(lohi(P0.x, P0.y), lohi(P0.z, P0.w), lohi(P1.x, P1.y),
                                           lohi(P1.z, P1.w)),
                              pox, poy, pdx, pdy);
      park_record(io_arg, pray, pprim, th, psteps);
      pray = -1;
    }
    if (st_now == WALK) {
      // Pair32 of exit slot s: nx ny w0 x0 | y0 w1 x1 y1; Pair64: nx ny | x0 y0 | x1 y1 | w0 w1.
      // Up to two triangles per load: n (across slot s) and, unless n's exit is constrained or
      // on the hull, the triangle after it.
      const bool terminal = MODE == 1 ? isnan(__int_as_float(R0.x)) : isnan(lohi(R0.x, R0.y));
      int word = MODE == 1 ? R0.z : RW.x;  // the word that ends the walk, if it ends here
      int end_slot = s;  // the slot whose word that is
      bool more = false, left = false;
      if (!terminal && (BOUNCE ? seg < ntri : steps < ntri)) {
        ++steps;  // in n
        if (BOUNCE) ++seg;
        if (MODE == 1) {
          const int sg = side32(r32, __int_as_float(R0.x), __int_as_float(R0.y));
          if (sg != 0) {
            left = sg > 0;
          } else {
            if (COUNT) ++c.fb32;
            const double2* v64 = BATCH ? batch.items[item].scene.v64 : sc_arg.v64;
            left = left_deferred<COUNT>(make_double2(ox, oy), make_double2(dx, dy), v64,
                                        slot32[s].vid, &c.fb64);
          }
          word = left ? R0.z : R1.y;
        } else {
          left = left64<COUNT>(ox, oy, dx, dy, lohi(R0.x, R0.y), lohi(R0.z, R0.w), c.fb64);
          word = left ? RW.x : RW.y;
        }
        end_slot = -1;  // n's exit slot, found from the one-step slot when needed
        if (word >= 0 && (BOUNCE ? seg < ntri : steps < ntri)) {
          ++steps;  // in the triangle after n
          if (BOUNCE) ++seg;
          bool left2;
          if (MODE == 1) {
            const float cx = __int_as_float(left ? R0.w : R1.z);
            const float cy = __int_as_float(left ? R1.x : R1.w);
            const int sg2 = side32(r32, cx, cy);
            if (sg2 != 0) {
              left2 = sg2 > 0;
            } else {
              if (COUNT) ++c.fb32;
              // the across vertex of n's exit slot: n and its entry edge from the one-step slot
              const int wn = slot32[s].word;
              int en = (wn & 3) + (left ? 1 : 2);
              en = en >= 3 ? en - 3 : en;
              const double2* v64 = BATCH ? batch.items[item].scene.v64 : sc_arg.v64;
              left2 = left_deferred<COUNT>(make_double2(ox, oy), make_double2(dx, dy), v64,
                                           slot32[3 * (wn >> 2) + en].vid, &c.fb64);
            }
          } else {
            const double cx = left ? lohi(R1.x, R1.y) : lohi(R2.x, R2.y);
            const double cy = left ? lohi(R1.z, R1.w) : lohi(R2.z, R2.w);
            left2 = left64<COUNT>(ox, oy, dx, dy, cx, cy, c.fb64);
          }
          int e = (word & 3) + (left2 ? 1 : 2);
          e = e >= 3 ? e - 3 : e;
          s = 3 * (word >> 2) + e;
          more = true;
        }
      } else if (!terminal) {
        word = 0;  // the step guard: another triangle to enter
      }
      if (!more) {
        if (BOUNCE && word <= -2) {
          // hit: the primitive and the vertex opposite the hit edge are loaded next iteration
          if (end_slot < 0) {
            const int wn = slot32[s].word;
            int en = (wn & 3) + (left ? 1 : 2);
            en = en >= 3 ? en - 3 : en;
            end_slot = 3 * (wn >> 2) + en;
          }
          hs = end_slot;
          cv = slot32[hs].vid;
          s = -word - 2;
          state = BNC;
        } else if (BOUNCE) {  // hull edge (miss) or the step guard
          bounce_result(io_arg, ray, word >= 0 ? -2 : -1, INFINITY, steps, nb, -1);
          if (COUNT) {
            c.steps += steps;
            ++c.rays;
          }
          state = IDLE;
        } else if (parked && word <= -2) {
          // constrained edge: a hit of primitive -word - 2, finished in the next iteration
          pray = ray;
          pprim = -word - 2;
          psteps = steps;
          pox = ox;
          poy = oy;
          pdx = dx;
          pdy = dy;
          if (COUNT) {
            c.steps += steps;
            ++c.rays;
          }
          state = IDLE;
        } else {
          // constrained edge (hit, primitive -word - 2; t from the finishing pass), hull edge
          // (miss) or the step guard
          const int code = word <= -2 ? -word - 2 : (word >= 0 ? -2 : -1);
          if (parked)
            park_record(io_arg, ray, code, INFINITY, steps);
          else
            park_result(BATCH ? batch.items[item].rays : io_arg, ray, code, steps);
          if (COUNT) {
            c.steps += steps;
            ++c.rays;
          }
          state = IDLE;
        }
      }
    } else if (st_now == FIRST) {
      // TriFirst: x0 x1 x2 y0 | y1 y2 tri -
      const int e = first_exit_slot<COUNT>(
          r32, make_double2(ox, oy), make_double2(dx, dy), __int_as_float(R0.x),
          __int_as_float(R0.y), __int_as_float(R0.z), __int_as_float(R0.w), __int_as_float(R1.x),
          __int_as_float(R1.y), R1.z, BATCH ? batch.items[item].scene : sc_arg, c.fb32, c.fb64);
      if (e >= 0) {
        s = e;
        state = WALK;
      } else {  // no exit edge: the origin is not inside the start triangle
        if (BOUNCE)
          bounce_result(io_arg, ray, -3, INFINITY, 0, 0, -1);
        else
          park_code(BATCH ? batch.items[item].rays : io_arg, ray, -3, 0);
        state = IDLE;
      }
    } else if (BOUNCE && st_now == BNC) {
      const double ax = lohi(R0.x, R0.y), ay = lohi(R0.z, R0.w);
      const double bx = lohi(R1.x, R1.y), by = lohi(R1.z, R1.w);
      const double th = hit_t(make_double4(ax, ay, bx, by), ox, oy, dx, dy);
      if (nb < io_arg.max_bounces) {
        // specular reflection: origin o + t d; direction d - k n, n = (-ey, ex), k = 2 (d.n)/(n.n)
        const double ex = bx - ax, ey = by - ay;
        const double nx = -ey, ny = ex;
        const double dn = dx * nx + dy * ny;
        const double nn = nx * nx + ny * ny;
        const double k = (2.0 * dn) / nn;
        const double nox = ox + th * dx, noy = oy + th * dy;
        const double ndx = dx - k * nx, ndy = dy - k * ny;
        ox = nox;
        oy = noy;
        dx = ndx;
        dy = ndy;
        if (MODE == 1) r32 = ray32(ox, oy, dx, dy, sc_arg.org_x, sc_arg.org_y);
        ++nb;
        ++steps;
        seg = 1;
        // the reflected ray enters the hit triangle through the hit edge: only the vertex
        // opposite that edge decides the exit
        const int e = hs % 3;
        const bool left = left64<COUNT>(ox, oy, dx, dy, lohi(R2.x, R2.y), lohi(R2.z, R2.w), c.fb64);
        const int ex2 = e + (left ? 1 : 2);
        s = hs - e + (ex2 >= 3 ? ex2 - 3 : ex2);
        state = WALK;
      } else {
        bounce_result(io_arg, ray, s, th, steps, nb, io_arg.face ? 4 * R3 + hs % 3 : -1);
        if (COUNT) {
          c.steps += steps;
          ++c.rays;
        }
        state = IDLE;
      }
    }
  }
  if (COUNT) {
    if (c.steps) atomicAdd(&stats[0], (unsigned long long)c.steps);
    if (c.fb32) atomicAdd(&stats[1], (unsigned long long)c.fb32);
    if (c.fb64) atomicAdd(&stats[2], (unsigned long long)c.fb64);
    if (c.rays) atomicAdd(&stats[3], (unsigned long long)c.rays);
  }
}

// Second kernel of a single trace: in input order, turn each ray's parked (internal primitive or
// code, steps) into the caller's primitive id, the hit distance (the primitive's own segment,
// binary64, Sec. 5.1's stop on scene geometry) and steps. Every access but the primitive record
// is coalesced.
__device__ __forceinline__ void finish_one(const PrimRec* __restrict__ prim,
                                           const double2* __restrict__ o,
                                           const double2* __restrict__ d,
                                           int32_t* __restrict__ hit_prim,
                                           double* __restrict__ hit_t_io,
                                           int32_t* __restrict__ steps, int64_t i) {
  // the ray is loaded alongside the parked result (nearly every ray hits)
  const unsigned long long v = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(hit_t_io) + i);
  typedef double vd2 __attribute__((ext_vector_type(2)));
  const vd2 oo = __builtin_nontemporal_load(reinterpret_cast<const vd2*>(o) + i);
  const vd2 dd = __builtin_nontemporal_load(reinterpret_cast<const vd2*>(d) + i);
  const int code = (int)(unsigned)v;
  double t = INFINITY;
  if (code >= 0) {
    const PrimRec r = prim[code];
    t = hit_t(make_double4(r.ax, r.ay, r.bx, r.by), oo.x, oo.y, dd.x, dd.y);
  }
  __builtin_nontemporal_store(code, hit_prim + i);
  __builtin_nontemporal_store(t, hit_t_io + i);
  __builtin_nontemporal_store((int)(unsigned)(v >> 32), steps + i);
}

__global__ void __launch_bounds__(256)
finish_rays(const PrimRec* __restrict__ prim, const double2* __restrict__ o,
            const double2* __restrict__ d, int32_t* __restrict__ hit_prim,
            double* __restrict__ hit_t_io, int32_t* __restrict__ steps, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) finish_one(prim, o, d, hit_prim, hit_t_io, steps, i);
}

// The same for a batch: block b finishes tile b of the batch's tile sequence (the walk's tiling,
// blockDim.x rays per tile).
__global__ void __launch_bounds__(256)
finish_batch(const BatchItem* __restrict__ items, int n_items) {
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = n_items - 1;  // the last item whose first tile is at or before this one
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const BatchItem& it = items[lo];
  const int64_t i = (tile - it.tile_begin) * blockDim.x + threadIdx.x;
  if (i < it.rays.n)
    finish_one(it.scene.prim, it.rays.o, it.rays.d, it.rays.prim, it.rays.t, it.rays.steps, i);
}

// Parked records of binned rays (t, code | steps << 32) to the caller's arrays, in input order.
__global__ void __launch_bounds__(256)
finish_copy(const double2* __restrict__ park, int32_t* __restrict__ hit_prim,
            double* __restrict__ hit_t, int32_t* __restrict__ steps, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  typedef long long vl2 __attribute__((ext_vector_type(2)));
  const vl2 v = __builtin_nontemporal_load(reinterpret_cast<const vl2*>(park) + i);
  __builtin_nontemporal_store(__longlong_as_double(v.x), hit_t + i);
  __builtin_nontemporal_store((int)(unsigned)(unsigned long long)v.y, hit_prim + i);
  __builtin_nontemporal_store((int)(unsigned)((unsigned long long)v.y >> 32), steps + i);
}

__global__ void reset_counters(unsigned long long* counter) {
  if (threadIdx.x < kClaimChunks) counter[threadIdx.x] = 0ull;
}

// ------------------------------------------------------------------------------ launchers

size_t walk_lds_bytes(int mode, const LaunchCfg& cfg) {
  (void)mode;
  return (size_t)(cfg.wg / 64) * cfg.tile * 40;
}

template <int MODE, int TPL, bool COUNT, bool VALIDATE, bool BATCH, bool BOUNCE>
static hipError_t go(const SceneDev& sc, const RaysDev& io, ItemRef br, int64_t total_tiles,
                     const LaunchCfg& cfg, size_t lds, unsigned long long* counter,
                     const Workspace& ws, int* errflag, hipStream_t stream) {
  hipLaunchKernelGGL((walk_persistent<MODE, TPL, COUNT, VALIDATE, BATCH, BOUNCE>), dim3(cfg.grid),
                     dim3(cfg.wg), lds, stream, sc, io, br, total_tiles, counter, cfg.refill_min,
                     cfg.chunks, cfg.group, ws.stats, errflag);
  return hipGetLastError();
}

template <int MODE, bool COUNT, bool VALIDATE, bool BATCH, bool BOUNCE = false>
static hipError_t pick_tile(const SceneDev& sc, const RaysDev& io, ItemRef br, int64_t total_tiles,
                            const LaunchCfg& cfg, size_t lds, unsigned long long* counter,
                            const Workspace& ws, int* errflag, hipStream_t stream) {
  switch (cfg.tile) {
    case 64: return go<MODE, 1, COUNT, VALIDATE, BATCH, BOUNCE>(sc, io, br, total_tiles, cfg, lds, counter, ws, errflag, stream);
    case 128: return go<MODE, 2, COUNT, VALIDATE, BATCH, BOUNCE>(sc, io, br, total_tiles, cfg, lds, counter, ws, errflag, stream);
    case 256: return go<MODE, 4, COUNT, VALIDATE, BATCH, BOUNCE>(sc, io, br, total_tiles, cfg, lds, counter, ws, errflag, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_walk(const SceneDev& sc, const RaysDev& io, int mode, bool count, bool validate,
                       const LaunchCfg& cfg, unsigned long long* counter, int* errflag,
                       const Workspace& ws, hipStream_t stream, hipEvent_t walk_begin,
                       hipEvent_t walk_end) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e;
  if (walk_begin) {
    e = hipEventRecord(walk_begin, stream);
    if (e != hipSuccess) return e;
  }
  const size_t lds = walk_lds_bytes(mode, cfg);
  const ItemRef none{nullptr, 0, nullptr, 0};
  const int64_t tiles = (io.n + cfg.tile - 1) / cfg.tile;
  e = hipErrorInvalidValue;
  const bool bounce = io.hits != nullptr;  // continued rays write their own results
  if (bounce) {
    if (validate) return hipErrorInvalidValue;
    if (mode == 0 && !count) e = pick_tile<0, false, false, false, true>(sc, io, none, tiles, cfg, lds, counter, ws, errflag, stream);
    if (mode == 0 && count) e = pick_tile<0, true, false, false, true>(sc, io, none, tiles, cfg, lds, counter, ws, errflag, stream);
    if (mode == 1 && !count) e = pick_tile<1, false, false, false, true>(sc, io, none, tiles, cfg, lds, counter, ws, errflag, stream);
    if (mode == 1 && count) e = pick_tile<1, true, false, false, true>(sc, io, none, tiles, cfg, lds, counter, ws, errflag, stream);
  }
#define CCSP_CASE(M, C, V) \
  if (!bounce && mode == M && count == C && validate == V) \
    e = pick_tile<M, C, V, false>(sc, io, none, tiles, cfg, lds, counter, ws, errflag, stream);
  CCSP_CASE(0, false, false) CCSP_CASE(0, true, false) CCSP_CASE(0, false, true) CCSP_CASE(0, true, true)
  CCSP_CASE(1, false, false) CCSP_CASE(1, true, false) CCSP_CASE(1, false, true) CCSP_CASE(1, true, true)
#undef CCSP_CASE
  if (e != hipSuccess) return e;
  if (walk_end) {
    e = hipEventRecord(walk_end, stream);
    if (e != hipSuccess) return e;
  }
  if (bounce) return hipSuccess;
  const int64_t blocks = (io.n + 255) / 256;
  if (io.park)
    hipLaunchKernelGGL(finish_copy, dim3((unsigned)blocks), dim3(256), 0, stream, io.park,
                       io.prim, io.t, io.steps, io.n);
  else
    hipLaunchKernelGGL(finish_rays, dim3((unsigned)blocks), dim3(256), 0, stream, sc.prim, io.o,
                       io.d, io.prim, io.t, io.steps, io.n);
  return hipGetLastError();
}

hipError_t launch_walk_batch(const BatchItem* items_dev, int n_items, int64_t total_tiles,
                             int mode, bool count, const LaunchCfg& cfg,
                             unsigned long long* counter, const Workspace& ws, hipStream_t stream,
                             hipEvent_t walk_begin, hipEvent_t walk_end) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e;
  if (walk_begin) {
    e = hipEventRecord(walk_begin, stream);
    if (e != hipSuccess) return e;
  }
  const int n_lds = n_items < 1024 ? n_items : 1024;
  const size_t lds = walk_lds_bytes(mode, cfg) + (size_t)((n_lds + 1) & ~1) * 8;
  const ItemRef br{items_dev, n_items, nullptr, n_lds};
  const SceneDev nosc{};
  const RaysDev noio{};
  e = hipErrorInvalidValue;
  if (mode == 0 && !count) e = pick_tile<0, false, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, nullptr, stream);
  if (mode == 0 && count) e = pick_tile<0, true, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, nullptr, stream);
  if (mode == 1 && !count) e = pick_tile<1, false, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, nullptr, stream);
  if (mode == 1 && count) e = pick_tile<1, true, false, true>(nosc, noio, br, total_tiles, cfg, lds, counter, ws, nullptr, stream);
  if (e != hipSuccess) return e;
  if (walk_end) {
    e = hipEventRecord(walk_end, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finish_batch, dim3((unsigned)total_tiles), dim3(cfg.tile), 0, stream,
                     items_dev, n_items);
  return hipGetLastError();
}

}  // namespace ccsp
