// Persistent stackless walk through a 3D constrained tetrahedralisation for gfx950 (CDNA4,
// wave64): the 3D form of the triangulation walk (Sec. 1.3 and 1.4: one decision per visited
// tetrahedron, the exit face among the three faces other than the entry face; Sec. 7.2).
//
// Mapping to the hardware:
//  * Like the 2D walk this is a chain of dependent gathers with a few flops each, bound by the rate
//    at which the memory system serves dependent random loads (about the same from 32 MiB to
//    4 GiB), not by bandwidth, MFMA or ALUs. One step is one 16-byte load, the slot of the exit
//    face: the neighbour and its entry face, the neighbour's fourth vertex (the apex) and the
//    order of the shared face's vertices seen from the neighbour; the face's own three vertices
//    travel in registers (relative to the origin), so a step needs no other memory.
//  * Two Plücker signs per step, both of the form X . m with m = d x W computed once per step
//    (W the apex, X a face vertex, all relative to o). Integer grid inputs make m exact in
//    binary64 (|m| < 2^40); X . m is rounded once per product and per sum, and accepted when a
//    forward error bound proves its sign. Otherwise an exact int64 evaluation decides, and a zero
//    takes the sign of the symbolically moved line (origin o + (e, e^2, e^3), direction
//    d + (e^10, e^20, e^30)).
//  * Waves are persistent: each takes rays_per_claim rays per global atomic, stages them 128 at a
//    time in its own LDS region with one round of coalesced loads, and refills idle lanes from
//    there as soon as refill_min of its 64 lanes are idle. Every lane then issues exactly one
//    round of loads per iteration, whatever its state (the start tetrahedron's vertices or an
//    exit slot), so lanes in different states share one memory round trip.
//
// Compiled with -ffp-contract=off: the error bound and the hit distance assume every operation
// is rounded separately.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ccsp_tet.h"
#include "scan.hpp"

namespace ccsp {
void set_last_error(const char* msg);
}

struct TetMesh {
  int device = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  const int4* slot = nullptr;   // 4 face slots per tetrahedron, in the internal (Morton) order
  const int4* first = nullptr;  // 4 per tetrahedron, in the caller's order: the four vertices
                                // (12 int32) and the internal id
  int64_t nt = 0, nv = 0, np = 0;
};

namespace {

constexpr int kGridBits = 19;
constexpr int32_t kGrid = 1 << kGridBits;
constexpr int32_t kMask = kGrid - 1;

// FACE[f][i], the local vertices of face f (opposite vertex f) counter-clockwise seen from
// outside: (1,2,3), (0,3,2), (0,1,3), (0,2,1); nibble 3f+i.
constexpr uint64_t kFace = 0x120310230321ull;
// After entering through face j (apex w, face vertices p, q, r in FACE[j] order) the exit face
// opposite p, q or r (k = 0, 1, 2) is held in registers in the order the decision yields it,
// (r, q, w), (p, r, w) or (p, w, q); that is FACE[e] rotated by rho(j, k): register i holds
// FACE[e][(i + rho) % 3]. 2 bits at 2 (3j + k).
constexpr uint32_t kRho = 0x2065u;

__host__ __device__ __forceinline__ int face_v(int f, int i) {
  return (int)((kFace >> (4 * (3 * f + i))) & 0xF);
}
__device__ __forceinline__ int face_rho(int j, int k) { return (int)((kRho >> (2 * (3 * j + k))) & 3); }

struct V3 {
  int x, y, z;
};

__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 sel(bool c, V3 a, V3 b) {
  return V3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}
// one of p, q, r, w by a 2-bit code
__device__ __forceinline__ V3 sel4(int code, V3 p, V3 q, V3 r, V3 w) {
  return sel(code & 2, sel(code & 1, w, r), sel(code & 1, q, p));
}
// a, b or c for t = 0, 1, 2
__device__ __forceinline__ V3 sel3(int t, V3 a, V3 b, V3 c) { return sel(t == 0, a, sel(t == 1, b, c)); }

struct M3 {
  double x, y, z;
};

// d x W, exact in binary64 (|components| < 2^39)
__device__ __forceinline__ M3 cross_dw(V3 d, V3 w) {
  return M3{(double)d.y * (double)w.z - (double)d.z * (double)w.y,
            (double)d.z * (double)w.x - (double)d.x * (double)w.z,
            (double)d.x * (double)w.y - (double)d.y * (double)w.x};
}

__device__ __forceinline__ int sgn64(int64_t v) { return (v > 0) - (v < 0); }

// Exact sign of d . (W x X) = X . (d x W), then of the moved line where it is zero.
__device__ __attribute__((noinline)) int plucker_exact(V3 d, V3 W, V3 X) {
  const int64_t mx = (int64_t)d.y * W.z - (int64_t)d.z * W.y;
  const int64_t my = (int64_t)d.z * W.x - (int64_t)d.x * W.z;
  const int64_t mz = (int64_t)d.x * W.y - (int64_t)d.y * W.x;
  const int64_t v = X.x * mx + X.y * my + X.z * mz;
  if (v != 0) return sgn64(v);
  // a = X - W (the edge), c = d x a: the origin moved by (e, e^2, e^3)
  const int64_t ax = (int64_t)X.x - W.x, ay = (int64_t)X.y - W.y, az = (int64_t)X.z - W.z;
  const int64_t cx = (int64_t)d.y * az - (int64_t)d.z * ay;
  if (cx != 0) return sgn64(cx);
  const int64_t cy = (int64_t)d.z * ax - (int64_t)d.x * az;
  if (cy != 0) return sgn64(cy);
  const int64_t cz = (int64_t)d.x * ay - (int64_t)d.y * ax;
  if (cz != 0) return sgn64(cz);
  // the edge is parallel to d: the direction turned by (e^10, e^20, e^30); Wx = (W x X)
  const int64_t wx = (int64_t)W.y * X.z - (int64_t)W.z * X.y;
  if (wx != 0) return sgn64(wx);
  if (az != 0) return -sgn64(az);
  if (ay != 0) return sgn64(ay);
  const int64_t wy = (int64_t)W.z * X.x - (int64_t)W.x * X.z;
  if (wy != 0) return sgn64(wy);
  return -sgn64(ax);  // az = ay = 0 here, so ax != 0 for distinct vertices
}

// sign of X . m with m = d x W (exact), through the binary64 filter
__device__ __forceinline__ int plucker(M3 m, V3 d, V3 W, V3 X) {
  const double px = (double)X.x * m.x, py = (double)X.y * m.y, pz = (double)X.z * m.z;
  const double v = (px + py) + pz;
  // |error| <= 3u (|px| + |py| + |pz|) (1 + O(u)); the bound takes 8u
  const double b = ((fabs(px) + fabs(py)) + fabs(pz)) * 0x1p-50;
  if (v > b) return 1;
  if (v < -b) return -1;
  return plucker_exact(d, W, X);
}

// sign of A . (B x C) (= -det[b - a; c - a; o - a] for points relative to o), exact
__device__ __attribute__((noinline)) int triple_exact(V3 A, V3 B, V3 C) {
  const int64_t cx = (int64_t)B.y * C.z - (int64_t)B.z * C.y;
  const int64_t cy = (int64_t)B.z * C.x - (int64_t)B.x * C.z;
  const int64_t cz = (int64_t)B.x * C.y - (int64_t)B.y * C.x;
  return sgn64(A.x * cx + A.y * cy + A.z * cz);
}

__device__ __forceinline__ bool triple_pos(V3 A, V3 B, V3 C) {
  const double cx = (double)B.y * C.z - (double)B.z * C.y;
  const double cy = (double)B.z * C.x - (double)B.x * C.z;
  const double cz = (double)B.x * C.y - (double)B.y * C.x;
  const double px = (double)A.x * cx, py = (double)A.y * cy, pz = (double)A.z * cz;
  const double v = (px + py) + pz;
  const double b = ((fabs(px) + fabs(py)) + fabs(pz)) * 0x1p-50;
  if (v > b) return true;
  if (v < -b) return false;
  return triple_exact(A, B, C) > 0;
}

// t from the face (A, B, C) (any rotation, either orientation: n is exact, so it only changes
// sign with the orientation, and num and den change sign together) and the primitive's first
// vertex `a`, all relative to o
__device__ __forceinline__ double hit_t(V3 A, V3 B, V3 C, V3 a, V3 d) {
  const double ux = (double)(B.x - A.x), uy = (double)(B.y - A.y), uz = (double)(B.z - A.z);
  const double vx = (double)(C.x - A.x), vy = (double)(C.y - A.y), vz = (double)(C.z - A.z);
  const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  const double num = ((double)a.x * nx + (double)a.y * ny) + (double)a.z * nz;
  const double den = ((double)d.x * nx + (double)d.y * ny) + (double)d.z * nz;
  return num / den;
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

struct Rays3Dev {
  const int32_t* o;
  const int32_t* d;
  const int32_t* start;
  int32_t* hit_prim;
  double* hit_t;
  int32_t* steps;
  int64_t n;
  int32_t limit;  // step guard: a walk may visit at most this many tetrahedra
};

__device__ __forceinline__ void finish(const Rays3Dev& io, int64_t ray, int prim, double t, int steps) {
  io.hit_prim[ray] = prim;
  io.hit_t[ray] = t;
  io.steps[ray] = steps;
}

__device__ __forceinline__ bool on_grid(int v) { return (unsigned)v < (unsigned)kGrid; }
__device__ __forceinline__ bool dir_ok(int v) { return v >= -kGrid && v <= kGrid; }

__device__ __forceinline__ void wave_lds_fence() {
  // a wave's LDS operations execute in order; this only keeps the compiler from moving the reads
  // of a freshly written tile above its writes
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kTile = 64;  // rays a wave stages in LDS per claim
constexpr int kTileBytes = 64 * kTile;
constexpr int kChunks = 8;  // claim chunks: one per XCD

// A ray ready to walk (64 bytes): origin and index, direction and the first exit slot (-1: the
// ray is invalid), then the first exit face's vertices relative to the origin, 20-bit fields.
struct RayRec3 {
  int4 oi;
  int4 ds;
  int4 ab;
  int4 c;
};

__device__ __forceinline__ int2 pack3(V3 v) {
  const uint64_t u = (uint64_t)(v.x & 0xFFFFF) | ((uint64_t)(v.y & 0xFFFFF) << 20) |
                     ((uint64_t)(v.z & 0xFFFFF) << 40);
  return make_int2((int)(uint32_t)u, (int)(uint32_t)(u >> 32));
}
__device__ __forceinline__ V3 unpack3(int lo, int hi) {
  const int64_t u = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  return V3{(int)((u << 44) >> 44), (int)((u << 24) >> 44), (int)((u << 4) >> 44)};
}

// Claim the next `claim` rays of [0, n): the rays are split into kChunks contiguous chunks with a
// counter each; a workgroup starts in chunk blockIdx.x % kChunks (workgroups go to the XCDs
// round-robin, so each XCD walks its own eighth of the binned rays, a region of space whose
// tetrahedra its own L2 keeps) and moves on to the next chunk once one is exhausted. Returns the
// first ray, or -1 when every chunk is exhausted. Wave-uniform.
__device__ __forceinline__ int64_t claim_rays(unsigned long long* counter, int64_t n, int claim,
                                              int& cur, int& tried, int lane, int64_t& end) {
  while (tried < kChunks) {
    const int64_t c0 = n * cur / kChunks, c1 = n * (cur + 1) / kChunks;
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(counter + cur, (unsigned long long)claim);
    const int64_t r = c0 + (int64_t)bcast64(b);
    if (r < c1) {
      end = min(r + claim, c1);
      return r;
    }
    cur = cur + 1 == kChunks ? 0 : cur + 1;
    ++tried;
  }
  return -1;
}

// One step of the walk: the ray leaves its tetrahedron through the face whose slot is q. Returns
// false once the ray is finished (hit, miss or guard; results written); otherwise the ray is in
// the neighbour, its exit face decided: k (0, 1, 2: opposite p, q, r of the entry face), X0..X2,
// rho and s (the exit slot) updated.
__device__ __forceinline__ bool advance(const int4 q, const Rays3Dev& io, int ray, V3 o, V3 d,
                                        V3& X0, V3& X1, V3& X2, int& rho, int& s, int& steps,
                                        int& k) {
  const int word = q.x;
  if (word < -1) {
    const V3 a = sub(V3{q.y, q.z, q.w & kMask}, o);
    finish(io, ray, -2 - word, hit_t(X0, X1, X2, a, d), steps);
    return false;
  }
  if (word == -1 || steps >= io.limit) {
    finish(io, ray, word == -1 ? -1 : -2, INFINITY, steps);
    return false;
  }
  const int nb = word >> 2, j = word & 3, perm = (q.w >> kGridBits) & 3;
  const V3 W = sub(V3{q.y, q.z, q.w & kMask}, o);
  // the slot names the neighbour's p as vertex `perm` of the face's FACE order; its q and r
  // follow in the reverse cyclic order
  int t = perm - rho;
  t += t < 0 ? 3 : 0;
  const V3 P = sel3(t, X0, X1, X2);
  const V3 Q = sel3(t, X2, X0, X1);
  const V3 R = sel3(t, X1, X2, X0);
  ++steps;
  const M3 m = cross_dw(d, W);
  const int sp = plucker(m, d, W, P);
  const int sx = plucker(m, d, W, sp > 0 ? R : Q);
  k = sp > 0 ? (sx < 0 ? 1 : 0) : (sx > 0 ? 2 : 0);
  // the exit face in decision order: (r, q, w), (p, r, w) or (p, w, q)
  X0 = sel(k == 0, R, P);
  X1 = sel(k == 0, Q, sel(k == 1, R, W));
  X2 = sel(k == 2, Q, W);
  rho = face_rho(j, k);
  s = 4 * nb + face_v(j, k);
  return true;
}

// The walk from the first exit slot on. Every lane issues one 16-byte slot load per iteration.
__global__ void __launch_bounds__(512)
walk3d(const int4* __restrict__ slots, Rays3Dev io, const RayRec3* __restrict__ recs,
       unsigned long long* __restrict__ counter, int claim, int refill_min) {
  extern __shared__ unsigned char lds[];
  const int lane = threadIdx.x & 63;
  RayRec3* const tile = reinterpret_cast<RayRec3*>(lds + (threadIdx.x >> 6) * kTileBytes);
  bool busy = false;
  int ray = 0;
  V3 o{0, 0, 0}, d{0, 0, 0};
  // the exit face, relative to o: register i holds vertex (i + rho) % 3 of its FACE order
  V3 X0{0, 0, 0}, X1{0, 0, 0}, X2{0, 0, 0};
  int rho = 0;
  int s = 0, steps = 0;  // exit slot, tetrahedra visited
  int64_t tbase = 0, next = 0, end = 0;   // the staged tile; the rest of the wave's claim
  int tlen = 0, thead = 0;
  int chunk_cur = (int)(blockIdx.x % (unsigned)kChunks), chunk_tried = 0;
  bool drained = false;
  for (;;) {
    const unsigned long long idle = __ballot(!busy);
    const int nidle = __popcll(idle);
    if (drained && nidle == 64) break;
    if (!drained && nidle >= refill_min) {
      const int rank = __popcll(idle & ((1ull << lane) - 1));
      int served = 0;
      while (served < nidle) {
        if (thead == tlen) {
          if (next == end) {
            next = claim_rays(counter, io.n, claim, chunk_cur, chunk_tried, lane, end);
            if (next < 0) {
              drained = true;
              break;
            }
          }
          tbase = next;
          tlen = (int)min((int64_t)kTile, end - next);
          next += tlen;
          thead = 0;
          if (lane < tlen) tile[lane] = recs[tbase + lane];  // one round of coalesced loads
          wave_lds_fence();
        }
        const int take = min(nidle - served, tlen - thead);
        if (!busy && rank >= served && rank < served + take) {
          const RayRec3 r = tile[thead + (rank - served)];
          ray = r.oi.w;
          s = r.ds.w;
          if (s >= 0) {
            o = V3{r.oi.x, r.oi.y, r.oi.z};
            d = V3{r.ds.x, r.ds.y, r.ds.z};
            X0 = unpack3(r.ab.x, r.ab.y);
            X1 = unpack3(r.ab.z, r.ab.w);
            X2 = unpack3(r.c.x, r.c.y);
            rho = 0;
            steps = 1;
            busy = true;
          } else {
            finish(io, ray, -3, INFINITY, 0);
          }
        }
        served += take;
        thead += take;
      }
    }
    if (!busy) continue;
    int k = 0;
    busy = advance(slots[s], io, ray, o, d, X0, X1, X2, rho, s, steps, k);
  }
}

// ---- the start of every ray (its first tetrahedron: the precondition checks and the exit face
// among all four, Sec. 1.4), and ray binning: a counting sort of the rays into the cells of an
// 8 x 8 x 8 grid over the coordinate cube numbered along a Morton curve (optionally each cell
// split by the octant of the direction), so that the rays an XCD walks start close together and
// those a wave walks also head the same way. A count kernel histograms the buckets per chunk of
// rays in LDS, a scan turns the (bucket, chunk) counts into destinations, and a scatter kernel
// writes each ray's 64-byte start record to its bucket's next place (or, unbinned, to the ray's
// own place).

constexpr int kCellBits = 3;
constexpr int kCells = 1 << (3 * kCellBits);
constexpr int kMaxBuckets = kCells * 8;  // cells x direction octants
constexpr int kBinChunk = 4096;          // rays per binning workgroup
constexpr int kBinThreads = 256;

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 3 bits -> every third bit
  return (v & 1) | ((v & 2) << 2) | ((v & 4) << 4);
}

// The ray's bucket: its origin's cell, then (dirs) the octant of its direction. Off-grid origins
// land in cell 0; their start record marks them invalid.
__device__ __forceinline__ int bucket_of(const int32_t* o, const int32_t* d, int dirs) {
  const uint32_t x = (uint32_t)o[0], y = (uint32_t)o[1], z = (uint32_t)o[2];
  int cell = 0;
  if (x < (uint32_t)kGrid && y < (uint32_t)kGrid && z < (uint32_t)kGrid) {
    const int sh = kGridBits - kCellBits;
    cell = (int)(spread3(x >> sh) | (spread3(y >> sh) << 1) | (spread3(z >> sh) << 2));
  }
  if (!dirs) return cell;
  return (cell << 3) | ((d[0] < 0) ? 1 : 0) | ((d[1] < 0) ? 2 : 0) | ((d[2] < 0) ? 4 : 0);
}

__global__ void __launch_bounds__(kBinThreads)
bin_count(const int32_t* __restrict__ o, const int32_t* __restrict__ d, int64_t n, int dirs,
          int nbk, uint32_t* __restrict__ H, int nchunks) {
  __shared__ uint32_t h[kMaxBuckets];
  for (int b = threadIdx.x; b < nbk; b += kBinThreads) h[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBinChunk;
  for (int q = 0; q < kBinChunk / kBinThreads; ++q) {
    const int64_t i = base + threadIdx.x + q * kBinThreads;
    if (i < n) atomicAdd(&h[bucket_of(o + 3 * i, d + 3 * i, dirs)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbk; b += kBinThreads) H[(size_t)b * nchunks + blockIdx.x] = h[b];
}

// The start record of ray i: checks (grid, direction, start range, origin strictly inside), the
// exit face of the start tetrahedron (the first face, in face order, whose three outside-ordered
// edges the ray passes positively) and that face's vertices relative to the origin.
__device__ RayRec3 start_record(const int4* __restrict__ firsts, int32_t nt, const Rays3Dev& io,
                                int64_t i) {
  const int32_t* po = io.o + 3 * i;
  const int32_t* pd = io.d + 3 * i;
  const V3 o{po[0], po[1], po[2]}, d{pd[0], pd[1], pd[2]};
  const int st = io.start[i];
  RayRec3 r;
  r.oi = make_int4(o.x, o.y, o.z, (int)i);
  r.ds = make_int4(d.x, d.y, d.z, -1);
  r.ab = make_int4(0, 0, 0, 0);
  r.c = make_int4(0, 0, 0, 0);
  const bool ok = on_grid(o.x) && on_grid(o.y) && on_grid(o.z) && dir_ok(d.x) && dir_ok(d.y) &&
                  dir_ok(d.z) && (d.x != 0 || d.y != 0 || d.z != 0) && st >= 0 && st < nt;
  if (!ok) return r;
  // vertices relative to o: x0 y0 z0 x1 | y1 z1 x2 y2 | z2 x3 y3 z3 | internal id
  const int4* p = firsts + 4 * (int64_t)st;
  const int4 F0 = p[0], F1 = p[1], F2 = p[2];
  const int id = p[3].x;
  const V3 v0 = sub(V3{F0.x, F0.y, F0.z}, o), v1 = sub(V3{F0.w, F1.x, F1.y}, o);
  const V3 v2 = sub(V3{F1.z, F1.w, F2.x}, o), v3 = sub(V3{F2.y, F2.z, F2.w}, o);
  // strictly inside: A . (B x C) > 0 for every face (A, B, C) in outside order
  if (!(triple_pos(v1, v2, v3) && triple_pos(v0, v3, v2) && triple_pos(v0, v1, v3) &&
        triple_pos(v0, v2, v1)))
    return r;
  const M3 m0 = cross_dw(d, v0), m1 = cross_dw(d, v1), m2 = cross_dw(d, v2);
  const int s01 = plucker(m0, d, v0, v1), s02 = plucker(m0, d, v0, v2);
  const int s03 = plucker(m0, d, v0, v3), s12 = plucker(m1, d, v1, v2);
  const int s13 = plucker(m1, d, v1, v3), s23 = plucker(m2, d, v2, v3);
  int e = -1;
  if (s12 > 0 && s23 > 0 && s13 < 0) e = 0;
  else if (s03 > 0 && s23 < 0 && s02 < 0) e = 1;
  else if (s01 > 0 && s13 > 0 && s03 < 0) e = 2;
  else if (s02 > 0 && s12 < 0 && s01 < 0) e = 3;
  if (e < 0) return r;
  const int2 a = pack3(sel4(face_v(e, 0), v0, v1, v2, v3));
  const int2 b = pack3(sel4(face_v(e, 1), v0, v1, v2, v3));
  const int2 c = pack3(sel4(face_v(e, 2), v0, v1, v2, v3));
  r.ds.w = 4 * id + e;
  r.ab = make_int4(a.x, a.y, b.x, b.y);
  r.c = make_int4(c.x, c.y, 0, 0);
  return r;
}

__global__ void __launch_bounds__(kBinThreads)
bin_scatter(const int4* __restrict__ firsts, int32_t nt, Rays3Dev io, int dirs, int nbk,
            const uint32_t* __restrict__ Hoff, int nchunks, RayRec3* __restrict__ out) {
  __shared__ uint32_t off[kMaxBuckets];
  for (int b = threadIdx.x; b < nbk; b += kBinThreads) off[b] = Hoff[(size_t)b * nchunks + blockIdx.x];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBinChunk;
  for (int q = 0; q < kBinChunk / kBinThreads; ++q) {
    const int64_t i = base + threadIdx.x + q * kBinThreads;
    if (i >= io.n) break;
    const RayRec3 r = start_record(firsts, nt, io, i);
    const uint32_t pos = atomicAdd(&off[bucket_of(io.o + 3 * i, io.d + 3 * i, dirs)], 1u);
    out[pos] = r;
  }
}

__global__ void __launch_bounds__(kBinThreads)
start_records(const int4* __restrict__ firsts, int32_t nt, Rays3Dev io, RayRec3* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < io.n) out[i] = start_record(firsts, nt, io, i);
}

__global__ void reset_counters(unsigned long long* c) {
  if (threadIdx.x < kChunks) c[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ host

thread_local char g_msg[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  ccsp::set_last_error(g_msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(CCSP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kCounterGroups = 128;  // launches in flight on one device that never share counters

struct Dev3 {
  unsigned long long* counters = nullptr;  // kCounterGroups x kChunks
  int cus = 0;
  std::atomic<uint64_t> next{0};
  // binning scratch, shared by the device's traces; bin_free marks the end of its last use
  std::mutex bin_mu;
  void* bin_ws = nullptr;
  size_t bin_ws_bytes = 0;
  hipEvent_t bin_free = nullptr;
  hipStream_t bin_last_stream = nullptr;
  // stage events of the last CCSP_TRACE_TIMED call
  std::mutex time_mu;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  bool timed = false;
};

std::mutex g_dev_mu;
Dev3 g_dev[64];

int dev_state(Dev3** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(CCSP_E_HIP, "device index %d unsupported", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  Dev3& ds = g_dev[dev];
  if (!ds.counters) {
    e = hipDeviceGetAttribute(&ds.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    if (!ds.bin_free) {
      e = hipEventCreateWithFlags(&ds.bin_free, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    for (auto& ev : ds.ev)
      if (!ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      }
    e = hipMalloc(&ds.counters, kCounterGroups * kChunks * sizeof(unsigned long long));
    if (e != hipSuccess) {
      ds.counters = nullptr;
      return fail(CCSP_E_OOM, "counter allocation failed: %s", hipGetErrorString(e));
    }
  }
  *out = &ds;
  return CCSP_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// binning scratch for n rays: (cell, chunk) counts and offsets, scan temporaries, records
size_t bin_bytes(int64_t n, size_t* scan_tmp) {
  const int64_t nchunks = (n + kBinChunk - 1) / kBinChunk;
  const size_t cnt = (size_t)kMaxBuckets * (size_t)nchunks;
  const size_t tmp = ccsp::exclusive_scan_bytes((int64_t)cnt);
  if (scan_tmp) *scan_tmp = tmp;
  return 2 * align256(cnt * sizeof(uint32_t)) + align256(tmp) + align256((size_t)n * sizeof(RayRec3));
}

RayRec3* binned_records(Dev3* ds, size_t scan_tmp, int64_t n) {
  const int64_t nchunks = (n + kBinChunk - 1) / kBinChunk;
  const size_t cnt = (size_t)kMaxBuckets * (size_t)nchunks;
  return reinterpret_cast<RayRec3*>(static_cast<char*>(ds->bin_ws) + 2 * align256(cnt * sizeof(uint32_t)) +
                                    align256(scan_tmp));
}

int64_t orient_host(const int32_t* a, const int32_t* b, const int32_t* c, const int32_t* q) {
  const int64_t u0 = (int64_t)b[0] - a[0], u1 = (int64_t)b[1] - a[1], u2 = (int64_t)b[2] - a[2];
  const int64_t v0 = (int64_t)c[0] - a[0], v1 = (int64_t)c[1] - a[1], v2 = (int64_t)c[2] - a[2];
  const int64_t w0 = (int64_t)q[0] - a[0], w1 = (int64_t)q[1] - a[1], w2 = (int64_t)q[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

// 10 bits of each coordinate interleaved (x lowest)
uint32_t morton30(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint32_t v) {
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
  };
  return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

template <class F>
void parallel_for(int64_t n, F&& f) {
  const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nth = n < 65536 ? 1 : hw;
  if (nth == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  for (int k = 0; k < nth; ++k)
    th.emplace_back([&, k] { f(n * k / nth, n * (k + 1) / nth, k); });
  for (auto& t : th) t.join();
}

}  // namespace

extern "C" {

int load_tetmesh(const TetMeshDesc* desc, TetMesh** out) {
  if (!desc || !out) return fail(CCSP_E_ARG, "load_tetmesh: null descriptor or output pointer");
  *out = nullptr;
  const int64_t V = desc->n_vertices, T = desc->n_tets, NP = desc->n_prims;
  if (V < 4 || V > INT32_MAX) return fail(CCSP_E_ARG, "n_vertices %lld out of range", (long long)V);
  if (T < 1 || T >= (int64_t(1) << 29))
    return fail(CCSP_E_ARG, "n_tets %lld out of range [1, 2^29)", (long long)T);
  if (NP < 0 || NP > (int64_t(1) << 29)) return fail(CCSP_E_ARG, "n_prims %lld out of range", (long long)NP);
  if (!desc->xyz || !desc->tet_v || !desc->tet_nbr || !desc->tet_prim || (NP > 0 && !desc->prims))
    return fail(CCSP_E_ARG, "load_tetmesh: null array");
  const int32_t* X = desc->xyz;
  const int32_t* tv = desc->tet_v;
  const int32_t* tn = desc->tet_nbr;
  const int32_t* tp = desc->tet_prim;
  const int32_t* pv = desc->prims;
  for (int64_t k = 0; k < 3 * V; ++k)
    if (X[k] < 0 || X[k] >= kGrid)
      return fail(CCSP_E_BAD_TRIANGULATION, "vertex %lld: coordinate %d off the grid [0, 2^19)",
                  (long long)(k / 3), X[k]);
  for (int64_t k = 0; k < 3 * NP; ++k)
    if (pv[k] < 0 || pv[k] >= V) return fail(CCSP_E_BAD_TRIANGULATION, "primitive %lld: vertex id out of range", (long long)(k / 3));
  for (int64_t k = 0; k < 4 * T; ++k)
    if (tv[k] < 0 || tv[k] >= V) return fail(CCSP_E_BAD_TRIANGULATION, "tetrahedron %lld: vertex id out of range", (long long)(k / 4));

  // internal order: tetrahedra sorted by the Morton code of their centroid, so that neighbours in
  // space are mostly neighbours in memory
  std::vector<uint64_t> key((size_t)T);
  parallel_for(T, [&](int64_t t0, int64_t t1, int) {
    for (int64_t t = t0; t < t1; ++t) {
      int64_t c[3] = {0, 0, 0};
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) c[k] += X[3 * (int64_t)tv[4 * t + i] + k];
      const uint32_t m = morton30((uint32_t)(c[0] >> 11), (uint32_t)(c[1] >> 11), (uint32_t)(c[2] >> 11));
      key[t] = ((uint64_t)m << 32) | (uint64_t)t;
    }
  });
  std::sort(key.begin(), key.end());
  std::vector<int32_t> to_int((size_t)T);
  for (int64_t k = 0; k < T; ++k) to_int[(uint32_t)key[k]] = (int32_t)k;

  std::vector<int4> slot((size_t)(4 * T)), first((size_t)(4 * T));
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::string> err((size_t)nth + 1);
  std::vector<int64_t> err_at((size_t)nth + 1, INT64_MAX);
  parallel_for(T, [&](int64_t t0, int64_t t1, int w) {
    char buf[256];
    auto bad = [&](int64_t t, const char* fmt, auto... args) {
      if (t < err_at[w]) {
        snprintf(buf, sizeof buf, fmt, args...);
        err[w] = buf;
        err_at[w] = t;
      }
    };
    for (int64_t t = t0; t < t1 && err_at[w] == INT64_MAX; ++t) {
      const int32_t* v = tv + 4 * t;
      const int32_t* P[4] = {X + 3 * (int64_t)v[0], X + 3 * (int64_t)v[1], X + 3 * (int64_t)v[2], X + 3 * (int64_t)v[3]};
      if (orient_host(P[0], P[1], P[2], P[3]) <= 0) {
        bad(t, "tetrahedron %lld is not positively oriented", (long long)t);
        break;
      }
      const int64_t ti = to_int[t];
      first[4 * t + 0] = make_int4(P[0][0], P[0][1], P[0][2], P[1][0]);
      first[4 * t + 1] = make_int4(P[1][1], P[1][2], P[2][0], P[2][1]);
      first[4 * t + 2] = make_int4(P[2][2], P[3][0], P[3][1], P[3][2]);
      first[4 * t + 3] = make_int4((int)ti, 0, 0, 0);
      for (int i = 0; i < 4; ++i) {
        const int32_t fa = v[face_v(i, 0)], fb = v[face_v(i, 1)], fc = v[face_v(i, 2)];
        const int32_t nb = tn[4 * t + i], pr = tp[4 * t + i];
        if (pr < -1 || pr >= NP) {
          bad(t, "tetrahedron %lld face %d: primitive id %d out of range", (long long)t, i, pr);
          break;
        }
        if (pr >= 0) {
          const int32_t* q = pv + 3 * (int64_t)pr;
          const bool same = (q[0] == fa || q[0] == fb || q[0] == fc) && (q[1] == fa || q[1] == fb || q[1] == fc) &&
                            (q[2] == fa || q[2] == fb || q[2] == fc) && q[0] != q[1] && q[1] != q[2] && q[0] != q[2];
          if (!same) {
            bad(t, "tetrahedron %lld face %d is not made of primitive %d's vertices", (long long)t, i, pr);
            break;
          }
        }
        int j = -1;
        if (nb >= 0) {
          if (nb >= T) {
            bad(t, "tetrahedron %lld: neighbour %d out of range", (long long)t, nb);
            break;
          }
          const int32_t* w = tv + 4 * (int64_t)nb;
          for (int jj = 0; jj < 4 && j < 0; ++jj) {
            if (tn[4 * (int64_t)nb + jj] != t) continue;
            const int32_t x0 = w[face_v(jj, 0)], x1 = w[face_v(jj, 1)], x2 = w[face_v(jj, 2)];
            // the same face, seen from the other side: a reversed rotation of (fa, fb, fc)
            if ((x0 == fa && x1 == fc && x2 == fb) || (x0 == fb && x1 == fa && x2 == fc) ||
                (x0 == fc && x1 == fb && x2 == fa))
              j = jj;
          }
          if (j < 0) {
            bad(t, "tetrahedron %lld face %d: neighbour %d does not share it back", (long long)t, i, nb);
            break;
          }
          if (orient_host(X + 3 * (int64_t)fa, X + 3 * (int64_t)fb, X + 3 * (int64_t)fc, X + 3 * (int64_t)w[j]) <= 0) {
            bad(t, "tetrahedra %lld and %d do not lie on opposite sides of their face", (long long)t, nb);
            break;
          }
          if (tp[4 * (int64_t)nb + j] != pr) {
            bad(t, "tetrahedra %lld and %d name different primitives for their face", (long long)t, nb);
            break;
          }
        }
        int4 r;
        if (pr >= 0) {
          const int32_t* a = X + 3 * (int64_t)pv[3 * (int64_t)pr];
          r = make_int4(-2 - pr, a[0], a[1], a[2]);
        } else if (nb < 0) {
          r = make_int4(-1, 0, 0, 0);
        } else {
          const int32_t* w = tv + 4 * (int64_t)nb;
          const int32_t x0 = w[face_v(j, 0)];
          const int perm = x0 == fa ? 0 : x0 == fb ? 1 : 2;
          const int32_t* apex = X + 3 * (int64_t)w[j];
          r = make_int4((to_int[nb] << 2) | j, apex[0], apex[1], apex[2] | (perm << kGridBits));
        }
        slot[4 * ti + i] = r;
      }
    }
  });
  for (int w = 0; w < nth; ++w)
    if (err_at[w] != INT64_MAX) return fail(CCSP_E_BAD_TRIANGULATION, "%s", err[w].c_str());

  auto* m = new (std::nothrow) TetMesh;
  if (!m) return fail(CCSP_E_OOM, "host allocation failed");
  const size_t sb = slot.size() * sizeof(int4), fb = first.size() * sizeof(int4);
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipMalloc(&m->mem, sb + fb);
  if (e != hipSuccess) {
    delete m;
    return fail(CCSP_E_OOM, "device allocation of %zu bytes failed: %s", sb + fb, hipGetErrorString(e));
  }
  m->bytes = sb + fb;
  e = hipMemcpy(m->mem, slot.data(), sb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(static_cast<char*>(m->mem) + sb, first.data(), fb, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(m->mem);
    delete m;
    return hip_fail(e, "hipMemcpy");
  }
  m->slot = static_cast<const int4*>(m->mem);
  m->first = reinterpret_cast<const int4*>(static_cast<char*>(m->mem) + sb);
  m->nt = T;
  m->nv = V;
  m->np = NP;
  *out = m;
  return CCSP_OK;
}

int free_tetmesh(TetMesh* mesh) {
  if (!mesh) return CCSP_OK;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess) e = hipSetDevice(mesh->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  const hipError_t ef = hipFree(mesh->mem);
  (void)hipSetDevice(cur);
  delete mesh;
  if (e != hipSuccess) return hip_fail(e, "free_tetmesh");
  if (ef != hipSuccess) return hip_fail(ef, "hipFree");
  return CCSP_OK;
}

int tetmesh_info(const TetMesh* mesh, int64_t* n_tets, int64_t* device_bytes) {
  if (!mesh) return fail(CCSP_E_ARG, "tetmesh_info: null mesh");
  if (n_tets) *n_tets = mesh->nt;
  if (device_bytes) *device_bytes = (int64_t)mesh->bytes;
  return CCSP_OK;
}

int trace_rays3d(const TetMesh* mesh, const int32_t* o, const int32_t* d, const int32_t* start,
                 int64_t n, int32_t flags, int32_t step_limit, const Tune3d* tune,
                 int32_t* hit_prim, double* hit_t, int32_t* steps, void* stream) {
  if (!mesh) return fail(CCSP_E_ARG, "trace_rays3d: null mesh");
  if (n < 0 || n > INT32_MAX) return fail(CCSP_E_ARG, "trace_rays3d: n %lld out of range", (long long)n);
  if (step_limit < 0) return fail(CCSP_E_ARG, "trace_rays3d: negative step_limit");
  if (flags & ~(CCSP_TRACE_INPUT_ORDER | CCSP_TRACE_TIMED)) return fail(CCSP_E_ARG, "trace_rays3d: unknown flags 0x%x", flags);
  if (n == 0) return CCSP_OK;
  if (!o || !d || !start || !hit_prim || !hit_t || !steps)
    return fail(CCSP_E_ARG, "trace_rays3d: null array");
  if ((reinterpret_cast<uintptr_t>(hit_t) & 7) || (reinterpret_cast<uintptr_t>(o) & 3) ||
      (reinterpret_cast<uintptr_t>(d) & 3) || (reinterpret_cast<uintptr_t>(start) & 3) ||
      (reinterpret_cast<uintptr_t>(hit_prim) & 3) || (reinterpret_cast<uintptr_t>(steps) & 3))
    return fail(CCSP_E_ARG, "trace_rays3d: misaligned array");
  int wg = 256, wpc = 12, claim = 256, refill = 8, bin_key = 1;
  if (tune) {
    if (tune->wg_size) wg = tune->wg_size;
    if (tune->waves_per_cu) wpc = tune->waves_per_cu;
    if (tune->rays_per_claim) claim = tune->rays_per_claim;
    if (tune->refill_min) refill = tune->refill_min;
    if (tune->bin_key) bin_key = tune->bin_key;
  }
  if (bin_key != 1 && bin_key != 2) return fail(CCSP_E_ARG, "bin_key %d must be 1 or 2", bin_key);
  const int dirs = bin_key == 2;
  if (wg < 64 || wg > 512 || wg % 64) return fail(CCSP_E_ARG, "wg_size %d must be 64..512, multiple of 64", wg);
  if (wpc < 1 || wpc > 64) return fail(CCSP_E_ARG, "waves_per_cu %d must be 1..64", wpc);
  if (claim < kTile || claim > 65536 || claim % kTile)
    return fail(CCSP_E_ARG, "rays_per_claim %d must be 64..65536, multiple of 64", claim);
  if (refill < 1 || refill > 64) return fail(CCSP_E_ARG, "refill_min %d must be 1..64", refill);
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != mesh->device) return fail(CCSP_E_ARG, "trace_rays3d: the mesh lives on device %d, not %d", mesh->device, cur);
  Dev3* ds = nullptr;
  const int rc = dev_state(&ds);
  if (rc != CCSP_OK) return rc;
  unsigned long long* counter = ds->counters + (size_t)(ds->next.fetch_add(1) % kCounterGroups) * kChunks;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t limit = (step_limit == 0 || step_limit > mesh->nt) ? mesh->nt : step_limit;
  Rays3Dev io{o, d, start, hit_prim, hit_t, steps, n, (int32_t)limit};
  const int waves = ds->cus * wpc;
  const int64_t need = (n + 63) / 64;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((waves + wg / 64 - 1) / (wg / 64), (need + wg / 64 - 1) / (wg / 64)));
  const bool timed = flags & CCSP_TRACE_TIMED;
  std::unique_lock<std::mutex> time_lock(ds->time_mu, std::defer_lock);
  if (timed) {
    time_lock.lock();
    e = hipEventRecord(ds->ev[0], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  const bool bin = !(flags & CCSP_TRACE_INPUT_ORDER);
  std::unique_lock<std::mutex> bin_lock(ds->bin_mu);
  RayRec3* recs = nullptr;
  {
    size_t tmp = 0;
    const size_t need_b = bin_bytes(n, &tmp);
    if (need_b > ds->bin_ws_bytes) {
      if (ds->bin_ws) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ds->bin_ws);
        ds->bin_ws = nullptr;
        ds->bin_ws_bytes = 0;
      }
      e = hipMalloc(&ds->bin_ws, need_b);
      if (e != hipSuccess) {
        ds->bin_ws = nullptr;
        return fail(CCSP_E_OOM, "ray binning scratch of %zu bytes: %s", need_b, hipGetErrorString(e));
      }
      ds->bin_ws_bytes = need_b;
    }
    // the shared scratch may still be in use by a trace on another stream
    if (ds->bin_last_stream != st) {
      e = hipStreamWaitEvent(st, ds->bin_free, 0);
      if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    recs = binned_records(ds, tmp, n);
    const int nchunks = (int)((n + kBinChunk - 1) / kBinChunk);
    uint32_t* H = reinterpret_cast<uint32_t*>(ds->bin_ws);
    uint32_t* Hoff = reinterpret_cast<uint32_t*>(static_cast<char*>(ds->bin_ws) +
                                                 align256((size_t)kMaxBuckets * nchunks * sizeof(uint32_t)));
    void* scan_tmp = static_cast<char*>(ds->bin_ws) + 2 * align256((size_t)kMaxBuckets * nchunks * sizeof(uint32_t));
    if (bin) {
      const int nbk = dirs ? kMaxBuckets : kCells;
      hipLaunchKernelGGL(bin_count, dim3(nchunks), dim3(kBinThreads), 0, st, o, d, n, dirs, nbk, H, nchunks);
      e = ccsp::launch_exclusive_scan(H, Hoff, (int64_t)nbk * nchunks,
                                      static_cast<uint32_t*>(scan_tmp), st);
      if (e != hipSuccess) return hip_fail(e, "bucket scan");
      hipLaunchKernelGGL(bin_scatter, dim3(nchunks), dim3(kBinThreads), 0, st, mesh->first,
                         (int32_t)mesh->nt, io, dirs, nbk, Hoff, nchunks, recs);
    } else {
      hipLaunchKernelGGL(start_records, dim3((unsigned)((n + kBinThreads - 1) / kBinThreads)), dim3(kBinThreads), 0, st,
                         mesh->first, (int32_t)mesh->nt, io, recs);
    }
  }
  if (timed) {
    e = hipEventRecord(ds->ev[1], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, counter);
  hipLaunchKernelGGL(walk3d, dim3(grid), dim3(wg), (wg / 64) * kTileBytes, st, mesh->slot, io, recs,
                     counter, claim, refill);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "walk3d launch");
  e = hipEventRecord(ds->bin_free, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  ds->bin_last_stream = st;
  if (timed) {
    e = hipEventRecord(ds->ev[2], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ds->timed = true;
  }
  return CCSP_OK;
}

int trace3d_stage_times(float* bin_ms, float* walk_ms) {
  Dev3* ds = nullptr;
  const int rc = dev_state(&ds);
  if (rc != CCSP_OK) return rc;
  std::lock_guard<std::mutex> lk(ds->time_mu);
  if (!ds->timed) return fail(CCSP_E_ARG, "trace3d_stage_times: no timed trace on this device");
  hipError_t e = hipEventSynchronize(ds->ev[2]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  float b = 0, w = 0;
  e = hipEventElapsedTime(&b, ds->ev[0], ds->ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&w, ds->ev[1], ds->ev[2]);
  if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
  if (bin_ms) *bin_ms = b;
  if (walk_ms) *walk_ms = w;
  return CCSP_OK;
}

}  // extern "C"
