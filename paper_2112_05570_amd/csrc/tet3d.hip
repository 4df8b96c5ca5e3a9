// Persistent stackless walk through a 3D constrained tetrahedralisation for gfx950 (CDNA4,
// wave64): the 3D form of the triangulation walk (Sec. 1.3 and 1.4: one decision per visited
// tetrahedron, the exit face among the three faces other than the entry face; Sec. 7.2).
//
// Mapping to the hardware:
//  * Like the 2D walk this is a chain of dependent gathers with a few flops each: bound by memory
//    latency, not by MFMA or ALUs. One step is one 16-byte load, the slot of the exit face:
//    neighbour and its entry face, the neighbour's fourth vertex (the apex) and the order of the
//    shared face's vertices seen from the neighbour. The face's own three vertices travel in
//    registers (relative to the origin), so a step needs no other memory.
//  * Two Plücker signs per step, both of the form X . m with m = d x W computed once per step
//    (W the apex, X a face vertex, all relative to o). Integer grid inputs make m exact in
//    binary64 (|m| < 2^40); X . m is rounded once per product and per sum, and accepted when a
//    forward error bound proves its sign. Otherwise an exact int64 evaluation decides, and a zero
//    takes the sign of the symbolically moved line (origin o + (e, e^2, e^3), direction
//    d + (e^10, e^20, e^30)).
//  * Waves are persistent: each takes rays_per_claim rays per global atomic and refills idle
//    lanes as soon as refill_min of its 64 lanes are idle. Every lane issues exactly one round of
//    loads per iteration, whatever its state (fetch the ray, read the start tetrahedron, or
//    read an exit slot), so lanes in different states share one memory round trip.
//
// Compiled with -ffp-contract=off: the error bound and the hit distance assume every operation
// is rounded separately.
#include <hip/hip_runtime.h>

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

namespace ccsp {
void set_last_error(const char* msg);
}

struct TetMesh {
  int device = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  const int4* slot = nullptr;   // 4 per tetrahedron
  const int4* first = nullptr;  // 3 per tetrahedron: the four vertices, 12 int32
  int64_t nt = 0, nv = 0, np = 0;
};

namespace {

constexpr int kGridBits = 19;
constexpr int32_t kGrid = 1 << kGridBits;
constexpr int32_t kMask = kGrid - 1;

// FACE[f][i], the local vertices of face f (opposite vertex f) counter-clockwise seen from
// outside: (1,2,3), (0,3,2), (0,1,3), (0,2,1); nibble 3f+i.
constexpr uint64_t kFace = 0x120310230321ull;
// position of local vertex l in FACE[j] (l != j); 2 bits at 4j+l
constexpr uint32_t kPos = 0x18846090u;

__host__ __device__ __forceinline__ int face_v(int f, int i) {
  return (int)((kFace >> (4 * (3 * f + i))) & 0xF);
}
__host__ __device__ __forceinline__ int face_pos(int j, int l) {
  return (int)((kPos >> (2 * (4 * j + l))) & 3);
}

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

__global__ void __launch_bounds__(512)
walk3d(const int4* __restrict__ slots, const int4* __restrict__ firsts, int32_t nt, Rays3Dev io,
       unsigned long long* __restrict__ counter, int claim, int refill_min) {
  enum : int { IDLE = 0, FETCH = 1, FIRST = 2, WALK = 3 };
  const int lane = threadIdx.x & 63;
  int state = IDLE;
  int64_t ray = 0;
  V3 o{0, 0, 0}, d{0, 0, 0};
  V3 A{0, 0, 0}, B{0, 0, 0}, C{0, 0, 0};  // the exit face in its tetrahedron's face order
  int s = 0, steps = 0;                   // start tetrahedron (FIRST) or exit slot (WALK)
  int64_t next = 0, end = 0;              // the wave's claimed rays
  bool drained = false;
  for (;;) {
    const unsigned long long idle = __ballot(state == IDLE);
    const int nidle = __popcll(idle);
    if (drained && nidle == 64) break;
    if (!drained && nidle >= refill_min) {
      const int rank = __popcll(idle & ((1ull << lane) - 1));
      int served = 0;
      while (served < nidle) {
        if (next == end) {
          unsigned long long b = 0;
          if (lane == 0) b = atomicAdd(counter, (unsigned long long)claim);
          const int64_t base = (int64_t)bcast64(b);
          if (base >= io.n) {
            drained = true;
            break;
          }
          next = base;
          end = min(base + claim, io.n);
        }
        const int take = (int)min((int64_t)(nidle - served), end - next);
        if (state == IDLE && rank >= served && rank < served + take) {
          ray = next + (rank - served);
          state = FETCH;
        }
        served += take;
        next += take;
      }
    }
    // ---- issue: one round of loads for every busy lane
    const int st_now = state;
    int4 R0 = make_int4(0, 0, 0, 0), R1 = R0, R2 = R0;
    if (st_now == WALK) {
      R0 = slots[s];
    } else if (st_now == FIRST) {
      const int4* p = firsts + 3 * (int64_t)s;
      R0 = p[0];
      R1 = p[1];
      R2 = p[2];
    } else if (st_now == FETCH) {
      const int32_t* po = io.o + 3 * ray;
      const int32_t* pd = io.d + 3 * ray;
      R0 = make_int4(po[0], po[1], po[2], pd[0]);
      R1 = make_int4(pd[1], pd[2], io.start[ray], 0);
    }
    __asm__ volatile("" ::"v"(R0.x), "v"(R0.y), "v"(R0.z), "v"(R0.w), "v"(R1.x), "v"(R1.y),
                     "v"(R1.z), "v"(R1.w), "v"(R2.x), "v"(R2.y), "v"(R2.z), "v"(R2.w));
    // ---- process
    if (st_now == WALK) {
      const int word = R0.x;
      if (word < -1) {
        const V3 a = sub(V3{R0.y, R0.z, R0.w & kMask}, o);
        finish(io, ray, -2 - word, hit_t(A, B, C, a, d), steps);
        state = IDLE;
      } else if (word == -1 || steps >= io.limit) {
        finish(io, ray, word == -1 ? -1 : -2, INFINITY, steps);
        state = IDLE;
      } else {
        const int nb = word >> 2, j = word & 3, perm = (R0.w >> kGridBits) & 3;
        const V3 W = sub(V3{R0.y, R0.z, R0.w & kMask}, o);
        // the entry face in the neighbour's face order: (A, C, B), (B, A, C) or (C, B, A)
        const V3 P = sel(perm == 0, A, sel(perm == 1, B, C));
        const V3 Q = sel(perm == 0, C, sel(perm == 1, A, B));
        const V3 R = sel(perm == 0, B, sel(perm == 1, C, A));
        ++steps;
        const M3 m = cross_dw(d, W);
        const int sp = plucker(m, d, W, P);
        const int sx = plucker(m, d, W, sp > 0 ? R : Q);
        const int k = sp > 0 ? (sx < 0 ? 1 : 0) : (sx > 0 ? 2 : 0);
        const int e = face_v(j, k);
        int code[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int l = face_v(e, i);
          code[i] = l == j ? 3 : face_pos(j, l);
        }
        A = sel4(code[0], P, Q, R, W);
        B = sel4(code[1], P, Q, R, W);
        C = sel4(code[2], P, Q, R, W);
        s = 4 * nb + e;
      }
    } else if (st_now == FIRST) {
      // vertices relative to o: x0 y0 z0 x1 | y1 z1 x2 y2 | z2 x3 y3 z3
      const V3 v0 = sub(V3{R0.x, R0.y, R0.z}, o), v1 = sub(V3{R0.w, R1.x, R1.y}, o);
      const V3 v2 = sub(V3{R1.z, R1.w, R2.x}, o), v3 = sub(V3{R2.y, R2.z, R2.w}, o);
      // strictly inside: A . (B x C) > 0 for every face (A, B, C) in outside order
      const bool inside = triple_pos(v1, v2, v3) && triple_pos(v0, v3, v2) &&
                          triple_pos(v0, v1, v3) && triple_pos(v0, v2, v1);
      int e = -1;
      if (inside) {
        const M3 m0 = cross_dw(d, v0), m1 = cross_dw(d, v1), m2 = cross_dw(d, v2);
        const int s01 = plucker(m0, d, v0, v1), s02 = plucker(m0, d, v0, v2);
        const int s03 = plucker(m0, d, v0, v3), s12 = plucker(m1, d, v1, v2);
        const int s13 = plucker(m1, d, v1, v3), s23 = plucker(m2, d, v2, v3);
        // face edges in outside order; the first face with all three positive
        if (s12 > 0 && s23 > 0 && s13 < 0) e = 0;
        else if (s03 > 0 && s23 < 0 && s02 < 0) e = 1;
        else if (s01 > 0 && s13 > 0 && s03 < 0) e = 2;
        else if (s02 > 0 && s12 < 0 && s01 < 0) e = 3;
      }
      if (e < 0) {
        finish(io, ray, -3, INFINITY, 0);
        state = IDLE;
      } else {
        A = sel4(face_v(e, 0), v0, v1, v2, v3);
        B = sel4(face_v(e, 1), v0, v1, v2, v3);
        C = sel4(face_v(e, 2), v0, v1, v2, v3);
        steps = 1;
        s = 4 * s + e;
        state = WALK;
      }
    } else if (st_now == FETCH) {
      o = V3{R0.x, R0.y, R0.z};
      d = V3{R0.w, R1.x, R1.y};
      s = R1.z;
      const bool ok = on_grid(o.x) && on_grid(o.y) && on_grid(o.z) && dir_ok(d.x) &&
                      dir_ok(d.y) && dir_ok(d.z) && (d.x != 0 || d.y != 0 || d.z != 0) &&
                      s >= 0 && s < nt;
      if (ok) {
        state = FIRST;
      } else {
        finish(io, ray, -3, INFINITY, 0);
        state = IDLE;
      }
    }
  }
}

__global__ void reset_counter(unsigned long long* c) { *c = 0; }

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

constexpr int kCounters = 1024;

struct Dev3 {
  unsigned long long* counters = nullptr;
  int cus = 0;
  std::atomic<uint64_t> next{0};
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
    e = hipMalloc(&ds.counters, kCounters * sizeof(unsigned long long));
    if (e != hipSuccess) {
      ds.counters = nullptr;
      return fail(CCSP_E_OOM, "counter allocation failed: %s", hipGetErrorString(e));
    }
  }
  *out = &ds;
  return CCSP_OK;
}

int64_t orient_host(const int32_t* a, const int32_t* b, const int32_t* c, const int32_t* q) {
  const int64_t u0 = (int64_t)b[0] - a[0], u1 = (int64_t)b[1] - a[1], u2 = (int64_t)b[2] - a[2];
  const int64_t v0 = (int64_t)c[0] - a[0], v1 = (int64_t)c[1] - a[1], v2 = (int64_t)c[2] - a[2];
  const int64_t w0 = (int64_t)q[0] - a[0], w1 = (int64_t)q[1] - a[1], w2 = (int64_t)q[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
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

  std::vector<int4> slot((size_t)(4 * T)), first((size_t)(3 * T));
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
      bool ids = true;
      for (int i = 0; i < 4; ++i) ids = ids && v[i] >= 0 && v[i] < V;
      if (!ids) {
        bad(t, "tetrahedron %lld: vertex id out of range", (long long)t);
        break;
      }
      const int32_t* P[4] = {X + 3 * (int64_t)v[0], X + 3 * (int64_t)v[1], X + 3 * (int64_t)v[2], X + 3 * (int64_t)v[3]};
      if (orient_host(P[0], P[1], P[2], P[3]) <= 0) {
        bad(t, "tetrahedron %lld is not positively oriented", (long long)t);
        break;
      }
      first[3 * t + 0] = make_int4(P[0][0], P[0][1], P[0][2], P[1][0]);
      first[3 * t + 1] = make_int4(P[1][1], P[1][2], P[2][0], P[2][1]);
      first[3 * t + 2] = make_int4(P[2][2], P[3][0], P[3][1], P[3][2]);
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
          if (w[j] < 0 || w[j] >= V ||
              orient_host(X + 3 * (int64_t)fa, X + 3 * (int64_t)fb, X + 3 * (int64_t)fc, X + 3 * (int64_t)w[j]) <= 0) {
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
          r = make_int4((nb << 2) | j, apex[0], apex[1], apex[2] | (perm << kGridBits));
        }
        slot[4 * t + i] = r;
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
                 int64_t n, int32_t step_limit, const Tune3d* tune, int32_t* hit_prim,
                 double* hit_t, int32_t* steps, void* stream) {
  if (!mesh) return fail(CCSP_E_ARG, "trace_rays3d: null mesh");
  if (n < 0 || n > INT32_MAX) return fail(CCSP_E_ARG, "trace_rays3d: n %lld out of range", (long long)n);
  if (step_limit < 0) return fail(CCSP_E_ARG, "trace_rays3d: negative step_limit");
  if (n == 0) return CCSP_OK;
  if (!o || !d || !start || !hit_prim || !hit_t || !steps)
    return fail(CCSP_E_ARG, "trace_rays3d: null array");
  if ((reinterpret_cast<uintptr_t>(hit_t) & 7) || (reinterpret_cast<uintptr_t>(o) & 3) ||
      (reinterpret_cast<uintptr_t>(d) & 3) || (reinterpret_cast<uintptr_t>(start) & 3) ||
      (reinterpret_cast<uintptr_t>(hit_prim) & 3) || (reinterpret_cast<uintptr_t>(steps) & 3))
    return fail(CCSP_E_ARG, "trace_rays3d: misaligned array");
  int wg = 256, wpc = 32, claim = 256, refill = 8;
  if (tune) {
    if (tune->wg_size) wg = tune->wg_size;
    if (tune->waves_per_cu) wpc = tune->waves_per_cu;
    if (tune->rays_per_claim) claim = tune->rays_per_claim;
    if (tune->refill_min) refill = tune->refill_min;
  }
  if (wg < 64 || wg > 512 || wg % 64) return fail(CCSP_E_ARG, "wg_size %d must be 64..512, multiple of 64", wg);
  if (wpc < 1 || wpc > 64) return fail(CCSP_E_ARG, "waves_per_cu %d must be 1..64", wpc);
  if (claim < 64 || claim > 65536 || claim % 64) return fail(CCSP_E_ARG, "rays_per_claim %d must be 64..65536, multiple of 64", claim);
  if (refill < 1 || refill > 64) return fail(CCSP_E_ARG, "refill_min %d must be 1..64", refill);
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != mesh->device) return fail(CCSP_E_ARG, "trace_rays3d: the mesh lives on device %d, not %d", mesh->device, cur);
  Dev3* ds = nullptr;
  const int rc = dev_state(&ds);
  if (rc != CCSP_OK) return rc;
  unsigned long long* counter = ds->counters + (ds->next.fetch_add(1) % kCounters);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t limit = (step_limit == 0 || step_limit > mesh->nt) ? mesh->nt : step_limit;
  Rays3Dev io{o, d, start, hit_prim, hit_t, steps, n, (int32_t)limit};
  const int waves = ds->cus * wpc;
  const int64_t need = (n + 63) / 64;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((waves + wg / 64 - 1) / (wg / 64), (need + wg / 64 - 1) / (wg / 64)));
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, counter);
  hipLaunchKernelGGL(walk3d, dim3(grid), dim3(wg), 0, st, mesh->slot, mesh->first, (int32_t)mesh->nt, io, counter, claim, refill);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "walk3d launch");
  return CCSP_OK;
}

}  // extern "C"
