// Per-ray decisions shared by the walk and the ray binning: the side of a vertex relative to the
// ray (binary32 filter, binary64 filter, exact expansion), the first triangle's exit edge and the
// hit distance. Device code only; every file including it is compiled with -ffp-contract=off,
// which the filter bounds and the hit distance formula assume.
#pragma once
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
static __device__ __attribute__((noinline)) int side_exact_call(double ox, double oy, double dx,
                                                                double dy, double vx, double vy) {
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
static __device__ __attribute__((noinline)) bool left_deferred(double2 o, double2 d,
                                                               const double2* v64, int vid,
                                                               unsigned* n_exact) {
  const double2 v = v64[vid];
  unsigned n = 0;
  const bool l = left64<COUNT>(o.x, o.y, d.x, d.y, v.x, v.y, n);
  if (COUNT) *n_exact += n;
  return l;
}

__device__ __forceinline__ double hit_t(const double4 g, double ox, double oy, double dx,
                                        double dy) {
  const double ex = g.z - g.x;
  const double ey = g.w - g.y;
  const double num = (g.x - ox) * ey - (g.y - oy) * ex;
  const double den = dx * ey - dy * ex;
  return num / den;
}

__device__ __forceinline__ double lohi(int lo, int hi) { return __hiloint2double(hi, lo); }

// The exit edge i of the first triangle is the one whose first endpoint is RIGHT of the ray and
// whose second is LEFT (three candidates: nothing is known about the entry).
__device__ __forceinline__ int first_edge(bool L0, bool L1, bool L2) {
  return (!L1 && L2) ? 0 : ((!L2 && L0) ? 1 : ((!L0 && L1) ? 2 : -1));
}

// Exit slot (3 * internal triangle + exit edge) of a ray's first triangle (Sec. 7.2: three
// candidate edges, nothing being known about an entry). x, y: the triangle's vertices relative to
// the scene origin in binary32, `tri` its internal id. Signs the binary32 filter leaves open go
// to the binary64 filter and then the exact expansion, so the result is exact in either precision
// mode. Returns -1 if no edge qualifies (the origin is not inside the triangle).
template <bool COUNT>
__device__ __forceinline__ int first_exit_slot(const Ray32& r, double2 o, double2 d, float x0,
                                               float x1, float x2, float y0, float y1, float y2,
                                               int tri, const SceneDev& sc, unsigned& fb32,
                                               unsigned& fb64) {
  int s0 = side32(r, x0, y0);
  int s1 = side32(r, x1, y1);
  int s2 = side32(r, x2, y2);
  if ((s0 == 0) | (s1 == 0) | (s2 == 0)) {
    const int4 tv = sc.triv[tri];
    if (s0 == 0) { if (COUNT) ++fb32; s0 = left_deferred<COUNT>(o, d, sc.v64, tv.x, &fb64) ? 1 : -1; }
    if (s1 == 0) { if (COUNT) ++fb32; s1 = left_deferred<COUNT>(o, d, sc.v64, tv.y, &fb64) ? 1 : -1; }
    if (s2 == 0) { if (COUNT) ++fb32; s2 = left_deferred<COUNT>(o, d, sc.v64, tv.z, &fb64) ? 1 : -1; }
  }
  const int e = first_edge(s0 > 0, s1 > 0, s2 > 0);
  return e >= 0 ? 3 * tri + e : -1;
}

// The ray in the binary32 frame of the scene (origin relative to the scene origin).
__device__ __forceinline__ Ray32 ray32(double ox, double oy, double dx, double dy, double org_x,
                                       double org_y) {
  return Ray32{(float)(ox - org_x), (float)(oy - org_y), (float)dx, (float)dy};
}

}  // namespace ccsp
