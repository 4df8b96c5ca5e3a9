// Point location on the GPU: the triangle containing each query point (paper Sec. 5.2).
//
// The scene carries a grid of seeds (a point strictly inside a known triangle per cell). For a
// query q the walk starts at the seed p of q's cell and follows the segment from p to q through
// the triangulation, to which constraints are transparent here (the `through` word of the
// binary64 slots), until it reaches the triangle that contains q. Decisions use the exact line
// through p and q (orientation predicates, binary64 filter then exact expansion), with the same
// tie rule as the ray walk: a vertex on the line counts as LEFT. The walk stops in the first
// triangle whose exit edge does not have q strictly on its outer side: the segment enters that
// triangle before q and leaves it after q, so q is in the closed triangle.
//
// One thread per query: the walks are a few steps long (the seed grid holds about one cell per
// four triangles), so the launch is a plain grid, not a persistent one.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "exact.hpp"
#include "walk.hpp"

namespace ccsp {

namespace {

// Sign of the orientation of (a, b, c): > 0 if c is left of the directed line a->b. A binary64
// filter (error bound (3 + 16u)u of the products' magnitude, taken as 2^-51) and the exact
// expansion when it cannot decide.
__device__ __forceinline__ int orient64(double2 a, double2 b, double2 c) {
  const double l = (b.x - a.x) * (c.y - a.y);
  const double r = (b.y - a.y) * (c.x - a.x);
  const double det = l - r, sum = fabs(l) + fabs(r);
  if (fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return orient_exact(a.x, a.y, b.x, b.y, c.x, c.y);
}

__device__ __forceinline__ double2 vtx(const SceneDev& sc, int v) { return sc.v64[v]; }

__global__ void __launch_bounds__(256)
locate_kernel(SceneDev sc, const double2* __restrict__ q_in, int64_t n, int32_t* __restrict__ tri_out,
              int32_t* __restrict__ status_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 Q = q_in[i];
  if (!isfinite(Q.x) || !isfinite(Q.y)) {
    tri_out[i] = -1;
    status_out[i] = -2;
    return;
  }
  const double hi = (double)(sc.seed_g - 1);
  const int cx = (int)fmin(fmax(floor((Q.x - sc.seed_x0) * sc.seed_inv), 0.0), hi);
  const int cy = (int)fmin(fmax(floor((Q.y - sc.seed_y0) * sc.seed_inv), 0.0), hi);
  const SeedCell seed = sc.seeds[(int64_t)cy * sc.seed_g + cx];
  const double2 P = make_double2(seed.x, seed.y);
  int t = seed.tri;
  const int4 tv = sc.triv[t];
  const double2 V[3] = {vtx(sc, tv.x), vtx(sc, tv.y), vtx(sc, tv.z)};
  double2 A, B, D;  // exit edge (A, B) of the current triangle; D the vertex opposite it
  int e;
  if (Q.x == P.x && Q.y == P.y) {  // the seed itself: strictly inside its triangle
    tri_out[i] = sc.orig[t];
    status_out[i] = 0;
    return;
  }
  {
    // first triangle: the exit edge i has v[i+1] RIGHT and v[i+2] LEFT of the line p->q
    const bool L0 = orient64(P, Q, V[0]) >= 0, L1 = orient64(P, Q, V[1]) >= 0,
               L2 = orient64(P, Q, V[2]) >= 0;
    e = (!L1 && L2) ? 0 : ((!L2 && L0) ? 1 : 2);  // p is strictly inside: one edge qualifies
    A = V[(e + 1) % 3];
    B = V[(e + 2) % 3];
    D = V[e];
  }
  int status = -3;  // the step guard (never expected)
  for (int steps = 0; steps <= sc.ntri; ++steps) {
    if (orient64(A, B, Q) >= 0) {  // q is not beyond the exit edge: it is in this triangle
      const int sab = orient64(A, B, Q), sbd = orient64(B, D, Q), sda = orient64(D, A, Q);
      status = (sab > 0 && sbd > 0 && sda > 0) ? 0 : ((sbd >= 0 && sda >= 0) ? 1 : -3);
      break;
    }
    const Slot64 sl = sc.slot64[3 * t + e];
    if (sl.through < 0) {  // the segment leaves the triangulation before q
      status = -1;
      break;
    }
    t = sl.through >> 2;
    const int eb = sl.through & 3;  // entry edge in the neighbour: (v[eb+1], v[eb+2]) = (B, A)
    const double2 C = make_double2(sl.x, sl.y);  // its vertex opposite the entry edge
    if (orient64(P, Q, C) >= 0) {  // C LEFT: exit through edge eb+1 = (A, C)
      e = eb == 2 ? 0 : eb + 1;
      D = B;
      B = C;
    } else {  // C RIGHT: exit through edge eb+2 = (C, B)
      e = eb == 0 ? 2 : eb - 1;
      D = A;
      A = C;
    }
  }
  tri_out[i] = status >= 0 ? sc.orig[t] : -1;
  status_out[i] = status;
}

}  // namespace

hipError_t launch_locate(const SceneDev& sc, const double2* q, int64_t n, int32_t* tri,
                         int32_t* status, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(locate_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, sc, q, n, tri,
                     status);
  return hipGetLastError();
}

}  // namespace ccsp
