// Annealing of a constrained triangulation by edge flips on the GPU (paper Sec. 3.2.7 for the move,
// Sec. 3.1 for the acceptance), with the total edge length as the energy: the C-ABI flip_anneal of
// ccsp_objective.h.
//
// A flip of the unconstrained interior edge (b, c) between triangles t = (a, b, c) and
// u = (d, c, b) replaces it by (a, d) when the quad a, b, d, c is strictly convex (exact
// orientations). It reads and writes t, u and the up to four triangles across their other edges
// (its touched triangles). Each round takes four passes:
//   flip_eval    (per slot) tests every candidate against the triangulation as the round found
//                it (convexity, change of weight, Metropolis with its own uniform) and records, in
//                both of the edge's slots, the id of its canonical slot if the flip would be
//                accepted;
//   flip_best    (per triangle) the accepted flip of highest (priority, canonical slot) among
//                those that touch the triangle: the edges of the triangle and of its neighbours;
//   flip_select  (per triangle) keeps an accepted flip when it is the best of all its touched
//                triangles, i.e. beats every other accepted flip touching one of them;
//   flip_apply   (per triangle) rewrites the kept flips, whose touched triangles are pairwise
//                disjoint, counts them per block, and clears the slot's record for the next round.
// The first three only read the triangulation, the fourth writes disjoint sets, so a round is the
// same as applying its kept flips one after another. Priorities and uniforms come from a
// counter-based generator, SplitMix64 (Steele, Lea and Flood, 2014): outputs k + 1 and k + 2 of the
// sequence from state seed, k = 2 * (round * 2^32 + canonical slot).
//
// Every triangle id read from the arrays is checked against the triangle count before use.
// Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "ccsp_objective.h"
#include "exact.hpp"
#include "walk.hpp"

namespace ccsp {
namespace {

constexpr int kFlipThreads = 256;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t priority(uint64_t seed, int round, int slot) {
  const uint64_t k = 2ull * (((uint64_t)round << 32) + (uint64_t)slot);
  return splitmix64(seed + (k + 1) * kGolden);
}

__device__ __forceinline__ double uniform(uint64_t seed, int round, int slot) {
  const uint64_t k = 2ull * (((uint64_t)round << 32) + (uint64_t)slot);
  return (double)(splitmix64(seed + (k + 2) * kGolden) >> 11) * 0x1p-53;
}

struct Tri {
  int32_t* v;
  int32_t* nbr;
  int32_t* prim;
  int32_t nt;
  int32_t nv;
  const int32_t* line;    // per vertex: its original edge if it is a Steiner vertex on one, else -1;
  const int32_t* prim_v;  // the two end vertices of each original edge; both null when not given
  int32_t np;
};

__device__ __forceinline__ int orient_sign(double2 a, double2 b, double2 c) {
  const double l = (b.x - a.x) * (c.y - a.y);
  const double r = (b.y - a.y) * (c.x - a.x);
  const double det = l - r, sum = fabs(l) + fabs(r);
  if (fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return orient_exact(a.x, a.y, b.x, b.y, c.x, c.y);
}

__device__ __forceinline__ double seg_len(double2 p, double2 q) {
  const double dx = q.x - p.x, dy = q.y - p.y;
  return sqrt(dx * dx + dy * dy);
}

// Local index in w of its edge shared with t, or -1.
__device__ __forceinline__ int back_of(const Tri& T, int w, int t) {
  for (int j = 0; j < 3; ++j)
    if (T.nbr[3 * w + j] == t) return j;
  return -1;
}

__device__ __forceinline__ bool valid_tri(const Tri& T, int x) { return x >= 0 && x < T.nt; }
__device__ __forceinline__ bool valid_vertex(const Tri& T, int x) { return x >= 0 && x < T.nv; }

__device__ __forceinline__ bool on_original(const Tri& T, int v, int k) {
  const int lv = T.line[v];
  if (lv >= 0) return lv == k;
  return T.prim_v[2 * k] == v || T.prim_v[2 * k + 1] == v;
}

// Whether the triangle (x, y, z) has all three vertices on one original edge: zero area in intent,
// which the exact convexity test lets through when rounding leaves a Steiner vertex off its line.
__device__ __forceinline__ bool flat_on_original(const Tri& T, int x, int y, int z) {
  if (!T.line) return false;
  const int ks[3] = {T.line[x], T.line[y], T.line[z]};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const int k = ks[m];
    if (k >= 0 && k < T.np && on_original(T, x, k) && on_original(T, y, k) && on_original(T, z, k))
      return true;
  }
  return false;
}

// Flip counts of a round are spread over this many counters, a block adding into one of them.
constexpr int kCountLanes = 64;

// Scratch of a call: no accepted flip recorded, no flip counted.
__global__ void __launch_bounds__(kFlipThreads)
flip_clear(int32_t* __restrict__ key, int64_t n, unsigned long long* __restrict__ count,
           int64_t n_count) {
  const int64_t stride = (int64_t)gridDim.x * kFlipThreads;
  for (int64_t s = (int64_t)blockIdx.x * kFlipThreads + threadIdx.x; s < n || s < n_count;
       s += stride) {
    if (s < n) key[s] = -1;
    if (s < n_count) count[s] = 0;
  }
}

// One thread per slot: the slot of a candidate edge in the triangle of lower id does the work.
__global__ void __launch_bounds__(kFlipThreads)
flip_eval(Tri T, const double2* __restrict__ xy, double temperature, uint64_t seed, int round,
          int32_t* __restrict__ key) {
  const int s = blockIdx.x * kFlipThreads + threadIdx.x;
  if (s >= 3 * T.nt) return;
  const int t = s / 3, i = s - 3 * t;
  const int u = T.nbr[s];
  if (!valid_tri(T, u) || u <= t) return;  // hull, malformed, or the slot of the other triangle
  int res = -1;
  const int j = back_of(T, u, t);
  if (T.prim[s] < 0 && j >= 0) {
    const int a = T.v[3 * t + i], b = T.v[3 * t + (i + 1) % 3], c = T.v[3 * t + (i + 2) % 3];
    const int d = T.v[3 * u + j];
    if (!valid_vertex(T, a) || !valid_vertex(T, b) || !valid_vertex(T, c) || !valid_vertex(T, d))
      return;
    const double2 pa = xy[a], pb = xy[b], pc = xy[c], pd = xy[d];
    if (orient_sign(pa, pb, pd) > 0 && orient_sign(pa, pd, pc) > 0 &&
        !flat_on_original(T, a, b, d) && !flat_on_original(T, a, d, c)) {
      const double change = seg_len(pa, pd) - seg_len(pb, pc);
      if (change < 0.0 ||
          (temperature > 0.0 && uniform(seed, round, s) < exp(-change / temperature)))
        res = s;
    }
  }
  key[s] = res;
  if (j >= 0) key[3 * u + j] = res;
}

__global__ void __launch_bounds__(kFlipThreads)
flip_best(Tri T, const int32_t* __restrict__ key, uint64_t seed, int round,
          int32_t* __restrict__ best) {
  const int x = blockIdx.x * kFlipThreads + threadIdx.x;
  if (x >= T.nt) return;
  int top = -1;
  uint64_t top_p = 0;
  for (int h = -1; h < 3; ++h) {
    const int y = h < 0 ? x : T.nbr[3 * x + h];
    if (!valid_tri(T, y)) continue;
    for (int k = 0; k < 3; ++k) {
      const int s2 = key[3 * y + k];
      if (s2 < 0 || s2 == top) continue;
      const uint64_t p2 = priority(seed, round, s2);
      if (top < 0 || p2 > top_p || (p2 == top_p && s2 > top)) {
        top = s2;
        top_p = p2;
      }
    }
  }
  best[x] = top;
}

// One thread per triangle, over its three slots.
__global__ void __launch_bounds__(kFlipThreads)
flip_select(Tri T, const int32_t* __restrict__ key, const int32_t* __restrict__ best,
            uint8_t* __restrict__ keep) {
  const int t = blockIdx.x * kFlipThreads + threadIdx.x;
  if (t >= T.nt) return;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int s = 3 * t + i;
    bool win = key[s] == s;
    if (win) {
      const int u = T.nbr[s];  // valid: flip_eval accepted the flip
      win = best[t] == s && best[u] == s;
      for (int k = 0; k < 3 && win; ++k) {
        const int xt = T.nbr[3 * t + k], xu = T.nbr[3 * u + k];
        if (valid_tri(T, xt) && best[xt] != s) win = false;
        if (valid_tri(T, xu) && best[xu] != s) win = false;
      }
    }
    keep[s] = win ? 1 : 0;
  }
}

// Rewrites the flip of slot s; false if the adjacency is not symmetric (never for a kept flip).
__device__ __forceinline__ bool apply_one(const Tri& T, int s) {
  const int t = s / 3, i = s - 3 * t;
  const int u = T.nbr[s];
  const int j = back_of(T, u, t);
  if (j < 0) return false;
  const int i1 = i == 2 ? 0 : i + 1, i2 = i1 == 2 ? 0 : i1 + 1;
  const int j1 = j == 2 ? 0 : j + 1, j2 = j1 == 2 ? 0 : j1 + 1;
  const int a = T.v[3 * t + i], b = T.v[3 * t + i1], c = T.v[3 * t + i2];
  const int d = T.v[3 * u + j];
  const int nt1 = T.nbr[3 * t + i1], pt1 = T.prim[3 * t + i1];  // edge (c, a)
  const int nt2 = T.nbr[3 * t + i2], pt2 = T.prim[3 * t + i2];  // edge (a, b)
  const int nu1 = T.nbr[3 * u + j1], pu1 = T.prim[3 * u + j1];  // edge (b, d)
  const int nu2 = T.nbr[3 * u + j2], pu2 = T.prim[3 * u + j2];  // edge (d, c)
  T.v[3 * t] = a;
  T.v[3 * t + 1] = b;
  T.v[3 * t + 2] = d;
  T.nbr[3 * t] = nu1;
  T.nbr[3 * t + 1] = u;
  T.nbr[3 * t + 2] = nt2;
  T.prim[3 * t] = pu1;
  T.prim[3 * t + 1] = -1;
  T.prim[3 * t + 2] = pt2;
  T.v[3 * u] = a;
  T.v[3 * u + 1] = d;
  T.v[3 * u + 2] = c;
  T.nbr[3 * u] = nu2;
  T.nbr[3 * u + 1] = nt1;
  T.nbr[3 * u + 2] = t;
  T.prim[3 * u] = pu2;
  T.prim[3 * u + 1] = pt1;
  T.prim[3 * u + 2] = -1;
  if (valid_tri(T, nu1)) {
    const int k = back_of(T, nu1, u);
    if (k >= 0) T.nbr[3 * nu1 + k] = t;
  }
  if (valid_tri(T, nt1)) {
    const int k = back_of(T, nt1, t);
    if (k >= 0) T.nbr[3 * nt1 + k] = u;
  }
  return true;
}

// One thread per triangle: a triangle holds at most one kept flip (kept flips touch disjoint
// triangles), which its thread rewrites; the thread also clears the triangle's three records.
__global__ void __launch_bounds__(kFlipThreads)
flip_apply(Tri T, const uint8_t* __restrict__ keep, int32_t* __restrict__ key,
           unsigned long long* __restrict__ count) {
  const int t = blockIdx.x * kFlipThreads + threadIdx.x;
  bool flip = false;
  if (t < T.nt) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int s = 3 * t + i;
      key[s] = -1;  // the record is not read again this round
      if (!flip && keep[s]) flip = apply_one(T, s);
    }
  }
  const int n = __syncthreads_count(flip);
  if (threadIdx.x == 0 && n > 0) atomicAdd(count + blockIdx.x % kCountLanes, (unsigned long long)n);
}

}  // namespace
}  // namespace ccsp

extern "C" int flip_anneal(int64_t n_vertices, const double* xy, int64_t n_triangles,
                           int32_t* tri_v, int32_t* tri_nbr, int32_t* tri_prim,
                           const int32_t* vertex_line, int64_t n_prims, const int32_t* prim_v,
                           int32_t n_rounds, const double* temperature, uint64_t seed,
                           int64_t* flips_out, void* stream) {
  using ccsp::set_last_error;
  auto fail = [](int code, const char* msg) {
    set_last_error(msg);
    return code;
  };
  if (!xy || !tri_v || !tri_nbr || !tri_prim || n_vertices <= 0 || n_triangles <= 0 ||
      n_rounds < 0 || (n_rounds > 0 && (!temperature || !flips_out)))
    return fail(CCSP_E_ARG, "flip_anneal: null argument or empty triangulation");
  if (n_triangles >= (int64_t(1) << 29) || n_vertices >= (int64_t(1) << 31))
    return fail(CCSP_E_ARG, "flip_anneal: triangulation too large for 32-bit slots");
  if (n_rounds > (1 << 20)) return fail(CCSP_E_ARG, "flip_anneal: more than 2^20 rounds");
  if (vertex_line && (n_prims <= 0 || n_prims >= (int64_t(1) << 31) || !prim_v))
    return fail(CCSP_E_ARG, "flip_anneal: vertex_line needs the original edges' ends");
  if (((uintptr_t)vertex_line & 3) != 0 || ((uintptr_t)prim_v & 3) != 0)
    return fail(CCSP_E_ARG, "flip_anneal: misaligned buffer");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)tri_v & 3) != 0 || ((uintptr_t)tri_nbr & 3) != 0 ||
      ((uintptr_t)tri_prim & 3) != 0)
    return fail(CCSP_E_ARG, "flip_anneal: misaligned buffer");
  for (int32_t r = 0; r < n_rounds; ++r)
    if (!(temperature[r] >= 0) || !std::isfinite(temperature[r]))
      return fail(CCSP_E_ARG, "flip_anneal: temperatures must be finite and >= 0");
  if (n_rounds == 0) return CCSP_OK;
  const int64_t slots = 3 * n_triangles;
  const int64_t n_count = (int64_t)n_rounds * ccsp::kCountLanes;
  void* mem = nullptr;
  // per-round counters first (8-byte aligned), then key, best and keep
  const size_t bytes = 8 * (size_t)n_count + 4 * (size_t)slots + 4 * (size_t)n_triangles +
                       (size_t)slots;
  hipError_t e = hipMalloc(&mem, bytes);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "flip_anneal: device allocation failed");
  auto* count = (unsigned long long*)mem;
  auto* key = (int32_t*)(count + n_count);
  auto* best = key + slots;
  auto* keep = (uint8_t*)(best + n_triangles);
  hipStream_t s = (hipStream_t)stream;
  const ccsp::Tri T{tri_v,
                    tri_nbr,
                    tri_prim,
                    (int32_t)n_triangles,
                    (int32_t)n_vertices,
                    vertex_line,
                    vertex_line ? prim_v : nullptr,
                    vertex_line ? (int32_t)n_prims : 0};
  const unsigned blocks = (unsigned)((slots + ccsp::kFlipThreads - 1) / ccsp::kFlipThreads);
  const unsigned tblocks = (unsigned)((n_triangles + ccsp::kFlipThreads - 1) / ccsp::kFlipThreads);
  hipLaunchKernelGGL(ccsp::flip_clear, dim3(blocks), dim3(ccsp::kFlipThreads), 0, s, key, slots,
                     count, n_count);
  for (int32_t r = 0; r < n_rounds; ++r) {
    hipLaunchKernelGGL(ccsp::flip_eval, dim3(blocks), dim3(ccsp::kFlipThreads), 0, s, T,
                       (const double2*)xy, temperature[r], seed, r, key);
    hipLaunchKernelGGL(ccsp::flip_best, dim3(tblocks), dim3(ccsp::kFlipThreads), 0, s, T, key, seed,
                       r, best);
    hipLaunchKernelGGL(ccsp::flip_select, dim3(tblocks), dim3(ccsp::kFlipThreads), 0, s, T, key,
                       best, keep);
    hipLaunchKernelGGL(ccsp::flip_apply, dim3(tblocks), dim3(ccsp::kFlipThreads), 0, s, T, keep, key,
                       count + (int64_t)r * ccsp::kCountLanes);
  }
  int rc = CCSP_OK;
  std::vector<unsigned long long> lanes((size_t)n_count);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(lanes.data(), count, 8 * (size_t)n_count, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) rc = fail(CCSP_E_HIP, "flip_anneal: launch or copy failed");
  for (int32_t r = 0; r < n_rounds && rc == CCSP_OK; ++r) {
    unsigned long long n = 0;
    for (int l = 0; l < ccsp::kCountLanes; ++l) n += lanes[(size_t)r * ccsp::kCountLanes + l];
    flips_out[r] = (int64_t)n;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(mem);
  return rc;
}
