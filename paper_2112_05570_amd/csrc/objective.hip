// The low-weight objective with fuzzy contraction (paper Sec. 2.2) and its change under
// single-vertex moves (Sec. 3.2.1), on the GPU: mesh construction, kernels and the C-ABI of
// ccsp_objective.h.
//
// Evaluation is two passes over edges and triangles. The first computes every edge's length,
// contractibility and contraction weight c(e) (and the length penalty). The second forms each
// edge's weight from the c of its neighbouring edges, and the angle penalty of every triangle.
// Both write one partial sum per workgroup, reduced in a fixed order by a last one-workgroup
// kernel, so results are reproducible.
//
// A move changes only terms near its vertex v. With N(v) the neighbours of v, the edges whose c
// can change ("C-edges") are those incident to v (length) and those joining two vertices of N(v)
// (v may be an opposite vertex or a 1-hop vertex of such an edge), found by looking up each pair of
// neighbours, so that a neighbour with a long row (the apex of a fan) costs one binary search. The edges whose weight can
// change are the C-edges and the other edges of the triangles holding a C-edge. One thread per
// move visits each of these edges once, using the canonical choice of the triangle that reports
// it, and sums new minus old terms; the angle terms of the triangles of v and the length terms of
// its edges are added in the same way. Every term uses the same operations, in the same order, as
// the evaluation, so a move back gives exactly the opposite term differences.
//
// Compiled with -ffp-contract=off: every binary64 expression is evaluated as written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "ccsp_objective.h"
#include "exact.hpp"
#include "scan.hpp"
#include "walk.hpp"

struct MovableMesh;

namespace ccsp {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;  // workgroups of the evaluation passes: 8 waves per CU

struct MeshDev {
  int32_t nv, nt, ne, np;
  const int2* edge_v;     // (a, b), a < b
  const int4* edge_nbr;   // neighbouring edges in product order; -1 pads the last two
  const int2* edge_opp;   // opposite vertex in each triangle of the edge; -1 pad
  const int2* edge_tri;   // triangles of the edge, increasing; -1 pad
  const int4* tri;        // vertices (x, y, z)
  const int4* tri_edge;   // local edges (x, y, z): edge i is opposite vertex i
  const int32_t* adj_off; // neighbours of each vertex, increasing, with the joining edge
  const int2* adj;
  const int32_t* vtri_off;  // triangles of each vertex, increasing
  const int32_t* vtri;
  const int2* vk;         // (kind, line)
  const int2* prim_v;
  const int32_t* hop_off; // nontrivial 1-hop vertices of each edge (common neighbours of its ends
  const int32_t* hop_v;   // that are not opposite vertices): topology only, found at load
  const int32_t* vold;    // internal vertex -> caller's vertex
  const int32_t* vnew;    // caller's vertex -> internal vertex
  const int32_t* eperm;   // internal edge -> caller's edge numbering
  double2* xyi;           // scratch: positions in internal order
  double* c;              // scratch: contraction weight, length, contractibility per edge
  double* len;
  uint8_t* contr;
  // per edge: bit 0, the conditioning restriction holds (it reads only ORIGINAL positions and
  // the original edges of CONSTRAINED vertices, which no move changes); bit 1, the flat-triangle
  // restriction may apply (a topological test, see flat_candidate). Kept across calls: edge_state
  // recomputes them when *stale is set, which mesh_load does and permute_positions does when an
  // ORIGINAL position differs, bit for bit, from the previous call's
  uint8_t* rule;
  int32_t* stale;
  double* partial;
};

struct Par {
  double eps, delta, eps0, mu_angle, mu_len;
  int polish;
};

__device__ __forceinline__ double2 pos(const double2* __restrict__ xy, int u, int mv, double2 q) {
  return u == mv ? q : xy[u];
}

__device__ __forceinline__ double dist(double2 a, double2 b) {
  const double dx = b.x - a.x, dy = b.y - a.y;
  return sqrt(dx * dx + dy * dy);
}

__device__ __forceinline__ double c_of_len(bool contractible, double len, double eps) {
  return contractible ? 0.5 + 0.5 * fmin(1.0, len / eps) : 1.0;
}

__device__ __forceinline__ double merged_weight(double x) {
  const double m = x < 0.25 ? 0.0 : (x <= 0.5 ? 4.0 * x - 1.0 : 1.0);
  return x * m;
}

__device__ __forceinline__ double short_term(double len, double eps0) {
  return fmax(0.0, eps0 - len) / eps0;
}

__device__ double corner_term(double2 o, double2 u, double2 w, double delta, int polish) {
  const double ux = u.x - o.x, uy = u.y - o.y, wx = w.x - o.x, wy = w.y - o.y;
  const double lu = sqrt(ux * ux + uy * uy), lw = sqrt(wx * wx + wy * wy);
  const double den = lu * lw;
  if (!(den > 0.0)) return 0.0;
  const double cs = (ux * wx + uy * wy) / den;
  return polish ? fmax(0.0, cs - (1.0 - delta)) / delta : fmax(0.0, (-1.0 + delta) - cs) / delta;
}

__device__ double triangle_angles(const double2* __restrict__ xy, int4 t, int mv, double2 q,
                                  double delta, int polish) {
  const double2 a = pos(xy, t.x, mv, q), b = pos(xy, t.y, mv, q), c = pos(xy, t.z, mv, q);
  double s = corner_term(a, b, c, delta, polish);
  s += corner_term(b, c, a, delta, polish);
  s += corner_term(c, a, b, delta, polish);
  return s;
}

// Exact sign of the orientation of (a, b, c): binary64 filter, then the exact expansion.
__device__ __forceinline__ int orient_sign(double2 a, double2 b, double2 c) {
  const double l = (b.x - a.x) * (c.y - a.y);
  const double r = (b.y - a.y) * (c.x - a.x);
  const double det = l - r, sum = fabs(l) + fabs(r);
  if (fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return orient_exact(a.x, a.y, b.x, b.y, c.x, c.y);
}

__device__ bool is_neighbour(const MeshDev& m, int v, int x) {
  int lo = m.adj_off[v], hi = m.adj_off[v + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int y = m.adj[mid].x;
    if (y == x) return true;
    if (y < x) lo = mid + 1; else hi = mid;
  }
  return false;
}

// Id of the edge joining a and b, or -1: binary search in the shorter of the two rows.
__device__ __forceinline__ int find_edge(const MeshDev& m, int a, int b) {
  if (m.adj_off[a + 1] - m.adj_off[a] > m.adj_off[b + 1] - m.adj_off[b]) {
    const int t = a;
    a = b;
    b = t;
  }
  int lo = m.adj_off[a], hi = m.adj_off[a + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int2 y = m.adj[mid];
    if (y.x == b) return y.y;
    if (y.x < b) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// Restrictions of the original geometry (Sec. 2.2.2).
__device__ bool direct_ok(const MeshDev& m, int a, int b) {
  const int2 ka = m.vk[a], kb = m.vk[b];
  if (ka.x == CCSP_VERTEX_ORIGINAL && kb.x == CCSP_VERTEX_ORIGINAL) return false;
  if (ka.x == CCSP_VERTEX_ORIGINAL && kb.x == CCSP_VERTEX_CONSTRAINED) {
    const int2 e = m.prim_v[kb.y];
    return e.x == a || e.y == a;
  }
  if (kb.x == CCSP_VERTEX_ORIGINAL && ka.x == CCSP_VERTEX_CONSTRAINED) {
    const int2 e = m.prim_v[ka.y];
    return e.x == b || e.y == b;
  }
  if (ka.x == CCSP_VERTEX_CONSTRAINED && kb.x == CCSP_VERTEX_CONSTRAINED) return ka.y == kb.y;
  return true;
}

// 1-hop rule (Sec. 2.2.2), with vertex mv at q: every nontrivial 1-hop vertex of edge e lies
// strictly closer than eps to one of its opposite vertices.
__device__ bool one_hop_ok(const MeshDev& m, const double2* __restrict__ xy, int e, int2 opp,
                           double eps, int mv, double2 q) {
  for (int j = m.hop_off[e], end = m.hop_off[e + 1]; j < end; ++j) {
    const double2 px = pos(xy, m.hop_v[j], mv, q);
    bool close = dist(px, pos(xy, opp.x, mv, q)) < eps;
    if (!close && opp.y >= 0) close = dist(px, pos(xy, opp.y, mv, q)) < eps;
    if (!close) return false;
  }
  return true;
}

// Near-collinearity (Sec. 2.2.2): 16 * area / perimeter^2 below kCollinear (a zero perimeter
// counts as collinear). The paper compares the area with the square of equal perimeter against a
// small critical value it does not give; 0.01 is the ratio of a triangle whose corner between two
// equal sides is 179 degrees, where the angle penalty starts.
constexpr double kCollinear = 0.01;

__device__ bool near_collinear(double2 a, double2 b, double2 c) {
  const double cross = (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
  const double area = 0.5 * fabs(cross);
  const double per = (dist(a, b) + dist(b, c)) + dist(c, a);
  if (!(per > 0.0)) return true;
  return (16.0 * area) / (per * per) < kCollinear;
}

__device__ __forceinline__ bool on_line(const MeshDev& m, int v, int line) {
  const int2 k = m.vk[v];
  if (k.x == CCSP_VERTEX_CONSTRAINED) return k.y == line;
  if (k.x == CCSP_VERTEX_ORIGINAL) {
    const int2 e = m.prim_v[line];
    return e.x == v || e.y == v;
  }
  return false;
}

__device__ __forceinline__ int dof(int kind) {
  return kind == CCSP_VERTEX_ORIGINAL ? 0 : (kind == CCSP_VERTEX_CONSTRAINED ? 1 : 2);
}

// Conditioning (Sec. 2.2.2) of the triangle (t0, t1, t2), in that order: badly conditioned for
// good from the positions of ORIGINAL vertices and the original edges of CONSTRAINED ones (all
// fixed while optimising). A FREE vertex: never. Three ORIGINAL: near-collinear. Two ORIGINAL and
// a CONSTRAINED s: near-collinear with s at both ends of its original edge and at its middle.
// One ORIGINAL o and two CONSTRAINED: their original edges collinear with each other and with o.
// Three CONSTRAINED: their original edges collinear. Three vertices on one original edge are the
// flat-triangle case (flat_ok), not this one.
__device__ bool conditioning_bad(const MeshDev& m, const double2* __restrict__ xy, int t0, int t1,
                                 int t2) {
  const int tv[3] = {t0, t1, t2};
  int no = 0, nc = 0, orig[3], cons[3];
  for (int j = 0; j < 3; ++j) {
    const int k = m.vk[tv[j]].x;
    if (k == CCSP_VERTEX_FREE) return false;
    if (k == CCSP_VERTEX_ORIGINAL) orig[no++] = tv[j];
    else cons[nc++] = tv[j];
  }
  for (int j = 0; j < nc; ++j) {
    const int L = m.vk[cons[j]].y;
    if (on_line(m, t0, L) && on_line(m, t1, L) && on_line(m, t2, L)) return false;
  }
  if (no == 3) return near_collinear(xy[orig[0]], xy[orig[1]], xy[orig[2]]);
  const int2 e0 = m.prim_v[m.vk[cons[0]].y];
  const double2 a = xy[e0.x], b = xy[e0.y];
  if (no == 2) {
    const double2 mid = make_double2((a.x + b.x) * 0.5, (a.y + b.y) * 0.5);
    const double2 o1 = xy[orig[0]], o2 = xy[orig[1]];
    return near_collinear(o1, o2, a) && near_collinear(o1, o2, b) && near_collinear(o1, o2, mid);
  }
  bool lines = true;
  for (int j = 1; j < nc; ++j) {
    const int2 ej = m.prim_v[m.vk[cons[j]].y];
    lines = lines && near_collinear(a, b, xy[ej.x]) && near_collinear(a, b, xy[ej.y]);
  }
  if (no == 1) return lines && near_collinear(a, b, xy[orig[0]]);
  return lines;
}

// Conditioning restriction of edge (a, b): when contracting it snaps the vertex with more degrees
// of freedom onto the other, no triangle of that vertex without the other may become badly
// conditioned for good (the other taking its place).
__device__ bool conditioning_ok(const MeshDev& m, const double2* __restrict__ xy, int a, int b) {
  const int da = dof(m.vk[a].x), db = dof(m.vk[b].x);
  if (da == db) return true;
  const int hi = da > db ? a : b, lo = da > db ? b : a;
  for (int k = m.vtri_off[hi], end = m.vtri_off[hi + 1]; k < end; ++k) {
    const int4 t = m.tri[m.vtri[k]];
    if (t.x == lo || t.y == lo || t.z == lo) continue;
    if (conditioning_bad(m, xy, t.x == hi ? lo : t.x, t.y == hi ? lo : t.y, t.z == hi ? lo : t.z))
      return false;
  }
  return true;
}

// Flat-triangle restriction (Sec. 2.2.2), with vertex mv at q: for an edge joining a FREE vertex F
// and a CONSTRAINED or ORIGINAL vertex C, every CONSTRAINED vertex of a triangle (F, X, Y) without C
// whose X and Y lie on an original edge L through C (it becomes the zero-area (C, X, Y)) must
// already be contracted to C or to an ORIGINAL end of L: a path along L of edges shorter than eps
// through F's fan (F's neighbours on L, and C) reaches one of them. Along L a vertex has at most
// two neighbours, so the path is followed in each direction from the trapped vertex.
__device__ bool flat_ok(const MeshDev& m, const double2* __restrict__ xy, int a, int b, double eps,
                        int mv, double2 q) {
  const int ka = m.vk[a].x, kb = m.vk[b].x;
  int F, C;
  if (ka == CCSP_VERTEX_FREE && kb != CCSP_VERTEX_FREE) {
    F = a;
    C = b;
  } else if (kb == CCSP_VERTEX_FREE && ka != CCSP_VERTEX_FREE) {
    F = b;
    C = a;
  } else {
    return true;
  }
  const int deg = m.adj_off[F + 1] - m.adj_off[F];
  for (int k = m.vtri_off[F], end = m.vtri_off[F + 1]; k < end; ++k) {
    const int4 t = m.tri[m.vtri[k]];
    if (t.x == C || t.y == C || t.z == C) continue;
    const int X = t.x == F ? t.y : t.x;
    const int Y = t.z == F ? t.y : t.z;
    const bool cx = m.vk[X].x == CCSP_VERTEX_CONSTRAINED, cy = m.vk[Y].x == CCSP_VERTEX_CONSTRAINED;
    if (!cx && !cy) continue;
    const int L = m.vk[cx ? X : Y].y;
    if (!(on_line(m, X, L) && on_line(m, Y, L) && on_line(m, C, L))) continue;
    for (int j = 0; j < 2; ++j) {
      const int T = j == 0 ? X : Y;
      if (m.vk[T].x != CCSP_VERTEX_CONSTRAINED) continue;
      bool reached = false;
      // each neighbour of T along L in the fan, reached by a short edge, starts one direction
      for (int s0 = m.adj_off[T], s1 = m.adj_off[T + 1]; s0 < s1 && !reached; ++s0) {
        int prev = T, cur = m.adj[s0].x;
        for (int steps = 0; steps <= deg + 1; ++steps) {
          if (!on_line(m, cur, L) || !(cur == C || is_neighbour(m, F, cur)) ||
              !(dist(pos(xy, prev, mv, q), pos(xy, cur, mv, q)) < eps))
            break;
          if (cur == C || m.vk[cur].x == CCSP_VERTEX_ORIGINAL) {
            reached = true;
            break;
          }
          int next = -1;
          for (int r = m.adj_off[cur], re = m.adj_off[cur + 1]; r < re; ++r) {
            const int w = m.adj[r].x;
            if (w != prev && on_line(m, w, L) && (w == C || is_neighbour(m, F, w))) {
              next = w;
              break;
            }
          }
          if (next < 0) break;
          prev = cur;
          cur = next;
        }
      }
      if (!reached) return false;
    }
  }
  return true;
}

// Whether flat_ok can fail for edge (a, b) at all: it joins a FREE F and a non-FREE C, and a
// triangle of F without C has its other two vertices, one of them CONSTRAINED, on an original
// edge through C. Kinds and topology only.
__device__ bool flat_candidate(const MeshDev& m, int a, int b) {
  const int ka = m.vk[a].x, kb = m.vk[b].x;
  if ((ka == CCSP_VERTEX_FREE) == (kb == CCSP_VERTEX_FREE)) return false;
  const int F = ka == CCSP_VERTEX_FREE ? a : b, C = ka == CCSP_VERTEX_FREE ? b : a;
  for (int k = m.vtri_off[F], end = m.vtri_off[F + 1]; k < end; ++k) {
    const int4 t = m.tri[m.vtri[k]];
    if (t.x == C || t.y == C || t.z == C) continue;
    const int X = t.x == F ? t.y : t.x;
    const int Y = t.z == F ? t.y : t.z;
    const bool cx = m.vk[X].x == CCSP_VERTEX_CONSTRAINED, cy = m.vk[Y].x == CCSP_VERTEX_CONSTRAINED;
    if (!cx && !cy) continue;
    const int L = m.vk[cx ? X : Y].y;
    if (on_line(m, X, L) && on_line(m, Y, L) && on_line(m, C, L)) return true;
  }
  return false;
}

// The position-independent restrictions of edge (a, b) for edge_state's rule bits.
__device__ __forceinline__ uint8_t rule_bits(const MeshDev& m, const double2* __restrict__ xy,
                                             int a, int b) {
  return (uint8_t)((conditioning_ok(m, xy, a, b) ? 1 : 0) | (flat_candidate(m, a, b) ? 2 : 0));
}

// Contractibility of edge e = (a, b) (Sec. 2.2.2), with vertex mv at q, given its rule bits.
__device__ bool contractible_rules(const MeshDev& m, const double2* __restrict__ xy, int e, int a,
                                   int b, double eps, int mv, double2 q, uint8_t rule) {
  return direct_ok(m, a, b) && (rule & 1) && one_hop_ok(m, xy, e, m.edge_opp[e], eps, mv, q) &&
         (!(rule & 2) || flat_ok(m, xy, a, b, eps, mv, q));
}

// Contractibility of edge e = (a, b), with vertex mv at q, from the rule bits of the call's
// edge_state (valid for any movable vertex's position: no move changes what they read).
__device__ __forceinline__ bool contractible_at(const MeshDev& m, const double2* __restrict__ xy,
                                                int e, int a, int b, double eps, int mv,
                                                double2 q) {
  return contractible_rules(m, xy, e, a, b, eps, mv, q, m.rule[e]);
}

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Caller positions into the mesh's internal vertex order; an ORIGINAL position that differs from
// the one staged by the previous call marks the rule bits stale.
__global__ void __launch_bounds__(kThreads)
permute_positions(MeshDev m, const double2* __restrict__ xy) {
  bool moved = false;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < m.nv; i += gridDim.x * kThreads) {
    const double2 q = xy[m.vold[i]];
    if (m.vk[i].x == CCSP_VERTEX_ORIGINAL) {
      const double2 o = m.xyi[i];
      moved = moved || __double_as_longlong(o.x) != __double_as_longlong(q.x) ||
              __double_as_longlong(o.y) != __double_as_longlong(q.y);
    }
    m.xyi[i] = q;
  }
  if (moved) *m.stale = 1;
}

// After edge_state: the rule bits match the staged ORIGINAL positions.
__global__ void rules_fresh(MeshDev m) {
  if (threadIdx.x == 0) *m.stale = 0;
}

// Pass 1: length, contractibility and c of every edge; length-penalty partial sums. Each thread
// takes a fixed stride of edges, so the partial sums do not depend on timing.
__global__ void __launch_bounds__(kThreads)
edge_state(MeshDev m, Par p, double* __restrict__ part) {
  __shared__ double sh[kThreads];
  const double2* __restrict__ xy = m.xyi;
  const bool stale = *m.stale != 0;
  double s = 0.0;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < m.ne; e += gridDim.x * kThreads) {
    const int2 ab = m.edge_v[e];
    const double len = dist(xy[ab.x], xy[ab.y]);
    uint8_t rule;
    if (stale) {
      rule = rule_bits(m, xy, ab.x, ab.y);
      m.rule[e] = rule;
    } else {
      rule = m.rule[e];
    }
    const bool ok = contractible_rules(m, xy, e, ab.x, ab.y, p.eps, -1, make_double2(0, 0), rule);
    m.len[e] = len;
    m.contr[e] = ok ? 1 : 0;
    m.c[e] = c_of_len(ok, len, p.eps);
    s += short_term(len, p.eps0);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ __forceinline__ double weight_from(const double* __restrict__ c, int4 n) {
  double x = c[n.x] * c[n.y];
  if (n.z >= 0) {
    x = x * c[n.z];
    x = x * c[n.w];
  }
  return merged_weight(x);
}

// Pass 2: weighted edge lengths and triangle angle penalties, partial sums of each. Per-edge
// outputs go to the caller's edge numbering.
__global__ void __launch_bounds__(kThreads)
terms_pass(MeshDev m, Par p, double* __restrict__ part_edge, double* __restrict__ part_angle,
           uint8_t* __restrict__ contr_out, double* __restrict__ w_out) {
  __shared__ double sh[kThreads];
  const int n = m.ne > m.nt ? m.ne : m.nt;
  double se = 0.0, sa = 0.0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    if (i < m.ne) {
      const double w = p.polish ? 1.0 : weight_from(m.c, m.edge_nbr[i]);
      se += w * m.len[i];
      if (w_out) w_out[m.eperm[i]] = w;
      if (contr_out) contr_out[m.eperm[i]] = m.contr[i];
    }
    if (i < m.nt)
      sa += triangle_angles(m.xyi, m.tri[i], -1, make_double2(0, 0), p.delta, p.polish);
  }
  se = block_sum(se, sh);
  sa = block_sum(sa, sh);
  if (threadIdx.x == 0) {
    part_edge[blockIdx.x] = se;
    part_angle[blockIdx.x] = sa;
  }
}

__device__ double sum_fixed(const double* __restrict__ v, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += v[i];
  return block_sum(s, sh);
}

__global__ void __launch_bounds__(kThreads)
finish_sums(const double* __restrict__ part, int n1, int n2, Par p, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const double pl = sum_fixed(part, n1, sh);
  const double wc = sum_fixed(part + n1, n2, sh);
  const double pa = sum_fixed(part + n1 + n2, n2, sh);
  if (threadIdx.x == 0) {
    out[0] = wc + p.mu_angle * pa + p.mu_len * pl;
    out[1] = wc;
    out[2] = pa;
    out[3] = pl;
  }
}

// ---- moves ----

constexpr int kLdsNbrs = 16;  // neighbours of a moved vertex kept in LDS (Steiner vertices have ~6)
constexpr int kCache = 8;     // entries of a move's cache of changed contraction weights

// The 32-bit finaliser of MurmurHash3 (Appleby): a bijection of the 32-bit integers that leaves no
// order between neighbouring values.
__device__ __forceinline__ uint32_t group_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// A thread's LDS columns for evaluating a move (stride kThreads): the moved vertex's neighbours,
// and a direct-mapped cache, by edge id, of the contraction weight c an edge takes after the move
// (each is read by up to four terms; computing it once per move keeps the neighbourhood gathers
// of its contractibility from repeating).
struct MoveLds {
  int* nb;
  int* ce;
  double* cc;
};

constexpr int kHash = 256;  // a wave's table of one move's C-edges (edge id -> slot)

// The context of one move's change of f. S is the stride of the LDS columns (a thread's own
// columns in a workgroup of kThreads, or 1 for a wave's shared ones). Without WAVE, the changed c
// of a C-edge is computed on first use into the thread's cache; with WAVE, the wave has computed
// every C-edge's changed c beforehand into its slot (hc), found through an open-addressing table
// (hkey, hslot).
template <int S, bool WAVE>
struct MoveCtxT {
  const MeshDev& m;
  const double2* __restrict__ xy;
  Par p;
  int v;
  double2 q;
  const int* nb;  // neighbours of v in LDS, stride S, when deg <= kLdsNbrs
  int deg;
  int* ce;        // the move's cache of changed c: edge ids (-1 empty) and values
  double* cc;
  const int* hkey;      // WAVE: table keys (-1 empty), their slots, and the slots' c
  const uint16_t* hslot;
  const double* hc;

  __device__ __forceinline__ bool adjacent(int x) const {
    if (deg > kLdsNbrs) return is_neighbour(m, v, x);
    for (int j = 0; j < deg; ++j)
      if (nb[j * S] == x) return true;
    return false;
  }
  // The edges whose c may change when v moves: v's edges (lengths; the flat-triangle rule of
  // an edge at v reads lengths at v), edges joining two neighbours of v (1-hop rule), and edges
  // joining a FREE neighbour of v to a vertex that is not FREE (the flat-triangle rule reads the
  // lengths of the edges among that neighbour's neighbours, v's among them).
  __device__ __forceinline__ bool in_c(int e) const {
    const int2 ab = m.edge_v[e];
    if (ab.x == v || ab.y == v) return true;
    const bool na = adjacent(ab.x), nb2 = adjacent(ab.y);
    if (na && nb2) return true;
    const bool fa = m.vk[ab.x].x == CCSP_VERTEX_FREE, fb = m.vk[ab.y].x == CCSP_VERTEX_FREE;
    return (fa && na && !fb) || (fb && nb2 && !fa);
  }
  __device__ __forceinline__ double len(int e, bool moved) const {
    const int2 ab = m.edge_v[e];
    if (!moved || (ab.x != v && ab.y != v)) return m.len[e];
    return dist(pos(xy, ab.x, v, q), pos(xy, ab.y, v, q));
  }
  __device__ __forceinline__ double c(int e, bool moved) const {
    if (!moved || !in_c(e)) return m.c[e];
    if constexpr (WAVE) {
      int h = (int)(group_hash((uint32_t)e) & (kHash - 1));
      for (int k = 0; k < kHash; ++k, h = (h + 1) & (kHash - 1))
        if (hkey[h] == e) return hc[hslot[h]];
      return __builtin_nan("");  // not reached: the table holds every C-edge
    } else {
      const int slot = (e & (kCache - 1)) * S;
      if (ce[slot] == e) return cc[slot];
      const int2 ab = m.edge_v[e];
      const double r =
          c_of_len(contractible_at(m, xy, e, ab.x, ab.y, p.eps, v, q), len(e, true), p.eps);
      ce[slot] = e;
      cc[slot] = r;
      return r;
    }
  }
  __device__ __forceinline__ double term(int e, bool moved) const {
    double w = 1.0;
    if (!p.polish) {
      const int4 n = m.edge_nbr[e];
      double x = c(n.x, moved) * c(n.y, moved);
      if (n.z >= 0) {
        x = x * c(n.z, moved);
        x = x * c(n.w, moved);
      }
      w = merged_weight(x);
    }
    return w * len(e, moved);
  }
  __device__ __forceinline__ double diff(int e) const { return term(e, true) - term(e, false); }
  __device__ __forceinline__ bool tri_has_c(int t) const {
    const int4 te = m.tri_edge[t];
    return in_c(te.x) || in_c(te.y) || in_c(te.z);
  }
  __device__ __forceinline__ int first_c(int t) const {
    const int4 te = m.tri_edge[t];
    return in_c(te.x) ? te.x : (in_c(te.y) ? te.y : te.z);
  }
  // The C-edge ec itself, then (once per triangle, from that triangle's first C-edge) the other
  // edges of its triangles that are not C-edges, each from the lowest-id triangle reaching it.
  __device__ __forceinline__ double visit(int ec) const {
    double s = diff(ec);
    const int2 tt = m.edge_tri[ec];
    for (int j = 0; j < 2; ++j) {
      const int t = j == 0 ? tt.x : tt.y;
      if (t < 0 || first_c(t) != ec) continue;
      const int4 te = m.tri_edge[t];
      for (int k = 0; k < 3; ++k) {
        const int e2 = k == 0 ? te.x : (k == 1 ? te.y : te.z);
        if (e2 == ec || in_c(e2)) continue;
        const int2 t2 = m.edge_tri[e2];
        const int tmin = tri_has_c(t2.x) ? t2.x : t2.y;
        if (tmin == t) s += diff(e2);
      }
    }
    return s;
  }
};

// Change of f (through *df) of moving internal vertex v to q, against positions xy (internal
// order) and the per-edge scratch of edge_state; with CHECK, CCSP_MOVE_FOLDS (and *df untouched)
// when a triangle of v would not stay strictly counter-clockwise. lds holds this thread's LDS
// columns.
template <bool CHECK, int S = kThreads>
__device__ __forceinline__ int move_change(const MeshDev& m, const double2* __restrict__ xy,
                                           const Par& p, int v, double2 q, MoveLds lds,
                                           double* df) {
  double sa = 0.0;
  for (int j = m.vtri_off[v], end = m.vtri_off[v + 1]; j < end; ++j) {
    const int4 t = m.tri[m.vtri[j]];
    if (CHECK &&
        orient_sign(pos(xy, t.x, v, q), pos(xy, t.y, v, q), pos(xy, t.z, v, q)) <= 0)
      return CCSP_MOVE_FOLDS;
    sa += triangle_angles(xy, t, v, q, p.delta, p.polish) -
          triangle_angles(xy, t, -1, q, p.delta, p.polish);
  }
  const int a0 = m.adj_off[v], deg = m.adj_off[v + 1] - a0;
  if (deg <= kLdsNbrs)
    for (int j = 0; j < deg; ++j) lds.nb[j * S] = m.adj[a0 + j].x;
#pragma unroll
  for (int k = 0; k < kCache; ++k) lds.ce[k * S] = -1;
  const MoveCtxT<S, false> ctx{m,      xy,     p,      v,      q,      lds.nb,
                               deg,    lds.ce, lds.cc, nullptr, nullptr, nullptr};
  double se = 0.0, ss = 0.0;
  for (int j = a0, end = a0 + deg; j < end; ++j) {
    const int e = m.adj[j].y;
    se += ctx.visit(e);
    ss += short_term(ctx.len(e, true), p.eps0) - short_term(m.len[e], p.eps0);
  }
  // edges joining two neighbours of v: pairs of its (increasing) neighbour row
  for (int j = a0, end = a0 + deg; j < end; ++j)
    for (int l = j + 1; l < end; ++l) {
      const int e = find_edge(m, m.adj[j].x, m.adj[l].x);
      if (e >= 0) se += ctx.visit(e);
    }
  // edges from a FREE neighbour F of v to a vertex that is not FREE and not v or a neighbour of
  // v (each once, from its FREE end)
  for (int j = a0, end = a0 + deg; j < end; ++j) {
    const int F = m.adj[j].x;
    if (m.vk[F].x != CCSP_VERTEX_FREE) continue;
    for (int k = m.adj_off[F], ke = m.adj_off[F + 1]; k < ke; ++k) {
      const int C = m.adj[k].x;
      if (C == v || m.vk[C].x == CCSP_VERTEX_FREE || ctx.adjacent(C)) continue;
      se += ctx.visit(m.adj[k].y);
    }
  }
  *df = se + p.mu_angle * sa + p.mu_len * ss;
  return CCSP_MOVE_OK;
}

// Status and change of f (through *df, +inf unless valid) of moving the vertex of caller id cv
// to q, against positions xy (internal order) and the per-edge scratch of edge_state. lds holds
// this thread's LDS columns.
__device__ __forceinline__ int evaluate_move(const MeshDev& m, const double2* __restrict__ xy,
                                             const Par& p, int cv, double2 q, MoveLds lds,
                                             double* df) {
  *df = __builtin_huge_val();
  if (cv < 0 || cv >= m.nv || !isfinite(q.x) || !isfinite(q.y)) return CCSP_MOVE_BAD;
  const int v = m.vnew[cv];
  if (m.vk[v].x == CCSP_VERTEX_ORIGINAL) return CCSP_MOVE_FIXED;
  return move_change<true>(m, xy, p, v, q, lds, df);
}

// Sort keys of a batch of moves: the moved vertex's internal id (nv for an id out of range), so
// that evaluating the moves in key order lets neighbouring threads share the cache lines of
// their neighbourhoods (internal ids follow a breadth-first order of the mesh).
__global__ void __launch_bounds__(kThreads)
move_keys(MeshDev m, const int32_t* __restrict__ vid, int64_t k, uint32_t* __restrict__ key,
          uint32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k) return;
  const int cv = vid[i];
  key[i] = (cv >= 0 && cv < m.nv) ? (uint32_t)m.vnew[cv] : (uint32_t)m.nv;
  idx[i] = (uint32_t)i;
}

// objective_delta's moves; order (NULL: the identity) lists the move each thread evaluates.
__global__ void __launch_bounds__(kThreads)
move_delta(MeshDev m, Par p, const int32_t* __restrict__ vid, const double2* __restrict__ qv,
           int64_t k, const uint32_t* __restrict__ order, double* __restrict__ delta,
           int32_t* __restrict__ status) {
  __shared__ int snb[kLdsNbrs * kThreads];
  __shared__ int sce[kCache * kThreads];
  __shared__ double scc[kCache * kThreads];
  const MoveLds lds{snb + threadIdx.x, sce + threadIdx.x, scc + threadIdx.x};
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= k) return;
  const int64_t i = order ? (int64_t)order[t] : t;
  double df;
  status[i] = evaluate_move(m, m.xyi, p, vid[i], qv[i], lds, &df);
  delta[i] = df;
}

// Metropolis moves (Sec. 3.1): vertex vid[i] displaced by disp[i] (projected on its original edge
// when constrained), accepted when valid and delta <= 0 or u[i] < exp(-delta / temperature);
// accepted positions are written to the caller's xy. Every move is evaluated against the
// positions before the call (xyi).
__global__ void __launch_bounds__(kThreads)
anneal_moves(MeshDev m, Par p, double temperature, double2* __restrict__ xy_out,
             const int32_t* __restrict__ vid, const double2* __restrict__ disp,
             const double* __restrict__ u, int64_t k, double* __restrict__ delta,
             int32_t* __restrict__ status) {
  __shared__ int snb[kLdsNbrs * kThreads];
  __shared__ int sce[kCache * kThreads];
  __shared__ double scc[kCache * kThreads];
  const MoveLds lds{snb + threadIdx.x, sce + threadIdx.x, scc + threadIdx.x};
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k) return;
  const int cv = vid[i];
  double2 q = make_double2(__builtin_nan(""), 0.0);
  if (cv >= 0 && cv < m.nv) {
    const int v = m.vnew[cv];
    const double2 o = m.xyi[v];
    double2 d = disp[i];
    const int2 kl = m.vk[v];
    if (kl.x == CCSP_VERTEX_CONSTRAINED) {
      const int2 ends = m.prim_v[kl.y];
      const double2 a = m.xyi[ends.x], b = m.xyi[ends.y];
      const double ex = b.x - a.x, ey = b.y - a.y;
      const double s = (d.x * ex + d.y * ey) / (ex * ex + ey * ey);
      d = make_double2(s * ex, s * ey);
    }
    q = make_double2(o.x + d.x, o.y + d.y);
  }
  double df;
  int st = evaluate_move(m, m.xyi, p, cv, q, lds, &df);
  if (st == CCSP_MOVE_OK) {
    if (df <= 0.0 || u[i] < exp(-df / temperature))
      xy_out[cv] = q;
    else
      st = CCSP_MOVE_REJECTED;
  }
  status[i] = st;
  delta[i] = df;
}

// After an accepted move of internal vertex v (already at its new position in m.xyi): recompute
// the scratch of the edges whose values depend on v's position, with the operations of
// edge_state: length and c of its edges, contractibility and c of the edges joining two of its
// neighbours (v may be an opposite or 1-hop vertex of those).
// Split in two (lengths, then the rest) for callers that refresh several vertices at once.
__device__ __forceinline__ void refresh_lengths(const MeshDev& m, int v) {
  const double2* __restrict__ xy = m.xyi;
  for (int j = m.adj_off[v], a1 = m.adj_off[v + 1]; j < a1; ++j) {
    const int e = m.adj[j].y;
    const int2 ab = m.edge_v[e];
    m.len[e] = dist(xy[ab.x], xy[ab.y]);
  }
}

__device__ __forceinline__ void refresh_rules(const MeshDev& m, const Par& p, int v) {
  const double2* __restrict__ xy = m.xyi;
  const int a0 = m.adj_off[v], a1 = m.adj_off[v + 1];
  const double2 nq = make_double2(0, 0);
  for (int j = a0; j < a1; ++j) {
    const int e = m.adj[j].y;
    const int2 ab = m.edge_v[e];
    const bool ok = contractible_at(m, xy, e, ab.x, ab.y, p.eps, -1, nq);
    m.contr[e] = ok ? 1 : 0;
    m.c[e] = c_of_len(ok, m.len[e], p.eps);
  }
  for (int j = a0; j < a1; ++j)
    for (int l = j + 1; l < a1; ++l) {
      const int a = m.adj[j].x, b = m.adj[l].x;
      const int e = find_edge(m, a, b);
      if (e < 0) continue;
      const bool ok = contractible_at(m, xy, e, a, b, p.eps, -1, nq);
      m.contr[e] = ok ? 1 : 0;
      m.c[e] = c_of_len(ok, m.len[e], p.eps);
    }
  for (int j = a0; j < a1; ++j) {
    const int F = m.adj[j].x;
    if (m.vk[F].x != CCSP_VERTEX_FREE) continue;
    for (int k = m.adj_off[F], ke = m.adj_off[F + 1]; k < ke; ++k) {
      const int C = m.adj[k].x;
      if (C == v || m.vk[C].x == CCSP_VERTEX_FREE || is_neighbour(m, v, C)) continue;
      const int e = m.adj[k].y;
      const bool ok = contractible_at(m, xy, e, F, C, p.eps, -1, nq);
      m.contr[e] = ok ? 1 : 0;
      m.c[e] = c_of_len(ok, m.len[e], p.eps);
    }
  }
}

__device__ __forceinline__ void refresh_scratch(const MeshDev& m, const Par& p, int v) {
  refresh_lengths(m, v);  // first: the c below read the lengths
  refresh_rules(m, p, v);
}

// Area of triangle t at the current positions, its vertices in the caller's order.
__device__ __forceinline__ double tri_area(const MeshDev& m, int t) {
  const int4 tr = m.tri[t];
  const double2 a = m.xyi[tr.x], b = m.xyi[tr.y], c = m.xyi[tr.z];
  return 0.5 * ((b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x));
}

// A position uniform by area over the triangles of internal vertex v (Sec. 3.2.4): the first
// triangle (caller order) at which the running sum of areas exceeds r0 times their total, and in
// it (1 - s) a + s (1 - r2) b + s r2 c, s = sqrt(r1), the sampling of Osada et al. (2002).
__device__ __forceinline__ double2 resample_star(const MeshDev& m, int v, double r0, double r1,
                                                 double r2) {
  const int j0 = m.vtri_off[v], j1 = m.vtri_off[v + 1];
  double total = 0.0;
  for (int j = j0; j < j1; ++j) total = total + tri_area(m, m.vtri[j]);
  const double target = r0 * total;
  double run = 0.0;
  int pick = m.vtri[j1 - 1];
  for (int j = j0; j < j1; ++j) {
    run = run + tri_area(m, m.vtri[j]);
    if (target < run) {
      pick = m.vtri[j];
      break;
    }
  }
  const int4 tr = m.tri[pick];
  const double2 a = m.xyi[tr.x], b = m.xyi[tr.y], c = m.xyi[tr.z];
  const double s = sqrt(r1);
  const double ka = 1.0 - s, kb = s * (1.0 - r2), kc = s * r2;
  return make_double2(ka * a.x + kb * b.x + kc * c.x, ka * a.y + kb * b.y + kc * c.y);
}

// Whether internal vertex v has an edge shorter than l: at its current position (the edges'
// current lengths), or with v at q.
__device__ __forceinline__ bool has_short_edge(const MeshDev& m, int v, double l) {
  for (int j = m.adj_off[v], end = m.adj_off[v + 1]; j < end; ++j)
    if (m.len[m.adj[j].y] < l) return true;
  return false;
}
__device__ __forceinline__ bool has_short_edge_at(const MeshDev& m, int v, double2 q, double l) {
  for (int j = m.adj_off[v], end = m.adj_off[v + 1]; j < end; ++j)
    if (dist(q, m.xyi[m.adj[j].x]) < l) return true;
  return false;
}

// The neighbour of internal vertex v whose caller id has rank k among its neighbours' caller ids.
__device__ __forceinline__ int neighbour_of_rank(const MeshDev& m, int v, int k) {
  const int a0 = m.adj_off[v], a1 = m.adj_off[v + 1];
  for (int j = a0; j < a1; ++j) {
    const int w = m.adj[j].x, cw = m.vold[w];
    int below = 0;
    for (int l = a0; l < a1; ++l) below += m.vold[m.adj[l].x] < cw ? 1 : 0;
    if (below == k) return w;
  }
  return m.adj[a1 - 1].x;  // not reached: caller ids are distinct
}

// The proposal of class member i (vertex v) of a sweep: its new position *q, or *skip when
// the proposal does not apply to it (Secs. 3.2.2, 3.2.4-3.2.6, as documented for anneal_sweep and
// anneal_propose).
__device__ __forceinline__ void propose_move(const MeshDev& m, const Par& p, double lambda,
                                             int kind, int v, int i,
                                             const double2* __restrict__ disp, double2* q_out,
                                             bool* skip_out) {
  const double2 o = m.xyi[v];
  bool skip = false;
  double2 d;
  if (kind == CCSP_PROPOSE_DISPLACE) {
    d = disp[i];
    if (lambda > 0.0) {
      // disp is a unit draw: scale by lambda * eta, eta the square root of the area of v's
      // triangles (Sec. 3.2.2), summed in the caller's triangle order at the current positions
      double area = 0.0;
      for (int j = m.vtri_off[v], end = m.vtri_off[v + 1]; j < end; ++j)
        area += tri_area(m, m.vtri[j]);
      const double k = lambda * sqrt(area);
      d = make_double2(k * d.x, k * d.y);
    }
  } else {
    const double2 ra = disp[2 * i], rb = disp[2 * i + 1];
    double2 target = o;
    if (kind == CCSP_PROPOSE_SWAP) {
      // Sec. 3.2.5: l uniform on [0.2 eps, 2 eps); only a vertex with an edge shorter than l
      const double l = (0.2 + 1.8 * ra.x) * p.eps;
      if (has_short_edge(m, v, l)) {
        const int deg = m.adj_off[v + 1] - m.adj_off[v];
        const int w = neighbour_of_rank(m, v, min((int)(ra.y * (double)deg), deg - 1));
        const double2 pw = m.xyi[w];
        target = make_double2(pw.x + l * rb.x, pw.y + l * rb.y);
      } else {
        skip = true;
      }
    } else {
      target = resample_star(m, v, ra.x, ra.y, rb.x);
    }
    d = make_double2(target.x - o.x, target.y - o.y);
  }
  const int2 kl = m.vk[v];
  if (kl.x == CCSP_VERTEX_CONSTRAINED) {
    const int2 ends = m.prim_v[kl.y];
    const double2 a = m.xyi[ends.x], b = m.xyi[ends.y];
    const double ex = b.x - a.x, ey = b.y - a.y;
    const double s = (d.x * ex + d.y * ey) / (ex * ex + ey * ey);
    d = make_double2(s * ex, s * ey);
  }
  const double2 q = make_double2(o.x + d.x, o.y + d.y);
  // Sec. 3.2.6: only a change of the contracted state is tried, once
  if (kind == CCSP_PROPOSE_CONTRACT &&
      has_short_edge(m, v, p.eps) == has_short_edge_at(m, v, q, p.eps))
    skip = true;
  *q_out = q;
  *skip_out = skip;
}

// ---- group moves (Sec. 3.2.3)
//
// The group of centre c is every movable vertex within distance d of it (a range query on a
// uniform grid of the current positions, as the paper does), with no limit on its size. A sweep
// runs in rounds. In a round every pending group finds its members and claims, by the lowest
// priority (atomicMin; a group's priority is its centre index scrambled by a bijection, so that
// groups whose indices run along a chain in space do not move one per round): the vertices within
// two edges of its members (along paths that avoid hubs, see is_hub), and the grid cells of its
// query disc and of its members' positions before and after the move. A group moves when it
// holds its cells and no vertex within three edges of its members carries a lower priority; the
// others wait for the next round. The pending group of lowest priority always moves. Two groups
// that move in one round have members more than five edges apart: otherwise a vertex on a
// shortest path between them lies within two edges of one and three of the other, and another
// within three of the first and two of the second, so each would see the other's priority as
// lower. A move writes positions and edge scratch within one edge of its members and reads within
// four, and neither group moves a vertex into or out of the other's disc: the two commute, and the
// sweep equals the sequential chain over the centres in the order (round, index).

constexpr double kQueryWiden = 1.0 + 0x1p-40;  // query extents, widened against rounding

// A group's claim priority: its index through the 32-bit finaliser of MurmurHash3, so that
// neighbouring indices carry unrelated priorities.
__device__ __forceinline__ uint32_t group_priority(int i) { return group_hash((uint32_t)i); }

struct VGrid {
  double x0, y0, inv;      // cell of p: floor((p - p0) * inv), clamped to the grid
  int gx, gy;
  const int32_t* start;    // gx * gy + 1 offsets into vert
  const int32_t* vert;     // internal vertex ids, cell by cell
};

// Clamped (so that a range stays a superset of the cells of the points in it) and monotone.
__device__ __forceinline__ int clamp_cell(double f, int g) {
  if (!(f > 0.0)) return 0;
  if (f >= (double)(g - 1)) return g - 1;
  return (int)f;
}

__device__ __forceinline__ int cell_of(const VGrid& g, double2 q) {
  return clamp_cell((q.y - g.y0) * g.inv, g.gy) * g.gx + clamp_cell((q.x - g.x0) * g.inv, g.gx);
}

// f(cell) for every cell meeting the square of half-side r around q.
template <class F>
__device__ __forceinline__ void for_cells(const VGrid& g, double2 q, double r, F&& f) {
  const int x0 = clamp_cell((q.x - r - g.x0) * g.inv, g.gx);
  const int x1 = clamp_cell((q.x + r - g.x0) * g.inv, g.gx);
  const int y0 = clamp_cell((q.y - r - g.y0) * g.inv, g.gy);
  const int y1 = clamp_cell((q.y + r - g.y0) * g.inv, g.gy);
  for (int cy = y0; cy <= y1; ++cy)
    for (int cx = x0; cx <= x1; ++cx) f(cy * g.gx + cx);
}

// f(cell) for every cell meeting the square of half-side r around q, spread over a wave's lanes.
template <class F>
__device__ __forceinline__ void for_cells_lanes(const VGrid& g, double2 q, double r, int lane,
                                                F&& f) {
  const int x0 = clamp_cell((q.x - r - g.x0) * g.inv, g.gx);
  const int x1 = clamp_cell((q.x + r - g.x0) * g.inv, g.gx);
  const int y0 = clamp_cell((q.y - r - g.y0) * g.inv, g.gy);
  const int y1 = clamp_cell((q.y + r - g.y0) * g.inv, g.gy);
  const int w = x1 - x0 + 1, count = w * (y1 - y0 + 1);
  for (int k = lane; k < count; k += 64) f((y0 + k / w) * g.gx + x0 + k % w);
}

// f(w) for every movable vertex w != c with dist(p_c, p_w) <= d (the distance as for edges).
template <class F>
__device__ __forceinline__ void for_members(const MeshDev& m, const VGrid& g, int c, double d,
                                            F&& f) {
  const double2 pc = m.xyi[c];
  for_cells(g, pc, d * kQueryWiden, [&](int cell) {
    for (int k = g.start[cell], end = g.start[cell + 1]; k < end; ++k) {
      const int w = g.vert[k];
      if (w != c && m.vk[w].x != CCSP_VERTEX_ORIGINAL && dist(pc, m.xyi[w]) <= d) f(w);
    }
  });
}

// A hub: an ORIGINAL vertex with more than kHubDegree neighbours, such as a box corner whose fan
// reaches hundreds of vertices. Its position never changes, and what a move reads or writes at a
// hub's edges (their lengths and contraction states, the terms of the edges beside them) lies at
// the moved vertex's own place in the fan, within two fan steps, which the fan's ring edges also
// join. Claims therefore neither hold hubs nor pass through them: otherwise every group near a
// corner would claim the corner's whole fan, and those groups would move one per round.
constexpr int kHubDegree = 32;

__device__ __forceinline__ bool is_hub(const MeshDev& m, int x) {
  return m.adj_off[x + 1] - m.adj_off[x] > kHubDegree && m.vk[x].x == CCSP_VERTEX_ORIGINAL;
}

// f(x) for every vertex within two edges of the movable vertex v along paths that avoid hubs
// (with repeats).
template <class F>
__device__ __forceinline__ void for_hops2(const MeshDev& m, int v, F&& f) {
  f(v);
  for (int a = m.adj_off[v], ae = m.adj_off[v + 1]; a < ae; ++a) {
    const int w = m.adj[a].x;
    if (is_hub(m, w)) continue;
    f(w);
    for (int b = m.adj_off[w], be = m.adj_off[w + 1]; b < be; ++b) {
      const int x = m.adj[b].x;
      if (!is_hub(m, x)) f(x);
    }
  }
}

// f(x) for every vertex within three edges of the movable vertex v along paths that avoid hubs
// (with repeats).
template <class F>
__device__ __forceinline__ void for_hops3(const MeshDev& m, int v, F&& f) {
  f(v);
  for (int a = m.adj_off[v], ae = m.adj_off[v + 1]; a < ae; ++a) {
    const int w = m.adj[a].x;
    if (is_hub(m, w)) continue;
    f(w);
    for (int b = m.adj_off[w], be = m.adj_off[w + 1]; b < be; ++b) {
      const int x = m.adj[b].x;
      if (is_hub(m, x)) continue;
      f(x);
      for (int e = m.adj_off[x], ee = m.adj_off[x + 1]; e < ee; ++e) {
        const int y = m.adj[e].x;
        if (!is_hub(m, y)) f(y);
      }
    }
  }
}

// The displacement D projected for a CONSTRAINED vertex v (as for single-vertex moves).
__device__ __forceinline__ double2 member_disp(const MeshDev& m, int v, double2 D) {
  const int2 kl = m.vk[v];
  if (kl.x != CCSP_VERTEX_CONSTRAINED) return D;
  const int2 ends = m.prim_v[kl.y];
  const double2 a = m.xyi[ends.x], b = m.xyi[ends.y];
  const double ex = b.x - a.x, ey = b.y - a.y;
  const double s = (D.x * ex + D.y * ey) / (ex * ex + ey * ey);
  return make_double2(s * ex, s * ey);
}

__global__ void __launch_bounds__(kThreads)
vgrid_count(MeshDev m, VGrid g, int32_t* __restrict__ cnt) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v < m.nv) atomicAdd(&cnt[cell_of(g, m.xyi[v])], 1);
}

__global__ void __launch_bounds__(kThreads)
vgrid_fill(MeshDev m, VGrid g, int32_t* __restrict__ cursor, int32_t* __restrict__ vert) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= m.nv) return;
  const int cell = cell_of(g, m.xyi[v]);
  vert[g.start[cell] + atomicAdd(&cursor[cell], 1)] = v;
}

// Centres by caller id to internal ids; a centre that is not a movable vertex is done at once
// (status CCSP_MOVE_BAD or CCSP_MOVE_FIXED, round -1).
__global__ void __launch_bounds__(kThreads)
group_setup(MeshDev m, const int32_t* __restrict__ centres, int n, int32_t* __restrict__ gcen,
            uint8_t* __restrict__ done, double* __restrict__ delta, int32_t* __restrict__ status,
            int32_t* __restrict__ members, int32_t* __restrict__ round) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int cv = centres[i];
  const bool bad = cv < 0 || cv >= m.nv;
  const bool fixed = !bad && m.vk[m.vnew[cv]].x == CCSP_VERTEX_ORIGINAL;
  gcen[i] = bad || fixed ? -1 : m.vnew[cv];
  done[i] = bad || fixed ? 1 : 0;
  if (bad || fixed) {
    status[i] = bad ? CCSP_MOVE_BAD : CCSP_MOVE_FIXED;
    delta[i] = __builtin_huge_val();
    members[i] = 0;
    round[i] = -1;
  }
}

__global__ void __launch_bounds__(kThreads)
group_count(MeshDev m, VGrid g, Par p, const int32_t* __restrict__ gcen,
            const double2* __restrict__ draws, const uint8_t* __restrict__ done, int n,
            int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int k = 0;
  if (!done[i]) {
    const double d = (0.5 + 4.5 * draws[2 * i + 1].x) * p.eps;
    k = 1;
    for_members(m, g, gcen[i], d, [&](int) { ++k; });
  }
  cnt[i] = k;
}

// Position of vertex w in group (M, K, nm): 0 for the centre M[0], else its index in the members
// M[1..nm) ordered by caller id K, or -1 when w is not a member.
__device__ __forceinline__ int member_pos(const MeshDev& m, const int* __restrict__ M,
                                          const int* __restrict__ K, int nm, int w) {
  if (w == M[0]) return 0;
  const int kw = m.vold[w];
  int lo = 1, hi = nm;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int km = K[mid];
    if (km == kw) return mid;
    if (km < kw) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// One wave per group (4 per workgroup). Members (the centre, then the others by increasing caller
// id) into mem[off[i]..] with their caller ids in key[off[i]..], the move's displacement, and the
// claims. Lane 0 collects the members of the range query; the lanes rank them by caller id
// (distinct, so the order is unique), mark for each member which of its triangles hold no earlier
// member, and make the claims; lane 0 adds the group's area in member order (the same sum as one
// thread taking the members one after another).
__global__ void __launch_bounds__(kThreads)
group_claim(MeshDev m, VGrid g, VGrid gc, Par p, double lambda,
            const int32_t* __restrict__ gcen,
            const double2* __restrict__ draws, const uint8_t* __restrict__ done, int n,
            const int32_t* __restrict__ off, const int32_t* __restrict__ cnt,
            int32_t* __restrict__ mem, int32_t* __restrict__ key, int32_t* __restrict__ tmpm,
            int32_t* __restrict__ tmpk, uint64_t* __restrict__ first, double2* __restrict__ disp,
            uint32_t* __restrict__ own_v, uint32_t* __restrict__ own_c) {
  const int i = (int)((blockIdx.x * (unsigned)kThreads + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const bool active = i < n && !done[i];
  const int c = active ? gcen[i] : -1;
  const int nm = active ? cnt[i] : 0;
  const int o0 = active ? off[i] : 0;
  int* M = mem + o0;
  int* K = key + o0;
  int* Mu = tmpm + o0;
  int* Ku = tmpk + o0;
  uint64_t* F = first + o0;
  const double d = active ? (0.5 + 4.5 * draws[2 * i + 1].x) * p.eps : 0.0;
  if (active && lane == 0) {
    int k = 1;
    for_members(m, g, c, d, [&](int w) {
      if (k < nm) {  // the same query as group_count's, so k stays below nm
        Mu[k] = w;
        Ku[k] = m.vold[w];
      }
      ++k;
    });
    M[0] = c;
    K[0] = m.vold[c];
  }
  __syncthreads();
  for (int j = 1 + lane; j < nm; j += 64) {
    const int kj = Ku[j];
    int r = 1;
    for (int l = 1; l < nm; ++l) r += Ku[l] < kj ? 1 : 0;
    M[r] = Mu[j];
    K[r] = kj;
  }
  __syncthreads();
  // bit k of F[j]: triangle k of member j holds no member before j (k < 64; lane 0 decides the
  // rest when it adds them up)
  for (int j = lane; j < nm; j += 64) {
    const int v = M[j];
    uint64_t bits = 0;
    for (int k = m.vtri_off[v], end = min(m.vtri_off[v + 1], m.vtri_off[v] + 64); k < end; ++k) {
      const int4 tr = m.tri[m.vtri[k]];
      const int px = member_pos(m, M, K, nm, tr.x), py = member_pos(m, M, K, nm, tr.y),
                pz = member_pos(m, M, K, nm, tr.z);
      const bool earlier = (px >= 0 && px < j) || (py >= 0 && py < j) || (pz >= 0 && pz < j);
      if (!earlier) bits |= 1ull << (k - m.vtri_off[v]);
    }
    F[j] = bits;
  }
  __syncthreads();
  if (active && lane == 0) {
    // area of the triangles holding any member, each at the first member (in order) holding it
    double area = 0.0;
    for (int j = 0; j < nm; ++j) {
      const int v = M[j];
      const uint64_t bits = F[j];
      const int k0 = m.vtri_off[v];
      for (int k = k0, end = m.vtri_off[v + 1]; k < end; ++k) {
        const int tid = m.vtri[k];
        bool is_first;
        if (k - k0 < 64) {
          is_first = (bits >> (k - k0)) & 1;
        } else {
          const int4 tr = m.tri[tid];
          const int px = member_pos(m, M, K, nm, tr.x), py = member_pos(m, M, K, nm, tr.y),
                    pz = member_pos(m, M, K, nm, tr.z);
          is_first = !((px >= 0 && px < j) || (py >= 0 && py < j) || (pz >= 0 && pz < j));
        }
        if (is_first) area = area + tri_area(m, tid);
      }
    }
    const double k = lambda * sqrt(area);
    const double2 xi = draws[2 * i];
    disp[i] = make_double2(k * xi.x, k * xi.y);
  }
  __syncthreads();
  if (!active || own_v == nullptr) return;  // no claims: the joint group moves
  const double2 D = disp[i];
  const uint32_t pri = group_priority(i);
  auto claim_c = [&](int cell) { atomicMin(&own_c[cell], pri); };
  for_cells_lanes(gc, m.xyi[c], d * kQueryWiden, lane, claim_c);
  for (int j = lane; j < nm; j += 64) {
    const int v = M[j];
    const double2 o = m.xyi[v], dv = member_disp(m, v, D);
    claim_c(cell_of(gc, o));
    claim_c(cell_of(gc, make_double2(o.x + dv.x, o.y + dv.y)));
    for_hops2(m, v, [&](int x) { atomicMin(&own_v[x], pri); });
  }
}

// One wave per group: whether group i may move, i.e. it holds the cells it claimed and no vertex
// within three edges of its members carries a lower priority (no position changes during this
// pass). The lanes take the members; the wave's vote decides.
__global__ void __launch_bounds__(kThreads)
group_check(MeshDev m, VGrid gc, Par p, const int32_t* __restrict__ gcen,
            const double2* __restrict__ draws, const uint8_t* __restrict__ done, int n,
            const int32_t* __restrict__ off, const int32_t* __restrict__ cnt,
            const int32_t* __restrict__ mem, const double2* __restrict__ disp,
            const uint32_t* __restrict__ own_v, const uint32_t* __restrict__ own_c,
            uint8_t* __restrict__ won) {
  const int i = (int)((blockIdx.x * (unsigned)kThreads + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  if (done[i]) {
    if (lane == 0) won[i] = 0;
    return;
  }
  bool ok = true;
  const uint32_t pri = group_priority(i);
  auto held_c = [&](int cell) { ok = ok && own_c[cell] == pri; };
  const double d = (0.5 + 4.5 * draws[2 * i + 1].x) * p.eps;
  for_cells_lanes(gc, m.xyi[gcen[i]], d * kQueryWiden, lane, held_c);
  const int* M = mem + off[i];
  const double2 D = disp[i];
  for (int j = lane; j < cnt[i] && ok; j += 64) {
    const int v = M[j];
    const double2 o = m.xyi[v], dv = member_disp(m, v, D);
    held_c(cell_of(gc, o));
    held_c(cell_of(gc, make_double2(o.x + dv.x, o.y + dv.y)));
    for_hops3(m, v, [&](int x) { ok = ok && own_v[x] >= pri; });
  }
  const bool all = __ballot(!ok) == 0;
  if (lane == 0) won[i] = all ? 1 : 0;
}

constexpr int kSlots = 160;    // C-edges of one move that a wave's tables hold
constexpr int kWaveThreads = 64;  // kernels that spread one move over a wave (a workgroup)

// A wave's LDS for one move (see wave_change).
struct WaveLds {
  int nb[kLdsNbrs];
  int slot_e[kSlots];
  double slot_c[kSlots];
  double slot_v[kSlots];
  uint8_t slot_ok[kSlots];
  double new_len[kLdsNbrs], short_d[kLdsNbrs], angle_d[kLdsNbrs];
  int free_n[kLdsNbrs], free_off[kLdsNbrs];
  int hkey[kHash];
  uint16_t hslot[kHash];
  int fnb[kLdsNbrs], fce[kCache];
  double fcc[kCache];
  int n_slots;
};

// The change of f of moving internal vertex v to q, spread over a wave: every lane of the
// workgroup calls it with the same v and q. The lanes list v's C-edges in move_change's order (its
// edges, the edges between pairs of its neighbours, one pair per lane, then the FREE neighbours'
// edges, placed by a prefix sum of their counts), compute each one's new c into an LDS hash table,
// visit them one per lane with move_change's code, and take the angle and length terms one per
// lane; lane 0 adds the results in move_change's order, so its *df is bit for bit move_change's.
// With CHECK, the result is CCSP_MOVE_FOLDS (on every lane, *df untouched) when a triangle of v
// would not stay strictly counter-clockwise. A vertex with more than kLdsNbrs neighbours or
// kSlots C-edges takes move_change on lane 0 (*wide set). wave_commit then applies the move.
template <bool CHECK>
__device__ __forceinline__ int wave_change(const MeshDev& m, const Par& p, int v, double2 q, WaveLds& w,
                           int lane, double* df, bool* wide_out) {
  const int a0 = m.adj_off[v], deg = m.adj_off[v + 1] - a0;
  const int t0 = m.vtri_off[v], nt = m.vtri_off[v + 1] - t0;
  const int npair = deg * (deg - 1) / 2;
  bool wide = deg > kLdsNbrs || nt > kLdsNbrs || deg + npair > kSlots;
  if (!wide) {
    bool folds = false;
    if (lane < deg) {
      const int2 a = m.adj[a0 + lane];
      w.nb[lane] = a.x;
      w.slot_e[lane] = a.y;
      const int2 ab = m.edge_v[a.y];
      const double ln = dist(pos(m.xyi, ab.x, v, q), pos(m.xyi, ab.y, v, q));
      w.new_len[lane] = ln;
      w.short_d[lane] = short_term(ln, p.eps0) - short_term(m.len[a.y], p.eps0);
    }
    if (lane < nt) {
      const int4 t = m.tri[m.vtri[t0 + lane]];
      if (CHECK)
        folds = orient_sign(pos(m.xyi, t.x, v, q), pos(m.xyi, t.y, v, q),
                            pos(m.xyi, t.z, v, q)) <= 0;
      w.angle_d[lane] = triangle_angles(m.xyi, t, v, q, p.delta, p.polish) -
                        triangle_angles(m.xyi, t, -1, q, p.delta, p.polish);
    }
    for (int h = lane; h < kHash; h += kWaveThreads) w.hkey[h] = -1;
    if (CHECK && __ballot(folds) != 0) {
      *wide_out = false;
      __syncthreads();
      return CCSP_MOVE_FOLDS;
    }
    __syncthreads();
    // edges joining two neighbours, pairs (a, b), a < b, in row order; -1 where none
    for (int pi = lane; pi < npair; pi += kWaveThreads) {
      int a = 0, r = pi;
      while (r >= deg - 1 - a) {
        r -= deg - 1 - a;
        ++a;
      }
      w.slot_e[deg + pi] = find_edge(m, w.nb[a], w.nb[a + 1 + r]);
    }
    // edges from a FREE neighbour F to a vertex that is not FREE, v or a neighbour of v
    auto qualifies = [&](int C) {
      if (C == v || m.vk[C].x == CCSP_VERTEX_FREE) return false;
      for (int l = 0; l < deg; ++l)
        if (w.nb[l] == C) return false;
      return true;
    };
    if (lane < deg) {
      const int F = w.nb[lane];
      int k = 0;
      if (m.vk[F].x == CCSP_VERTEX_FREE)
        for (int r = m.adj_off[F], re = m.adj_off[F + 1]; r < re; ++r)
          k += qualifies(m.adj[r].x) ? 1 : 0;
      w.free_n[lane] = k;
    }
    __syncthreads();
    if (lane == 0) {
      int total = deg + npair;
      for (int l = 0; l < deg; ++l) {
        w.free_off[l] = total;
        total += w.free_n[l];
      }
      w.n_slots = total <= kSlots ? total : -1;
    }
    __syncthreads();
    const int ns = w.n_slots;
    wide = ns < 0;
    if (!wide) {
      if (lane < deg && w.free_n[lane] > 0) {
        const int F = w.nb[lane];
        int k = w.free_off[lane];
        for (int r = m.adj_off[F], re = m.adj_off[F + 1]; r < re; ++r)
          if (qualifies(m.adj[r].x)) w.slot_e[k++] = m.adj[r].y;
      }
      __syncthreads();
      // the new c of every C-edge (each listed once), into the slots and the table
      for (int sl = lane; sl < ns; sl += kWaveThreads) {
        const int e = w.slot_e[sl];
        if (e < 0) continue;
        const int2 ab = m.edge_v[e];
        const bool ok = contractible_at(m, m.xyi, e, ab.x, ab.y, p.eps, v, q);
        const double c = c_of_len(ok, sl < deg ? w.new_len[sl] : m.len[e], p.eps);
        w.slot_c[sl] = c;
        w.slot_ok[sl] = ok ? 1 : 0;
        int h = (int)(group_hash((uint32_t)e) & (kHash - 1));
        while (atomicCAS(&w.hkey[h], -1, e) != -1) h = (h + 1) & (kHash - 1);
        w.hslot[h] = (uint16_t)sl;
      }
      __syncthreads();
      const MoveCtxT<1, true> ctx{m,       m.xyi,   p,      v,       q,        w.nb,
                                  deg,     nullptr, nullptr, w.hkey, w.hslot, w.slot_c};
      for (int sl = lane; sl < ns; sl += kWaveThreads) {
        const int e = w.slot_e[sl];
        w.slot_v[sl] = e >= 0 ? ctx.visit(e) : 0.0;
      }
      __syncthreads();
      if (lane == 0) {
        double sa = 0.0, se = 0.0, ss = 0.0;
        for (int t = 0; t < nt; ++t) sa += w.angle_d[t];
        for (int k = 0; k < deg; ++k) {
          se += w.slot_v[k];
          ss += w.short_d[k];
        }
        for (int sl = deg; sl < ns; ++sl)
          if (w.slot_e[sl] >= 0) se += w.slot_v[sl];
        *df = se + p.mu_angle * sa + p.mu_len * ss;
      }
      *wide_out = false;
      return CCSP_MOVE_OK;
    }
  }
  *wide_out = true;
  int st = CCSP_MOVE_OK;
  if (lane == 0) {
    double dfj = 0.0;
    st = move_change<CHECK, 1>(m, m.xyi, p, v, q, MoveLds{w.fnb, w.fce, w.fcc}, &dfj);
    if (st == CCSP_MOVE_OK) *df = dfj;
    w.n_slots = st;
  }
  __syncthreads();
  st = w.n_slots;
  __syncthreads();
  return st;
}

// Applies the move of wave_change (status CCSP_MOVE_OK): v's new position and the scratch the
// move changes, from the wave's tables as refresh_scratch would write it (on lane 0 with
// refresh_scratch for a wide vertex). Every lane calls it; ends with the workgroup in step.
__device__ __forceinline__ void wave_commit(const MeshDev& m, const Par& p, int v, double2 q, WaveLds& w,
                            int lane, bool wide) {
  if (wide) {
    if (lane == 0) {
      m.xyi[v] = q;
      refresh_scratch(m, p, v);
    }
    __syncthreads();
    return;
  }
  const int deg = m.adj_off[v + 1] - m.adj_off[v];
  const int ns = w.n_slots;
  if (lane == 0) m.xyi[v] = q;
  for (int sl = lane; sl < ns; sl += kWaveThreads) {
    const int e = w.slot_e[sl];
    if (e < 0) continue;
    if (sl < deg) m.len[e] = w.new_len[sl];
    m.contr[e] = w.slot_ok[sl];
    m.c[e] = w.slot_c[sl];
  }
  __syncthreads();
}

// The move of every group that holds its claims, one wave (a workgroup) per group: its members
// moved one after another by D (projected when constrained), each with its change of f against
// the positions and scratch its predecessors left (wave_change), so that the changes add up to the
// change of f of the whole move; valid when every triangle of every member is strictly
// counter-clockwise at the end; rejected or invalid moves are undone from xy_out, which holds the
// positions before them.
__global__ void __launch_bounds__(kWaveThreads)
group_apply(MeshDev m, Par p, double temperature, double2* __restrict__ xy_out, int n,
            const int32_t* __restrict__ off, const int32_t* __restrict__ cnt,
            const int32_t* __restrict__ mem, const double2* __restrict__ disp,
            const double* __restrict__ u, const uint8_t* __restrict__ won, int rnd,
            uint8_t* __restrict__ done, double* __restrict__ delta,
            int32_t* __restrict__ status, int32_t* __restrict__ members,
            int32_t* __restrict__ round, unsigned long long* __restrict__ applied) {
  __shared__ WaveLds w;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n || !won[i]) return;
  const int* M = mem + off[i];
  const int nm = cnt[i];
  const double2 D = disp[i];
  double df = 0.0;  // lane 0's
  for (int j = 0; j < nm; ++j) {
    const int v = M[j];
    const double2 o = m.xyi[v], dv = member_disp(m, v, D);
    const double2 q = make_double2(o.x + dv.x, o.y + dv.y);
    double dfj = 0.0;
    bool wide = false;
    wave_change<false>(m, p, v, q, w, lane, &dfj, &wide);
    if (lane == 0) df += dfj;
    wave_commit(m, p, v, q, w, lane, wide);
  }
  bool ok = true;
  for (int j = lane; j < nm && ok; j += kWaveThreads) {
    const int v = M[j];
    for (int k = m.vtri_off[v], end = m.vtri_off[v + 1]; k < end && ok; ++k) {
      const int4 tr = m.tri[m.vtri[k]];
      ok = orient_sign(m.xyi[tr.x], m.xyi[tr.y], m.xyi[tr.z]) > 0;
    }
  }
  const bool valid = __ballot(!ok) == 0;
  bool took = false;
  if (lane == 0) {
    int st = CCSP_MOVE_FOLDS;
    if (valid) {
      st = CCSP_MOVE_REJECTED;
      if (df <= 0.0 || u[i] < exp(-df / temperature)) {
        st = CCSP_MOVE_OK;
        took = true;
      }
    } else {
      df = __builtin_huge_val();
    }
    status[i] = st;
    delta[i] = df;
    members[i] = nm;
    round[i] = rnd;
    done[i] = 1;
    atomicAdd(applied, 1ull);
  }
  took = __ballot(took) != 0;
  if (took) {
    for (int j = lane; j < nm; j += kWaveThreads) xy_out[m.vold[M[j]]] = m.xyi[M[j]];
    return;
  }
  // undo: every member back, then the scratch around them (lengths first; each edge's values
  // depend on the positions and lengths alone, so the lanes' order does not matter)
  for (int j = lane; j < nm; j += kWaveThreads) m.xyi[M[j]] = xy_out[m.vold[M[j]]];
  __syncthreads();
  for (int j = lane; j < nm; j += kWaveThreads) refresh_lengths(m, M[j]);
  __syncthreads();
  for (int j = lane; j < nm; j += kWaveThreads) refresh_rules(m, p, M[j]);
}

// One class of a sweep: Metropolis steps for its vertices (internal ids), which are pairwise more
// than four edges apart, so that each move's reads (within four edges of its vertex) and writes
// (its position, and scratch of edges within one edge of it) never meet another's. One wave (a
// 64-thread workgroup) per vertex: every lane makes the vertex's proposal alike (the same loads),
// and wave_change spreads its change of f over the lanes (bit for bit move_change's).
// kind CCSP_PROPOSE_DISPLACE: the vertex moves by disp[i] (scaled by lambda * eta when lambda > 0);
// the other kinds draw the new position from the vertex's neighbourhood with draws[2i], draws[2i+1]
// (Secs. 3.2.4-3.2.6). Accepted moves are counted into *accepted when it is given.
__global__ void __launch_bounds__(kWaveThreads)
anneal_class(MeshDev m, Par p, double temperature, double lambda, int kind,
                  double2* __restrict__ xy_out, const int32_t* __restrict__ cls,
                  const double2* __restrict__ disp, const double* __restrict__ u, int n,
                  double* __restrict__ delta, int32_t* __restrict__ status,
                  unsigned long long* __restrict__ accepted) {
  __shared__ WaveLds w;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n) return;
  const int v = cls[i];
  const int cv = m.vold[v];
  double2 q;
  bool skip;
  propose_move(m, p, lambda, kind, v, i, disp, &q, &skip);
  double df = __builtin_huge_val();
  int st = CCSP_MOVE_SKIPPED;
  bool took = false;
  if (!skip) {
    if (!isfinite(q.x) || !isfinite(q.y)) {
      st = CCSP_MOVE_BAD;
    } else if (m.vk[v].x == CCSP_VERTEX_ORIGINAL) {
      st = CCSP_MOVE_FIXED;
    } else {
      double dfl = 0.0;
      bool wide = false;
      st = wave_change<true>(m, p, v, q, w, lane, &dfl, &wide);
      if (st == CCSP_MOVE_OK) {
        df = __shfl(dfl, 0);
        if (df <= 0.0 || u[i] < exp(-df / temperature)) {
          wave_commit(m, p, v, q, w, lane, wide);
          took = true;
        } else {
          st = CCSP_MOVE_REJECTED;
        }
      }
    }
  }
  if (lane == 0) {
    if (took) xy_out[cv] = q;
    status[i] = st;
    delta[i] = df;
    if (took && accepted) atomicAdd(accepted, 1ull);
  }
}

// ---- joint moves of many vertices with one decision (the second variant of Sec. 3.2.2)

// Flags of a joint move (bits of *flags).
constexpr int kJointBad = 1;    // an id out of range, not movable, repeated, or a draw not finite
constexpr int kJointFolds = 2;  // a triangle of a moved vertex not strictly counter-clockwise

// Every term of f at the staged positions and edge scratch: te[e] = w(e) |e| (as terms_pass),
// ts[e] the length penalty of e, ta[t] the angle penalty of t.
__global__ void __launch_bounds__(kThreads)
joint_terms(MeshDev m, Par p, double* __restrict__ te, double* __restrict__ ts,
            double* __restrict__ ta) {
  const int n = m.ne > m.nt ? m.ne : m.nt;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    if (i < m.ne) {
      const double w = p.polish ? 1.0 : weight_from(m.c, m.edge_nbr[i]);
      te[i] = w * m.len[i];
      ts[i] = short_term(m.len[i], p.eps0);
    }
    if (i < m.nt) ta[i] = triangle_angles(m.xyi, m.tri[i], -1, make_double2(0, 0), p.delta, p.polish);
  }
}

// New position of every vertex of the joint move, from the positions before it: vid[i] (caller
// id) moves by lambda * eta * xi[i], eta the square root of the area of its triangles (summed in
// the caller's triangle order), projected on its original edge when constrained. mark holds the
// epoch of the last joint move that named each vertex, which finds repeats.
__global__ void __launch_bounds__(kThreads)
joint_prepare(MeshDev m, double lambda, const int32_t* __restrict__ vid,
              const double2* __restrict__ xi, int64_t k, uint32_t epoch,
              uint32_t* __restrict__ mark, double2* __restrict__ qnew, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k) return;
  const int cv = vid[i];
  const double2 x = xi[i];
  if (cv < 0 || cv >= m.nv || !isfinite(x.x) || !isfinite(x.y)) {
    atomicOr(flags, kJointBad);
    return;
  }
  const int v = m.vnew[cv];
  if (m.vk[v].x == CCSP_VERTEX_ORIGINAL || atomicExch(&mark[v], epoch) == epoch) {
    atomicOr(flags, kJointBad);
    return;
  }
  double area = 0.0;
  for (int j = m.vtri_off[v], end = m.vtri_off[v + 1]; j < end; ++j)
    area += tri_area(m, m.vtri[j]);
  const double kk = lambda * sqrt(area);
  double2 d = make_double2(kk * x.x, kk * x.y);
  const int2 kl = m.vk[v];
  if (kl.x == CCSP_VERTEX_CONSTRAINED) {
    const int2 ends = m.prim_v[kl.y];
    const double2 a = m.xyi[ends.x], b = m.xyi[ends.y];
    const double ex = b.x - a.x, ey = b.y - a.y;
    const double s = (d.x * ex + d.y * ey) / (ex * ex + ey * ey);
    d = make_double2(s * ex, s * ey);
  }
  const double2 o = m.xyi[v];
  qnew[i] = make_double2(o.x + d.x, o.y + d.y);
}

// The joint move's positions into the staged ones (unless a flag is set).
__global__ void __launch_bounds__(kThreads)
joint_apply(MeshDev m, const int32_t* __restrict__ vid, const double2* __restrict__ qnew,
            int64_t k, const int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k || *flags != 0) return;
  m.xyi[m.vnew[vid[i]]] = qnew[i];
}

// Validity after the joint move: every triangle of every moved vertex strictly counter-clockwise.
__global__ void __launch_bounds__(kThreads)
joint_check(MeshDev m, const int32_t* __restrict__ vid, int64_t k, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k || (*flags & kJointBad) != 0) return;
  const int v = m.vnew[vid[i]];
  for (int j = m.vtri_off[v], end = m.vtri_off[v + 1]; j < end; ++j) {
    const int4 t = m.tri[m.vtri[j]];
    if (orient_sign(m.xyi[t.x], m.xyi[t.y], m.xyi[t.z]) <= 0) {
      atomicOr(flags, kJointFolds);
      return;
    }
  }
}

// Per-workgroup sums (fixed stride per thread) of every term's new minus stored old value:
// part[b] edges' w |e|, part[nb + b] angle penalties, part[2 nb + b] length penalties.
__global__ void __launch_bounds__(kThreads)
joint_diff(MeshDev m, Par p, const double* __restrict__ te, const double* __restrict__ ts,
           const double* __restrict__ ta, double* __restrict__ part) {
  __shared__ double sh[kThreads];
  const int n = m.ne > m.nt ? m.ne : m.nt;
  double se = 0.0, sa = 0.0, sl = 0.0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    if (i < m.ne) {
      const double w = p.polish ? 1.0 : weight_from(m.c, m.edge_nbr[i]);
      se += w * m.len[i] - te[i];
      sl += short_term(m.len[i], p.eps0) - ts[i];
    }
    if (i < m.nt)
      sa += triangle_angles(m.xyi, m.tri[i], -1, make_double2(0, 0), p.delta, p.polish) - ta[i];
  }
  se = block_sum(se, sh);
  sa = block_sum(sa, sh);
  sl = block_sum(sl, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = se;
    part[gridDim.x + blockIdx.x] = sa;
    part[2 * gridDim.x + blockIdx.x] = sl;
  }
}

// out[0] = the change of f, out[1..3] = those of w_contr, P_angle and P_len (one workgroup).
__global__ void __launch_bounds__(kThreads)
joint_finish(const double* __restrict__ part, int nb, Par p, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const double dw = sum_fixed(part, nb, sh);
  const double da = sum_fixed(part + nb, nb, sh);
  const double dl = sum_fixed(part + 2 * nb, nb, sh);
  if (threadIdx.x == 0) {
    out[0] = dw + p.mu_angle * da + p.mu_len * dl;
    out[1] = dw;
    out[2] = da;
    out[3] = dl;
  }
}

// An accepted joint move's positions into the caller's array.
__global__ void __launch_bounds__(kThreads)
joint_commit(const int32_t* __restrict__ vid, const double2* __restrict__ qnew, int64_t k,
             double2* __restrict__ xy_out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < k) xy_out[vid[i]] = qnew[i];
}

// ---- the joint move of several groups (the second variant of Sec. 3.2.3): every member moves
// with the displacement of the first group, in centre order, that holds it; one decision.

// owner[v] = the lowest index of the groups holding v (one wave per group).
__global__ void __launch_bounds__(kThreads)
jgroup_owner(const int32_t* __restrict__ off, const int32_t* __restrict__ cnt,
             const int32_t* __restrict__ mem, int n, int32_t* __restrict__ owner) {
  const int i = (int)((blockIdx.x * (unsigned)kThreads + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int* M = mem + off[i];
  for (int j = lane; j < cnt[i]; j += 64) atomicMin(&owner[M[j]], i);
}

// Member slot off[i] + j of group i: its vertex (internal id) and new position when the group owns
// it, else -1 (one wave per group).
__global__ void __launch_bounds__(kThreads)
jgroup_prepare(MeshDev m, const int32_t* __restrict__ off, const int32_t* __restrict__ cnt,
               const int32_t* __restrict__ mem, const double2* __restrict__ disp,
               const int32_t* __restrict__ owner, int n, int32_t* __restrict__ vint,
               double2* __restrict__ qlist) {
  const int i = (int)((blockIdx.x * (unsigned)kThreads + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int* M = mem + off[i];
  const double2 D = disp[i];
  for (int j = lane; j < cnt[i]; j += 64) {
    const int v = M[j];
    const int slot = off[i] + j;
    if (owner[v] == i) {
      const double2 o = m.xyi[v], dv = member_disp(m, v, D);
      vint[slot] = v;
      qlist[slot] = make_double2(o.x + dv.x, o.y + dv.y);
    } else {
      vint[slot] = -1;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
jgroup_apply(MeshDev m, const int32_t* __restrict__ vint, const double2* __restrict__ qlist,
             int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < k && vint[i] >= 0) m.xyi[vint[i]] = qlist[i];
}

__global__ void __launch_bounds__(kThreads)
jgroup_check(MeshDev m, const int32_t* __restrict__ vint, int64_t k, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= k || vint[i] < 0) return;
  const int v = vint[i];
  for (int j = m.vtri_off[v], end = m.vtri_off[v + 1]; j < end; ++j) {
    const int4 t = m.tri[m.vtri[j]];
    if (orient_sign(m.xyi[t.x], m.xyi[t.y], m.xyi[t.z]) <= 0) {
      atomicOr(flags, kJointFolds);
      return;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
jgroup_commit(MeshDev m, const int32_t* __restrict__ vint, const double2* __restrict__ qlist,
              int64_t k, double2* __restrict__ xy_out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < k && vint[i] >= 0) xy_out[m.vold[vint[i]]] = qlist[i];
}

// objective_delta's moves with one wave (a 64-thread workgroup) per move: wave_change gives the
// change of f bit for bit as move_change. order (NULL: the identity) lists the move each
// workgroup evaluates.
__global__ void __launch_bounds__(kWaveThreads)
move_delta_wave(MeshDev m, Par p, const int32_t* __restrict__ vid, const double2* __restrict__ qv,
                int64_t k, const uint32_t* __restrict__ order, double* __restrict__ delta,
                int32_t* __restrict__ status) {
  __shared__ WaveLds w;
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x;
  if (t >= k) return;
  const int64_t i = order ? (int64_t)order[t] : t;
  const int cv = vid[i];
  const double2 q = qv[i];
  int st;
  double df = __builtin_huge_val();
  if (cv < 0 || cv >= m.nv || !isfinite(q.x) || !isfinite(q.y)) {
    st = CCSP_MOVE_BAD;
  } else if (m.vk[m.vnew[cv]].x == CCSP_VERTEX_ORIGINAL) {
    st = CCSP_MOVE_FIXED;
  } else {
    double dfl = 0.0;
    bool wide = false;
    st = wave_change<true>(m, p, m.vnew[cv], q, w, lane, &dfl, &wide);
    if (st == CCSP_MOVE_OK) df = dfl;
  }
  if (lane == 0) {
    status[i] = st;
    delta[i] = df;
  }
}

__global__ void __launch_bounds__(kThreads)
fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) a[i] = v;
}

// Bounding box of the positions: each workgroup reduces a grid-stride share of the vertices into
// part[4 * blockIdx.x ..] (min x, min y, max x, max y); with part == out and one workgroup over
// nparts partial boxes instead (nparts > 0), the final box.
__global__ void __launch_bounds__(kThreads)
bbox_kernel(MeshDev m, const double* __restrict__ in, int nparts, double* __restrict__ out) {
  __shared__ double sh[4][kThreads];
  double a = __builtin_huge_val(), b = a, c = -a, e = -a;
  if (nparts == 0) {
    for (int v = blockIdx.x * kThreads + threadIdx.x; v < m.nv; v += gridDim.x * kThreads) {
      const double2 q = m.xyi[v];
      a = fmin(a, q.x);
      b = fmin(b, q.y);
      c = fmax(c, q.x);
      e = fmax(e, q.y);
    }
  } else {
    for (int k = threadIdx.x; k < nparts; k += kThreads) {
      a = fmin(a, in[4 * k]);
      b = fmin(b, in[4 * k + 1]);
      c = fmax(c, in[4 * k + 2]);
      e = fmax(e, in[4 * k + 3]);
    }
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  sh[3][threadIdx.x] = e;
  __syncthreads();
  for (int s2 = kThreads / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + s2]);
      sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + s2]);
      sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + s2]);
      sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + s2]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void zero_counter(unsigned long long* __restrict__ c) {
  if (threadIdx.x == 0) c[0] = 0ull;
}

}  // namespace
}  // namespace ccsp

// ---- host: mesh construction and the C-ABI ----

struct MovableMesh {
  int device = -1;
  ccsp::MeshDev d{};
  void* mem = nullptr;
  std::vector<int32_t> edge_v;  // 2E in the caller's numbering, for mesh_info
  std::vector<int64_t> class_off;  // mesh_classes, computed on the first call
  std::vector<int32_t> class_v;    // caller ids, class by class
  int32_t* class_dev = nullptr;    // the same vertices, internal ids, on the device
  void* sched = nullptr;           // anneal_schedule: delta and status per movable vertex, counter
  void* order_ws = nullptr;        // objective_delta: sort keys, move indices, sort temporaries
  size_t order_bytes = 0;
  void* joint_ws = nullptr;        // anneal_joint: stored terms, marks, sums, new positions
  size_t joint_bytes = 0;
  uint32_t joint_epoch = 0;
};

namespace {

using ccsp::set_last_error;

int fail(int code, const std::string& msg) {
  set_last_error(msg.c_str());
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(CCSP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool check_params(const ObjectiveParams* p) {
  if (!p) return false;
  if (!(p->eps > 0) || !(p->delta > 0) || !(p->eps0 > 0) || !std::isfinite(p->eps) ||
      !std::isfinite(p->delta) || !std::isfinite(p->eps0) || !std::isfinite(p->mu_angle) ||
      !std::isfinite(p->mu_len) || p->reserved != 0)
    return false;
  return true;
}

// Workgroups of a pass over n items: enough to cover them, at most kMaxBlocks (the partial sums
// buffer holds 3 * kMaxBlocks values).
int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(ccsp::kMaxBlocks,
                                                     (n + ccsp::kThreads - 1) / ccsp::kThreads));
}

// Every call's first step: the caller's positions into internal order, then every edge's length,
// contractibility and c (edge_state, length-penalty partial sums in d.partial[0..grid_for(ne))).
void stage_edges(const ccsp::MeshDev& d, const ccsp::Par& p, const void* xy, hipStream_t s) {
  hipLaunchKernelGGL(ccsp::permute_positions, dim3(grid_for(d.nv)), dim3(ccsp::kThreads), 0, s, d,
                     (const double2*)xy);
  hipLaunchKernelGGL(ccsp::edge_state, dim3(grid_for(d.ne)), dim3(ccsp::kThreads), 0, s, d, p,
                     d.partial);
  hipLaunchKernelGGL(ccsp::rules_fresh, dim3(1), dim3(64), 0, s, d);
}

ccsp::Par to_par(const ObjectiveParams* p) {
  return ccsp::Par{p->eps, p->delta, p->eps0, p->mu_angle, p->mu_len, p->polish != 0};
}

int check_device(const MovableMesh* m) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != m->device) return fail(CCSP_E_ARG, "the mesh was loaded on another device");
  return CCSP_OK;
}

// Batches of at least this many moves are evaluated in the order of their vertices' internal ids
// (a breadth-first order of the mesh, so that close ids are close vertices), so that threads of a
// wave share the cache lines of their neighbourhoods; a random batch of 2^20 moves on 8 million vertices otherwise fetches each
// move's neighbourhood from memory on its own.
constexpr int64_t kSortMoves = 4096;

// Radix-sorts the move indices 0..k-1 by internal vertex id into the mesh's order workspace
// (grown, after synchronising `s`, when k exceeds every earlier batch); *order receives them.
int sort_moves(MovableMesh* mesh, const int32_t* vid, int64_t k, hipStream_t s,
               const uint32_t** order) {
  const ccsp::MeshDev& d = mesh->d;
  int end_bit = 1;
  while (end_bit < 32 && (int64_t(1) << end_bit) <= (int64_t)d.nv) ++end_bit;
  size_t tmp = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint32_t*)nullptr,
                                                    (uint32_t*)nullptr, (const uint32_t*)nullptr,
                                                    (uint32_t*)nullptr, (int)k, 0, end_bit, s);
  if (e != hipSuccess) return hip_fail(e, "objective_delta: sort size");
  const size_t col = (4 * (size_t)k + 255) & ~size_t(255);
  const size_t need = 4 * col + tmp;
  if (need > mesh->order_bytes) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "objective_delta: synchronise");
    if (mesh->order_ws) (void)hipFree(mesh->order_ws);
    mesh->order_ws = nullptr;
    mesh->order_bytes = 0;
    if (hipMalloc(&mesh->order_ws, need) != hipSuccess) {
      (void)hipGetLastError();
      mesh->order_ws = nullptr;
      return fail(CCSP_E_OOM, "objective_delta: device allocation failed");
    }
    mesh->order_bytes = need;
  }
  char* w = (char*)mesh->order_ws;
  auto* key = (uint32_t*)w;
  auto* key2 = (uint32_t*)(w + col);
  auto* idx = (uint32_t*)(w + 2 * col);
  auto* idx2 = (uint32_t*)(w + 3 * col);
  hipLaunchKernelGGL(ccsp::move_keys, dim3((unsigned)((k + ccsp::kThreads - 1) / ccsp::kThreads)),
                     dim3(ccsp::kThreads), 0, s, d, vid, k, key, idx);
  e = hipcub::DeviceRadixSort::SortPairs(w + 4 * col, tmp, key, key2, idx, idx2, (int)k, 0,
                                         end_bit, s);
  if (e != hipSuccess) return hip_fail(e, "objective_delta: sort");
  *order = idx2;
  return CCSP_OK;
}

}  // namespace

// Device scratch of one group sweep, released on every return.
struct GroupScratch {
  std::vector<void*> blocks;
  ~GroupScratch() {
    for (void* b : blocks) (void)hipFree(b);
  }
  template <class T>
  hipError_t get(T** p, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) blocks.push_back(q);
    *p = static_cast<T*>(q);
    return e;
  }
};

extern "C" {

int mesh_load(const MeshDesc* desc, MovableMesh** out) {
  if (!desc || !out) return fail(CCSP_E_ARG, "mesh_load: null argument");
  *out = nullptr;
  const int64_t V = desc->n_vertices, T = desc->n_triangles, P = desc->n_prims;
  if (V <= 0 || T <= 0 || P < 0 || !desc->kind || !desc->line || !desc->tri_v ||
      (P > 0 && !desc->prim_v))
    return fail(CCSP_E_ARG, "mesh_load: empty mesh or null array");
  if (V >= (int64_t(1) << 30) || T >= (int64_t(1) << 29) || P >= (int64_t(1) << 30))
    return fail(CCSP_E_ARG, "mesh_load: mesh too large for 32-bit ids");
  const int32_t* ctv = desc->tri_v;
  for (int64_t i = 0; i < V; ++i) {
    const int k = desc->kind[i];
    if (k != CCSP_VERTEX_ORIGINAL && k != CCSP_VERTEX_CONSTRAINED && k != CCSP_VERTEX_FREE)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_load: unknown vertex kind at " + std::to_string(i));
    if (k == CCSP_VERTEX_CONSTRAINED && (desc->line[i] < 0 || desc->line[i] >= P))
      return fail(CCSP_E_BAD_TRIANGULATION,
                  "mesh_load: constrained vertex " + std::to_string(i) + " names no original edge");
  }
  for (int64_t i = 0; i < 2 * P; ++i)
    if (desc->prim_v[i] < 0 || desc->prim_v[i] >= V)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_load: original edge end out of range");
  for (int64_t t = 0; t < T; ++t) {
    const int a = ctv[3 * t], b = ctv[3 * t + 1], c = ctv[3 * t + 2];
    if (a < 0 || a >= V || b < 0 || b >= V || c < 0 || c >= V)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_load: vertex id out of range in triangle " +
                                                std::to_string(t));
    if (a == b || b == c || c == a)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_load: triangle " + std::to_string(t) +
                                                " repeats a vertex");
  }
  const int64_t n3 = 3 * T;

  // Internal vertex order: breadth-first over the triangles' adjacency, so that neighbours get
  // nearby ids and the gathers of a pass stay within a narrow band of memory.
  std::vector<int32_t> vold, vnew(V, -1);
  {
    std::vector<int64_t> noff(V + 1, 0);
    for (int64_t f = 0; f < n3; ++f) noff[ctv[f] + 1] += 2;
    for (int64_t v = 0; v < V; ++v) noff[v + 1] += noff[v];
    std::vector<int32_t> nb(2 * n3);
    std::vector<int64_t> fill(noff.begin(), noff.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int i = 0; i < 3; ++i) {
        const int a = ctv[3 * t + i];
        nb[fill[a]++] = ctv[3 * t + (i + 1) % 3];
        nb[fill[a]++] = ctv[3 * t + (i + 2) % 3];
      }
    vold.reserve(V);
    for (int64_t s = 0; s < V; ++s) {
      if (vnew[s] >= 0) continue;
      size_t head = vold.size();
      vnew[s] = (int32_t)vold.size();
      vold.push_back((int32_t)s);
      while (head < vold.size()) {
        const int u = vold[head++];
        for (int64_t j = noff[u]; j < noff[u + 1]; ++j) {
          const int w = nb[j];
          if (vnew[w] < 0) {
            vnew[w] = (int32_t)vold.size();
            vold.push_back(w);
          }
        }
      }
    }
  }
  // Internal triangles: ordered by their lowest internal vertex (stable in the caller's order),
  // vertices relabelled, local order kept.
  std::vector<int32_t> told(T), tv(n3);
  {
    std::vector<int64_t> off(V + 1, 0);
    auto low = [&](int64_t t) {
      return std::min(vnew[ctv[3 * t]], std::min(vnew[ctv[3 * t + 1]], vnew[ctv[3 * t + 2]]));
    };
    for (int64_t t = 0; t < T; ++t) ++off[low(t) + 1];
    for (int64_t v = 0; v < V; ++v) off[v + 1] += off[v];
    for (int64_t t = 0; t < T; ++t) told[off[low(t)]++] = (int32_t)t;
    for (int64_t ti = 0; ti < T; ++ti)
      for (int i = 0; i < 3; ++i) tv[3 * ti + i] = vnew[ctv[3 * told[ti] + i]];
  }
  // local edges of the internal triangles sorted by (lower end, higher end, flat index)
  auto lo_of = [&](int64_t f) {
    const int64_t t = f / 3, i = f % 3;
    return std::min(tv[3 * t + (i + 1) % 3], tv[3 * t + (i + 2) % 3]);
  };
  auto hi_of = [&](int64_t f) {
    const int64_t t = f / 3, i = f % 3;
    return std::max(tv[3 * t + (i + 1) % 3], tv[3 * t + (i + 2) % 3]);
  };
  std::vector<int32_t> order(n3);
  {
    std::vector<int64_t> boff(V + 1, 0);
    for (int64_t f = 0; f < n3; ++f) ++boff[lo_of(f) + 1];
    for (int64_t v = 0; v < V; ++v) boff[v + 1] += boff[v];
    std::vector<int64_t> fill(boff.begin(), boff.end() - 1);
    for (int64_t f = 0; f < n3; ++f) order[fill[lo_of(f)]++] = (int32_t)f;
    for (int64_t v = 0; v < V; ++v)
      std::stable_sort(order.begin() + boff[v], order.begin() + boff[v + 1],
                       [&](int32_t x, int32_t y) { return hi_of(x) < hi_of(y); });
  }
  // Edges. The triangles of an edge are kept in the caller's triangle order: it fixes the order
  // of the product x.
  std::vector<int32_t> tri_edge(n3), ev, etri, eloc;
  ev.reserve(n3 + 16);
  for (int64_t j = 0; j < n3;) {
    const int32_t f = order[j];
    const int lo = lo_of(f), hi = hi_of(f);
    int64_t k = j + 1;
    while (k < n3 && lo_of(order[k]) == lo && hi_of(order[k]) == hi) ++k;
    if (k - j > 2)
      return fail(CCSP_E_BAD_TRIANGULATION,
                  "mesh_load: edge (" + std::to_string(vold[lo]) + ", " + std::to_string(vold[hi]) +
                      ") lies in more than two triangles");
    int32_t g0 = order[j], g1 = k - j == 2 ? order[j + 1] : -1;
    if (g1 >= 0) {
      auto from = [&](int32_t g) { return tv[3 * (g / 3) + (g % 3 + 1) % 3]; };
      if (from(g0) == from(g1))
        return fail(CCSP_E_BAD_TRIANGULATION,
                    "mesh_load: triangles " + std::to_string(told[g0 / 3]) + " and " +
                        std::to_string(told[g1 / 3]) + " run through their shared edge the same way");
      if (told[g1 / 3] < told[g0 / 3]) std::swap(g0, g1);
    }
    const int32_t e = (int32_t)(ev.size() / 2);
    ev.push_back(lo);
    ev.push_back(hi);
    etri.push_back(g0 / 3);
    eloc.push_back(g0 % 3);
    etri.push_back(g1 >= 0 ? g1 / 3 : -1);
    eloc.push_back(g1 >= 0 ? g1 % 3 : -1);
    for (int64_t s = j; s < k; ++s) tri_edge[order[s]] = e;
    j = k;
  }
  const int64_t E = (int64_t)ev.size() / 2;
  std::vector<int32_t> enbr(4 * E, -1), eopp(2 * E, -1);
  for (int64_t e = 0; e < E; ++e)
    for (int s = 0; s < 2; ++s) {
      const int32_t t = etri[2 * e + s], i = eloc[2 * e + s];
      if (t < 0) continue;
      eopp[2 * e + s] = tv[3 * t + i];
      enbr[4 * e + 2 * s] = tri_edge[3 * t + (i + 1) % 3];
      enbr[4 * e + 2 * s + 1] = tri_edge[3 * t + (i + 2) % 3];
    }
  // the caller's edge numbering: edges sorted by (lower, higher) caller vertex id
  std::vector<int32_t> eperm(E), edge_can(2 * E);
  {
    std::vector<int32_t> clo(E), chi(E);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t a = vold[ev[2 * e]], b = vold[ev[2 * e + 1]];
      clo[e] = std::min(a, b);
      chi[e] = std::max(a, b);
    }
    std::vector<int64_t> off(V + 1, 0);
    for (int64_t e = 0; e < E; ++e) ++off[clo[e] + 1];
    for (int64_t v = 0; v < V; ++v) off[v + 1] += off[v];
    std::vector<int32_t> eo(E);
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (int64_t e = 0; e < E; ++e) eo[fill[clo[e]]++] = (int32_t)e;
    for (int64_t v = 0; v < V; ++v)
      std::sort(eo.begin() + off[v], eo.begin() + off[v + 1],
                [&](int32_t x, int32_t y) { return chi[x] < chi[y]; });
    for (int64_t r = 0; r < E; ++r) {
      eperm[eo[r]] = (int32_t)r;
      edge_can[2 * r] = clo[eo[r]];
      edge_can[2 * r + 1] = chi[eo[r]];
    }
  }
  // neighbours: edges are sorted by (lo, hi), so each vertex's list comes out increasing
  std::vector<int32_t> adj_off(V + 1, 0), adj(4 * E);
  for (int64_t e = 0; e < E; ++e) {
    ++adj_off[ev[2 * e] + 1];
    ++adj_off[ev[2 * e + 1] + 1];
  }
  for (int64_t v = 0; v < V; ++v) adj_off[v + 1] += adj_off[v];
  {
    std::vector<int32_t> fill(adj_off.begin(), adj_off.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int a = ev[2 * e], b = ev[2 * e + 1];
      int32_t* pa = &adj[2 * fill[a]++];
      pa[0] = b;
      pa[1] = (int32_t)e;
      int32_t* pb = &adj[2 * fill[b]++];
      pb[0] = a;
      pb[1] = (int32_t)e;
    }
  }
  // nontrivial 1-hop vertices: common neighbours of an edge's ends other than its opposite
  // vertices (rows of adj are increasing, so a merge finds the common ones)
  std::vector<int32_t> hop_off(E + 1, 0), hop_v;
  for (int64_t e = 0; e < E; ++e) {
    const int a = ev[2 * e], b = ev[2 * e + 1];
    int32_t i = adj_off[a], j = adj_off[b];
    const int32_t ie = adj_off[a + 1], je = adj_off[b + 1];
    while (i < ie && j < je) {
      const int x = adj[2 * i], y = adj[2 * j];
      if (x < y) {
        ++i;
      } else if (y < x) {
        ++j;
      } else {
        if (x != eopp[2 * e] && x != eopp[2 * e + 1]) hop_v.push_back(x);
        ++i;
        ++j;
      }
    }
    hop_off[e + 1] = (int32_t)hop_v.size();
  }
  if (hop_v.empty()) hop_v.push_back(0);
  std::vector<int32_t> vtri_off(V + 1, 0), vtri(n3);
  for (int64_t f = 0; f < n3; ++f) ++vtri_off[tv[f] + 1];
  for (int64_t v = 0; v < V; ++v) vtri_off[v + 1] += vtri_off[v];
  {
    // each vertex's triangles in the caller's triangle order (sums over a vertex's triangles,
    // such as its star area, then have a caller-visible order)
    std::vector<int32_t> tnew(T);
    for (int64_t ti = 0; ti < T; ++ti) tnew[told[ti]] = (int32_t)ti;
    std::vector<int32_t> fill(vtri_off.begin(), vtri_off.end() - 1);
    for (int64_t ct = 0; ct < T; ++ct) {
      const int32_t ti = tnew[ct];
      for (int i = 0; i < 3; ++i) vtri[fill[tv[3 * (int64_t)ti + i]]++] = ti;
    }
  }
  std::vector<int32_t> tri4(4 * T), tedge4(4 * T), vk(2 * V);
  for (int64_t t = 0; t < T; ++t) {
    for (int i = 0; i < 3; ++i) {
      tri4[4 * t + i] = tv[3 * t + i];
      tedge4[4 * t + i] = tri_edge[3 * t + i];
    }
    tri4[4 * t + 3] = tedge4[4 * t + 3] = 0;
  }
  for (int64_t vi = 0; vi < V; ++vi) {
    const int32_t v = vold[vi];
    vk[2 * vi] = desc->kind[v];
    vk[2 * vi + 1] = desc->kind[v] == CCSP_VERTEX_CONSTRAINED ? desc->line[v] : -1;
  }
  std::vector<int32_t> pv(2 * std::max<int64_t>(P, 1), 0);
  for (int64_t i = 0; i < 2 * P; ++i) pv[i] = vnew[desc->prim_v[i]];

  struct Part { const void* src; size_t bytes; void** dst; };
  auto m = new MovableMesh();
  hipError_t he = hipGetDevice(&m->device);
  if (he != hipSuccess) {
    delete m;
    return hip_fail(he, "hipGetDevice");
  }
  ccsp::MeshDev& d = m->d;
  d.nv = (int32_t)V;
  d.nt = (int32_t)T;
  d.ne = (int32_t)E;
  d.np = (int32_t)P;
  void* p_edge_v; void* p_nbr; void* p_opp; void* p_etri; void* p_tri; void* p_tedge;
  void* p_adj_off; void* p_adj; void* p_vtri_off; void* p_vtri; void* p_vk; void* p_prim;
  void* p_vold; void* p_vnew; void* p_eperm; void* p_xyi; void* p_hop_off; void* p_hop_v;
  void* p_c; void* p_len; void* p_contr; void* p_rule; void* p_stale; void* p_part;
  const int32_t stale_at_load = 1;
  const Part parts[] = {
      {ev.data(), 8 * (size_t)E, &p_edge_v}, {enbr.data(), 16 * (size_t)E, &p_nbr},
      {eopp.data(), 8 * (size_t)E, &p_opp}, {etri.data(), 8 * (size_t)E, &p_etri},
      {tri4.data(), 16 * (size_t)T, &p_tri}, {tedge4.data(), 16 * (size_t)T, &p_tedge},
      {adj_off.data(), 4 * (size_t)(V + 1), &p_adj_off}, {adj.data(), 16 * (size_t)E, &p_adj},
      {vtri_off.data(), 4 * (size_t)(V + 1), &p_vtri_off}, {vtri.data(), 4 * (size_t)n3, &p_vtri},
      {vk.data(), 8 * (size_t)V, &p_vk}, {pv.data(), 4 * pv.size(), &p_prim},
      {vold.data(), 4 * (size_t)V, &p_vold}, {vnew.data(), 4 * (size_t)V, &p_vnew},
      {eperm.data(), 4 * (size_t)E, &p_eperm}, {nullptr, 16 * (size_t)V, &p_xyi},
      {hop_off.data(), 4 * (size_t)(E + 1), &p_hop_off}, {hop_v.data(), 4 * hop_v.size(), &p_hop_v},
      {nullptr, 8 * (size_t)E, &p_c}, {nullptr, 8 * (size_t)E, &p_len},
      {nullptr, (size_t)E, &p_contr}, {nullptr, (size_t)E, &p_rule},
      {&stale_at_load, sizeof(int32_t), &p_stale},
      {nullptr, 8 * 3 * (size_t)ccsp::kMaxBlocks, &p_part}};
  size_t total = 0;
  for (const Part& pt : parts) total += (pt.bytes + 255) & ~size_t(255);
  he = hipMalloc(&m->mem, total);
  if (he != hipSuccess) {
    delete m;
    return fail(CCSP_E_OOM, "mesh_load: device allocation of " + std::to_string(total) +
                                " bytes failed");
  }
  size_t off = 0;
  for (const Part& pt : parts) {
    *pt.dst = (char*)m->mem + off;
    if (pt.src) {
      he = hipMemcpy(*pt.dst, pt.src, pt.bytes, hipMemcpyHostToDevice);
      if (he != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return hip_fail(he, "mesh_load: hipMemcpy");
      }
    }
    off += (pt.bytes + 255) & ~size_t(255);
  }
  d.edge_v = (const int2*)p_edge_v;
  d.edge_nbr = (const int4*)p_nbr;
  d.edge_opp = (const int2*)p_opp;
  d.edge_tri = (const int2*)p_etri;
  d.tri = (const int4*)p_tri;
  d.tri_edge = (const int4*)p_tedge;
  d.adj_off = (const int32_t*)p_adj_off;
  d.adj = (const int2*)p_adj;
  d.vtri_off = (const int32_t*)p_vtri_off;
  d.vtri = (const int32_t*)p_vtri;
  d.vk = (const int2*)p_vk;
  d.prim_v = (const int2*)p_prim;
  d.hop_off = (const int32_t*)p_hop_off;
  d.hop_v = (const int32_t*)p_hop_v;
  d.vold = (const int32_t*)p_vold;
  d.vnew = (const int32_t*)p_vnew;
  d.eperm = (const int32_t*)p_eperm;
  d.xyi = (double2*)p_xyi;
  d.c = (double*)p_c;
  d.len = (double*)p_len;
  d.contr = (uint8_t*)p_contr;
  d.rule = (uint8_t*)p_rule;
  d.stale = (int32_t*)p_stale;
  d.partial = (double*)p_part;
  m->edge_v = std::move(edge_can);
  *out = m;
  return CCSP_OK;
}

int mesh_info(const MovableMesh* mesh, int64_t* n_edges, int32_t* edge_v) {
  if (!mesh || !n_edges) return fail(CCSP_E_ARG, "mesh_info: null argument");
  *n_edges = mesh->d.ne;
  if (edge_v) std::memcpy(edge_v, mesh->edge_v.data(), sizeof(int32_t) * mesh->edge_v.size());
  return CCSP_OK;
}

int objective_eval(MovableMesh* mesh, const double* xy, const ObjectiveParams* params, double* out,
                   uint8_t* contractible, double* weight, void* stream) {
  if (!mesh || !xy || !out) return fail(CCSP_E_ARG, "objective_eval: null argument");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)out & 7) != 0 || ((uintptr_t)weight & 7) != 0)
    return fail(CCSP_E_ARG, "objective_eval: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "objective_eval: invalid parameters");
  if (int r = check_device(mesh)) return r;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  const int n1 = grid_for(d.ne), n2 = grid_for(std::max(d.ne, d.nt));
  stage_edges(d, p, xy, s);
  hipLaunchKernelGGL(ccsp::terms_pass, dim3(n2), dim3(ccsp::kThreads), 0, s, d, p,
                     d.partial + n1, d.partial + n1 + n2, contractible, weight);
  hipLaunchKernelGGL(ccsp::finish_sums, dim3(1), dim3(ccsp::kThreads), 0, s, d.partial, n1, n2, p,
                     out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "objective_eval: launch");
}

}  // extern "C"

namespace {

// The joint moves' device workspace, kept by the mesh: the terms before the move (te, ts per
// edge, ta per triangle), the vertex marks, the partial sums, the result and the flags, then k
// new positions. Grown (after synchronising s) when k exceeds every earlier call's.
struct JointBuf {
  double *te, *ts, *ta, *part, *out;
  uint32_t* mark;
  int* flags;
  double2* q;
};

int joint_buffers(MovableMesh* mesh, int64_t k, hipStream_t s, JointBuf* jb) {
  const ccsp::MeshDev& d = mesh->d;
  const int T = ccsp::kThreads;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t o_ts = al(8 * (size_t)d.ne), o_ta = o_ts + al(8 * (size_t)d.ne);
  const size_t o_mark = o_ta + al(8 * (size_t)d.nt), o_part = o_mark + al(4 * (size_t)d.nv);
  const size_t o_out = o_part + al(8 * 3 * (size_t)ccsp::kMaxBlocks), o_flags = o_out + 256;
  const size_t o_q = o_flags + 256, need = o_q + al(16 * (size_t)k);
  if (need > mesh->joint_bytes) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "joint moves: synchronise");
    if (mesh->joint_ws) (void)hipFree(mesh->joint_ws);
    mesh->joint_ws = nullptr;
    mesh->joint_bytes = 0;
    if (hipMalloc(&mesh->joint_ws, need) != hipSuccess) {
      (void)hipGetLastError();
      mesh->joint_ws = nullptr;
      return fail(CCSP_E_OOM, "joint moves: device allocation failed");
    }
    mesh->joint_bytes = need;
    mesh->joint_epoch = 0;
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((unsigned)((d.nv + T - 1) / T)), dim3(T), 0, s,
                       (int32_t*)((char*)mesh->joint_ws + o_mark), (int64_t)d.nv, 0);
  }
  char* w = (char*)mesh->joint_ws;
  jb->te = (double*)w;
  jb->ts = (double*)(w + o_ts);
  jb->ta = (double*)(w + o_ta);
  jb->mark = (uint32_t*)(w + o_mark);
  jb->part = (double*)(w + o_part);
  jb->out = (double*)(w + o_out);
  jb->flags = (int*)(w + o_flags);
  jb->q = (double2*)(w + o_q);
  return CCSP_OK;
}

}  // namespace

extern "C" {

int anneal_joint(MovableMesh* mesh, double* xy, const ObjectiveParams* params,
                 double temperature, double lambda, const int32_t* vid, int64_t k,
                 const double* xi, double u, double* delta_out, int32_t* status_out,
                 void* stream) {
  if (!mesh || !xy || !delta_out || !status_out || (k > 0 && (!vid || !xi)))
    return fail(CCSP_E_ARG, "anneal_joint: null argument");
  if (k < 1 || k >= (int64_t(1) << 31)) return fail(CCSP_E_ARG, "anneal_joint: bad vertex count");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)xi & 15) != 0 || ((uintptr_t)vid & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_joint: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_joint: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_joint: temperature must be finite and >= 0");
  if (!(lambda >= 0) || !std::isfinite(lambda))
    return fail(CCSP_E_ARG, "anneal_joint: lambda must be finite and >= 0");
  if (int r = check_device(mesh)) return r;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  const int T = ccsp::kThreads;
  const int nb = grid_for(std::max(d.ne, d.nt));
  JointBuf jb;
  if (int r = joint_buffers(mesh, k, s, &jb)) return r;
  double *te = jb.te, *ts = jb.ts, *ta = jb.ta, *part = jb.part, *out = jb.out;
  uint32_t* mark = jb.mark;
  int* flags = jb.flags;
  auto* qnew = jb.q;
  if (++mesh->joint_epoch == 0) {  // marks hold epochs: after a wrap, clear them
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((unsigned)((d.nv + T - 1) / T)), dim3(T), 0, s,
                       (int32_t*)mark, (int64_t)d.nv, 0);
    mesh->joint_epoch = 1;
  }
  hipError_t e;
  const unsigned kb = (unsigned)((k + T - 1) / T);
  stage_edges(d, p, xy, s);
  hipLaunchKernelGGL(ccsp::fill_i32, dim3(1), dim3(T), 0, s, (int32_t*)flags, (int64_t)1, 0);
  hipLaunchKernelGGL(ccsp::joint_terms, dim3(nb), dim3(T), 0, s, d, p, te, ts, ta);
  hipLaunchKernelGGL(ccsp::joint_prepare, dim3(kb), dim3(T), 0, s, d, lambda, vid,
                     (const double2*)xi, k, mesh->joint_epoch, mark, qnew, flags);
  hipLaunchKernelGGL(ccsp::joint_apply, dim3(kb), dim3(T), 0, s, d, vid, qnew, k, flags);
  hipLaunchKernelGGL(ccsp::joint_check, dim3(kb), dim3(T), 0, s, d, vid, k, flags);
  hipLaunchKernelGGL(ccsp::edge_state, dim3(grid_for(d.ne)), dim3(T), 0, s, d, p, d.partial);
  hipLaunchKernelGGL(ccsp::joint_diff, dim3(nb), dim3(T), 0, s, d, p, te, ts, ta, part);
  hipLaunchKernelGGL(ccsp::joint_finish, dim3(1), dim3(T), 0, s, part, nb, p, out);
  double hout[4];
  int hflags = 0;
  e = hipMemcpyAsync(hout, out, sizeof hout, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint");
  *delta_out = __builtin_huge_val();
  if (hflags & ccsp::kJointBad) {
    *status_out = CCSP_MOVE_BAD;
  } else if (hflags & ccsp::kJointFolds) {
    *status_out = CCSP_MOVE_FOLDS;
  } else {
    const double df = hout[0];
    *delta_out = df;
    if (df <= 0.0 || u < std::exp(-df / temperature)) {
      *status_out = CCSP_MOVE_OK;
      hipLaunchKernelGGL(ccsp::joint_commit, dim3(kb), dim3(T), 0, s, vid, qnew, k,
                         (double2*)xy);
    } else {
      *status_out = CCSP_MOVE_REJECTED;
    }
  }
  e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_joint: launch");
}

int anneal_joint_groups(MovableMesh* mesh, double* xy, const ObjectiveParams* params,
                        double temperature, double lambda, const int32_t* centres, int64_t n,
                        const double* draws, double u, double* delta_out, int32_t* status_out,
                        void* stream) {
  if (!mesh || !xy || !delta_out || !status_out || (n > 0 && (!centres || !draws)))
    return fail(CCSP_E_ARG, "anneal_joint_groups: null argument");
  if (n < 1 || n >= (int64_t(1) << 26))
    return fail(CCSP_E_ARG, "anneal_joint_groups: bad centre count");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)draws & 15) != 0 || ((uintptr_t)centres & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_joint_groups: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_joint_groups: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_joint_groups: temperature must be finite and >= 0");
  if (!(lambda >= 0) || !std::isfinite(lambda))
    return fail(CCSP_E_ARG, "anneal_joint_groups: lambda must be finite and >= 0");
  if (int r = check_device(mesh)) return r;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  const int T = ccsp::kThreads;
  const int N = (int)n;
  const int nb = grid_for(std::max(d.ne, d.nt));
  JointBuf jb;
  if (int r = joint_buffers(mesh, 1, s, &jb)) return r;
  stage_edges(d, p, xy, s);
  hipLaunchKernelGGL(ccsp::joint_terms, dim3(nb), dim3(T), 0, s, d, p, jb.te, jb.ts, jb.ta);
  // the query grid of the positions (as for anneal_group)
  GroupScratch gs;
  const int nbox = grid_for(d.nv);
  double* box = nullptr;
  hipError_t e = gs.get(&box, 4 * (size_t)nbox + 4);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_joint_groups: scratch allocation failed");
  hipLaunchKernelGGL(ccsp::bbox_kernel, dim3(nbox), dim3(T), 0, s, d, nullptr, 0, box + 4);
  hipLaunchKernelGGL(ccsp::bbox_kernel, dim3(1), dim3(T), 0, s, d, box + 4, nbox, box);
  double hb[4];
  e = hipMemcpyAsync(hb, box, sizeof hb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: bounding box");
  const double ext = std::max(hb[2] - hb[0], hb[3] - hb[1]);
  double h = std::max(5.0 * p.eps, ext / 1024.0);
  if (!(h > 0) || !std::isfinite(h)) h = 1.0;
  ccsp::VGrid g{};
  g.x0 = std::isfinite(hb[0]) ? hb[0] : 0.0;
  g.y0 = std::isfinite(hb[1]) ? hb[1] : 0.0;
  g.inv = 1.0 / h;
  g.gx = (int)std::min(1024.0, std::max(1.0, std::floor((hb[2] - g.x0) * g.inv) + 1.0));
  g.gy = (int)std::min(1024.0, std::max(1.0, std::floor((hb[3] - g.y0) * g.inv) + 1.0));
  if (!(g.gx >= 1)) g.gx = 1;
  if (!(g.gy >= 1)) g.gy = 1;
  const int ncells = g.gx * g.gy;
  int32_t *gcen = nullptr, *cnt = nullptr, *off = nullptr, *start = nullptr, *cursor = nullptr;
  int32_t *vert = nullptr, *rnd = nullptr, *st = nullptr, *mem_n = nullptr;
  uint32_t* sums = nullptr;
  uint8_t* done = nullptr;
  double* dl = nullptr;
  double2* disp = nullptr;
  e = gs.get(&gcen, N);
  if (e == hipSuccess) e = gs.get(&cnt, (size_t)N + 1);
  if (e == hipSuccess) e = gs.get(&off, (size_t)N + 1);
  if (e == hipSuccess) e = gs.get(&start, (size_t)ncells + 1);
  if (e == hipSuccess) e = gs.get(&cursor, (size_t)ncells + 1);
  if (e == hipSuccess) e = gs.get(&vert, d.nv);
  if (e == hipSuccess) e = gs.get(&done, N);
  if (e == hipSuccess) e = gs.get(&disp, N);
  if (e == hipSuccess) e = gs.get(&rnd, N);
  if (e == hipSuccess) e = gs.get(&st, N);
  if (e == hipSuccess) e = gs.get(&mem_n, N);
  if (e == hipSuccess) e = gs.get(&dl, N);
  if (e == hipSuccess)
    e = gs.get(&sums, ccsp::exclusive_scan_bytes(std::max<int64_t>(N, ncells) + 1) / 4);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_joint_groups: scratch allocation failed");
  g.start = start;
  g.vert = vert;
  hipLaunchKernelGGL(ccsp::fill_i32, dim3((ncells + T) / T), dim3(T), 0, s, cursor,
                     (int64_t)ncells + 1, 0);
  hipLaunchKernelGGL(ccsp::vgrid_count, dim3((d.nv + T - 1) / T), dim3(T), 0, s, d, g, cursor);
  e = ccsp::launch_exclusive_scan((const uint32_t*)cursor, (uint32_t*)start, ncells + 1, sums, s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: grid scan");
  hipLaunchKernelGGL(ccsp::fill_i32, dim3((ncells + T) / T), dim3(T), 0, s, cursor,
                     (int64_t)ncells + 1, 0);
  hipLaunchKernelGGL(ccsp::vgrid_fill, dim3((d.nv + T - 1) / T), dim3(T), 0, s, d, g, cursor,
                     vert);
  // centres; a centre that is not a movable vertex makes the whole move BAD
  const unsigned gb = (unsigned)((N + T - 1) / T);
  hipLaunchKernelGGL(ccsp::group_setup, dim3(gb), dim3(T), 0, s, d, centres, N, gcen, done, dl,
                     st, mem_n, rnd);
  std::vector<uint8_t> hd(N);
  e = hipMemcpyAsync(hd.data(), done, N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: setup");
  *delta_out = __builtin_huge_val();
  for (uint8_t x : hd)
    if (x) {
      *status_out = CCSP_MOVE_BAD;
      return CCSP_OK;
    }
  // the groups, their members, areas and displacements at the positions before the move
  hipLaunchKernelGGL(ccsp::fill_i32, dim3((N + T) / T), dim3(T), 0, s, cnt, (int64_t)N + 1, 0);
  hipLaunchKernelGGL(ccsp::group_count, dim3(gb), dim3(T), 0, s, d, g, p, gcen,
                     (const double2*)draws, done, N, cnt);
  e = ccsp::launch_exclusive_scan((const uint32_t*)cnt, (uint32_t*)off, N + 1, sums, s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: member scan");
  int32_t total = 0;
  e = hipMemcpyAsync(&total, off + N, sizeof total, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: member count");
  int32_t *mem = nullptr, *key = nullptr, *tmpm = nullptr, *tmpk = nullptr, *owner = nullptr;
  int32_t* vint = nullptr;
  uint64_t* first = nullptr;
  double2* qlist = nullptr;
  e = gs.get(&mem, (size_t)total);
  if (e == hipSuccess) e = gs.get(&key, (size_t)total);
  if (e == hipSuccess) e = gs.get(&tmpm, (size_t)total);
  if (e == hipSuccess) e = gs.get(&tmpk, (size_t)total);
  if (e == hipSuccess) e = gs.get(&first, (size_t)total);
  if (e == hipSuccess) e = gs.get(&vint, (size_t)total);
  if (e == hipSuccess) e = gs.get(&qlist, (size_t)total);
  if (e == hipSuccess) e = gs.get(&owner, d.nv);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_joint_groups: member buffer allocation failed");
  const unsigned wb = (unsigned)((N + T / 64 - 1) / (T / 64));  // one wave per group
  hipLaunchKernelGGL(ccsp::group_claim, dim3(wb), dim3(T), 0, s, d, g, g, p, lambda, gcen,
                     (const double2*)draws, done, N, off, cnt, mem, key, tmpm, tmpk, first, disp,
                     (uint32_t*)nullptr, (uint32_t*)nullptr);
  hipLaunchKernelGGL(ccsp::fill_i32, dim3((d.nv + T - 1) / T), dim3(T), 0, s, owner,
                     (int64_t)d.nv, INT32_MAX);
  hipLaunchKernelGGL(ccsp::jgroup_owner, dim3(wb), dim3(T), 0, s, off, cnt, mem, N, owner);
  hipLaunchKernelGGL(ccsp::jgroup_prepare, dim3(wb), dim3(T), 0, s, d, off, cnt, mem, disp,
                     owner, N, vint, qlist);
  // the move, its validity and its change of f
  const unsigned kb = (unsigned)((total + T - 1) / T);
  hipLaunchKernelGGL(ccsp::fill_i32, dim3(1), dim3(T), 0, s, (int32_t*)jb.flags, (int64_t)1, 0);
  if (total > 0) {
    hipLaunchKernelGGL(ccsp::jgroup_apply, dim3(kb), dim3(T), 0, s, d, vint, qlist,
                       (int64_t)total);
    hipLaunchKernelGGL(ccsp::jgroup_check, dim3(kb), dim3(T), 0, s, d, vint, (int64_t)total,
                       jb.flags);
  }
  hipLaunchKernelGGL(ccsp::edge_state, dim3(grid_for(d.ne)), dim3(T), 0, s, d, p, d.partial);
  hipLaunchKernelGGL(ccsp::joint_diff, dim3(nb), dim3(T), 0, s, d, p, jb.te, jb.ts, jb.ta,
                     jb.part);
  hipLaunchKernelGGL(ccsp::joint_finish, dim3(1), dim3(T), 0, s, jb.part, nb, p, jb.out);
  double hout[4];
  int hflags = 0;
  e = hipMemcpyAsync(hout, jb.out, sizeof hout, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflags, jb.flags, sizeof hflags, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups");
  if (hflags & ccsp::kJointFolds) {
    *status_out = CCSP_MOVE_FOLDS;
  } else {
    const double df = hout[0];
    *delta_out = df;
    if (df <= 0.0 || u < std::exp(-df / temperature)) {
      *status_out = CCSP_MOVE_OK;
      if (total > 0)
        hipLaunchKernelGGL(ccsp::jgroup_commit, dim3(kb), dim3(T), 0, s, d, vint, qlist,
                           (int64_t)total, (double2*)xy);
      e = hipStreamSynchronize(s);  // the group scratch is freed on return
      if (e != hipSuccess) return hip_fail(e, "anneal_joint_groups: commit");
    } else {
      *status_out = CCSP_MOVE_REJECTED;
    }
  }
  e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_joint_groups: launch");
}

int objective_delta(MovableMesh* mesh, const double* xy, const ObjectiveParams* params,
                    const int32_t* vid, const double* q_xy, int64_t k, double* delta,
                    int32_t* status, void* stream) {
  if (!mesh || !xy || k < 0) return fail(CCSP_E_ARG, "objective_delta: null argument or k < 0");
  if (k > 0 && (!vid || !q_xy || !delta || !status))
    return fail(CCSP_E_ARG, "objective_delta: null argument");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)q_xy & 15) != 0 || ((uintptr_t)delta & 7) != 0 ||
      ((uintptr_t)vid & 3) != 0 || ((uintptr_t)status & 3) != 0)
    return fail(CCSP_E_ARG, "objective_delta: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "objective_delta: invalid parameters");
  if (k >= (int64_t(1) << 40)) return fail(CCSP_E_ARG, "objective_delta: too many moves");
  if (int r = check_device(mesh)) return r;
  if (k == 0) return CCSP_OK;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  stage_edges(d, p, xy, s);
  const int64_t blocks = (k + ccsp::kThreads - 1) / ccsp::kThreads;
  const uint32_t* order = nullptr;
  if (k >= kSortMoves && k < (int64_t(1) << 31)) {
    if (int r = sort_moves(mesh, vid, k, s, &order)) return r;
  }
  if (k < (int64_t(1) << 31))
    hipLaunchKernelGGL(ccsp::move_delta_wave, dim3((unsigned)k), dim3(ccsp::kWaveThreads), 0, s,
                       d, p, vid, (const double2*)q_xy, k, order, delta, status);
  else
    hipLaunchKernelGGL(ccsp::move_delta, dim3((unsigned)blocks), dim3(ccsp::kThreads), 0, s, d, p,
                       vid, (const double2*)q_xy, k, order, delta, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "objective_delta: launch");
}

// Greedy colouring of the movable vertices over balls of `radius` edges along paths that do not
// pass through hubs (see is_hub: what a move reads or writes at a hub lies at the moved vertex's
// own place in its fan, which the fan's ring edges join): members of a class are more than
// `radius` edges apart along such paths. A box corner's fan would otherwise put all of its
// hundreds of vertices in different classes.
int build_classes(MovableMesh* mesh, int radius, std::vector<int64_t>& class_off,
                  std::vector<int32_t>& class_v, int32_t*& class_dev) {
  if (class_off.empty()) {
    if (int r = check_device(mesh)) return r;
    const ccsp::MeshDev& d = mesh->d;
    const int64_t V = d.nv;
    std::vector<int32_t> adj_off(V + 1), adj(4 * (int64_t)d.ne), vk(2 * V), vold(V);
    hipError_t e = hipMemcpy(adj_off.data(), d.adj_off, 4 * (V + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(adj.data(), d.adj, 16 * (size_t)d.ne, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(vk.data(), d.vk, 8 * V, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(vold.data(), d.vold, 4 * V, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "mesh_classes: hipMemcpy");
    // each movable vertex takes the smallest class not used by a movable vertex within radius
    std::vector<int32_t> colour(V, -1), stamp(V, -1), ball, used;
    int32_t n = 0;
    for (int64_t v = 0; v < V; ++v) {
      if (vk[2 * v] == CCSP_VERTEX_ORIGINAL) continue;
      ball.assign(1, (int32_t)v);
      stamp[v] = (int32_t)v;
      size_t lo = 0;
      for (int r = 0; r < radius; ++r) {
        const size_t hi = ball.size();
        for (size_t j = lo; j < hi; ++j) {
          const int32_t u = ball[j];
          if (vk[2 * u] == CCSP_VERTEX_ORIGINAL && adj_off[u + 1] - adj_off[u] > ccsp::kHubDegree)
            continue;  // a hub: in the ball, not passed through
          for (int32_t k = adj_off[u]; k < adj_off[u + 1]; ++k) {
            const int32_t w = adj[2 * k];
            if (stamp[w] != (int32_t)v) {
              stamp[w] = (int32_t)v;
              ball.push_back(w);
            }
          }
        }
        lo = hi;
      }
      used.assign(n + 1, 0);
      for (int32_t w : ball)
        if (colour[w] >= 0) used[colour[w]] = 1;
      int32_t c = 0;
      while (used[c]) ++c;
      colour[v] = c;
      n = std::max(n, c + 1);
    }
    std::vector<int64_t> off(n + 1, 0);
    for (int64_t v = 0; v < V; ++v)
      if (colour[v] >= 0) ++off[colour[v] + 1];
    for (int32_t c = 0; c < n; ++c) off[c + 1] += off[c];
    std::vector<int32_t> cv(off[n]), ci(off[n]);
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (int64_t v = 0; v < V; ++v)
      if (colour[v] >= 0) {
        ci[fill[colour[v]]] = (int32_t)v;
        cv[fill[colour[v]]++] = vold[v];
      }
    if (n == 0) off.assign(1, 0);
    if (!ci.empty()) {
      e = hipMalloc(&class_dev, 4 * ci.size());
      if (e != hipSuccess) return fail(CCSP_E_OOM, "mesh_classes: device allocation failed");
      e = hipMemcpy(class_dev, ci.data(), 4 * ci.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipFree(class_dev);
        class_dev = nullptr;
        return hip_fail(e, "mesh_classes: hipMemcpy");
      }
    }
    class_off = std::move(off);
    class_v = std::move(cv);
  }
  return CCSP_OK;
}

int ensure_classes(MovableMesh* mesh) {
  return build_classes(mesh, 4, mesh->class_off, mesh->class_v, mesh->class_dev);
}


int mesh_classes(MovableMesh* mesh, int32_t* n_classes, int64_t* class_off, int32_t* class_v) {
  if (!mesh || !n_classes) return fail(CCSP_E_ARG, "mesh_classes: null argument");
  if (int r = ensure_classes(mesh)) return r;
  *n_classes = (int32_t)mesh->class_off.size() - 1;
  if (class_off) std::memcpy(class_off, mesh->class_off.data(), 8 * mesh->class_off.size());
  if (class_v) std::memcpy(class_v, mesh->class_v.data(), 4 * mesh->class_v.size());
  return CCSP_OK;
}

int anneal_group(MovableMesh* mesh, double* xy, const ObjectiveParams* params, double temperature,
                 double lambda, const int32_t* centres, int64_t n, const double* draws,
                 const double* u, double* delta, int32_t* status, int32_t* members,
                 int32_t* round, void* stream) {
  if (!mesh || !xy || (n > 0 && (!centres || !draws || !u || !delta || !status || !members ||
                                 !round)))
    return fail(CCSP_E_ARG, "anneal_group: null argument");
  if (n < 0 || n >= (int64_t(1) << 30)) return fail(CCSP_E_ARG, "anneal_group: bad centre count");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)draws & 15) != 0 || ((uintptr_t)u & 7) != 0 ||
      ((uintptr_t)delta & 7) != 0 || ((uintptr_t)status & 3) != 0 ||
      ((uintptr_t)members & 3) != 0 || ((uintptr_t)round & 3) != 0 ||
      ((uintptr_t)centres & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_group: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_group: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_group: temperature must be finite and >= 0");
  if (!(lambda >= 0) || !std::isfinite(lambda))
    return fail(CCSP_E_ARG, "anneal_group: lambda must be finite and >= 0");
  if (int r = check_device(mesh)) return r;
  if (n == 0) return CCSP_OK;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  const int N = (int)n;
  const int T = ccsp::kThreads;
  const unsigned gb = (unsigned)((N + T - 1) / T), vb = (unsigned)((d.nv + T - 1) / T);
  stage_edges(d, p, xy, s);
  GroupScratch gs;
  double* box = nullptr;
  unsigned long long* applied = nullptr;
  const int nbox = grid_for(d.nv);  // workgroups of the bounding-box pass
  hipError_t e = gs.get(&box, 4 * (size_t)nbox + 4);
  if (e == hipSuccess) e = gs.get(&applied, 1);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_group: scratch allocation failed");
  hipLaunchKernelGGL(ccsp::bbox_kernel, dim3(nbox), dim3(T), 0, s, d, nullptr, 0, box + 4);
  hipLaunchKernelGGL(ccsp::bbox_kernel, dim3(1), dim3(T), 0, s, d, box + 4, nbox, box);
  double hb[4];
  e = hipMemcpyAsync(hb, box, sizeof hb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_group: bounding box");
  // grid cells of side at least 5 eps (the largest query radius), at most 1024 per side
  const double ext = std::max(hb[2] - hb[0], hb[3] - hb[1]);
  double h = std::max(5.0 * p.eps, ext / 1024.0);
  if (!(h > 0) || !std::isfinite(h)) h = 1.0;
  ccsp::VGrid g{};
  g.x0 = std::isfinite(hb[0]) ? hb[0] : 0.0;
  g.y0 = std::isfinite(hb[1]) ? hb[1] : 0.0;
  g.inv = 1.0 / h;
  g.gx = (int)std::min(1024.0, std::max(1.0, std::floor((hb[2] - g.x0) * g.inv) + 1.0));
  g.gy = (int)std::min(1024.0, std::max(1.0, std::floor((hb[3] - g.y0) * g.inv) + 1.0));
  if (!(g.gx >= 1)) g.gx = 1;
  if (!(g.gy >= 1)) g.gy = 1;
  const int ncells = g.gx * g.gy;
  // the claims' grid: cells a quarter of the query grid's side, at most 4096 per side (groups
  // whose discs only share a coarse cell then do not conflict)
  ccsp::VGrid gc = g;
  gc.inv = 4.0 * g.inv;
  gc.gx = (int)std::min(4096.0, std::max(1.0, std::floor((hb[2] - gc.x0) * gc.inv) + 1.0));
  gc.gy = (int)std::min(4096.0, std::max(1.0, std::floor((hb[3] - gc.y0) * gc.inv) + 1.0));
  if (!(gc.gx >= 1)) gc.gx = 1;
  if (!(gc.gy >= 1)) gc.gy = 1;
  const int nclaim = gc.gx * gc.gy;
  int32_t *gcen = nullptr, *cnt = nullptr, *off = nullptr, *start = nullptr, *cursor = nullptr;
  int32_t *vert = nullptr, *mem = nullptr, *key = nullptr, *tmpm = nullptr, *tmpk = nullptr;
  uint64_t* first = nullptr;
  uint32_t *own_v = nullptr, *own_c = nullptr;
  uint8_t *done = nullptr, *won = nullptr;
  double2* disp = nullptr;
  e = gs.get(&gcen, N);
  if (e == hipSuccess) e = gs.get(&cnt, (size_t)N + 1);
  if (e == hipSuccess) e = gs.get(&off, (size_t)N + 1);
  if (e == hipSuccess) e = gs.get(&start, (size_t)ncells + 1);
  if (e == hipSuccess) e = gs.get(&cursor, (size_t)ncells + 1);
  if (e == hipSuccess) e = gs.get(&vert, d.nv);
  if (e == hipSuccess) e = gs.get(&own_v, d.nv);
  if (e == hipSuccess) e = gs.get(&own_c, nclaim);
  if (e == hipSuccess) e = gs.get(&done, N);
  if (e == hipSuccess) e = gs.get(&won, N);
  if (e == hipSuccess) e = gs.get(&disp, N);
  size_t scan_bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, cnt, off,
                                         std::max(N, ncells) + 1);
  void* scan_tmp = nullptr;
  if (e == hipSuccess) e = gs.get(reinterpret_cast<unsigned char**>(&scan_tmp), scan_bytes);
  if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_group: scratch allocation failed");
  size_t mem_cap = 0;
  g.start = start;
  g.vert = vert;
  hipLaunchKernelGGL(ccsp::group_setup, dim3(gb), dim3(T), 0, s, d, centres, N, gcen, done, delta,
                     status, members, round);
  std::vector<uint8_t> hd(N);
  e = hipMemcpyAsync(hd.data(), done, N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "anneal_group: setup");
  int64_t remaining = 0;
  for (uint8_t x : hd) remaining += x ? 0 : 1;
  for (int rnd = 0; remaining > 0; ++rnd) {
    if (rnd > N) return fail(CCSP_E_HIP, "anneal_group: no group could move in a round");
    // the grid of the current positions
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((ncells + T) / T), dim3(T), 0, s, cursor,
                       (int64_t)ncells + 1, 0);
    hipLaunchKernelGGL(ccsp::vgrid_count, dim3(vb), dim3(T), 0, s, d, g, cursor);
    e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, cursor, start, ncells + 1, s);
    if (e != hipSuccess) return hip_fail(e, "anneal_group: grid scan");
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((ncells + T) / T), dim3(T), 0, s, cursor,
                       (int64_t)ncells + 1, 0);
    hipLaunchKernelGGL(ccsp::vgrid_fill, dim3(vb), dim3(T), 0, s, d, g, cursor, vert);
    // group sizes, their offsets, and room for the members
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((N + T) / T), dim3(T), 0, s, cnt, (int64_t)N + 1, 0);
    hipLaunchKernelGGL(ccsp::group_count, dim3(gb), dim3(T), 0, s, d, g, p, gcen,
                       (const double2*)draws, done, N, cnt);
    e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, cnt, off, N + 1, s);
    if (e != hipSuccess) return hip_fail(e, "anneal_group: member scan");
    int32_t total = 0;
    e = hipMemcpyAsync(&total, off + N, sizeof total, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "anneal_group: member count");
    if ((size_t)total > mem_cap) {
      mem_cap = std::max<size_t>((size_t)total, 2 * mem_cap);
      if (gs.get(&mem, mem_cap) != hipSuccess || gs.get(&key, mem_cap) != hipSuccess ||
          gs.get(&tmpm, mem_cap) != hipSuccess || gs.get(&tmpk, mem_cap) != hipSuccess ||
          gs.get(&first, mem_cap) != hipSuccess)
        return fail(CCSP_E_OOM, "anneal_group: member buffer allocation failed");
    }
    // claims, their check, and the moves of the groups holding all of theirs
    hipLaunchKernelGGL(ccsp::fill_i32, dim3(vb), dim3(T), 0, s, reinterpret_cast<int32_t*>(own_v),
                       (int64_t)d.nv, -1);
    hipLaunchKernelGGL(ccsp::fill_i32, dim3((nclaim + T - 1) / T), dim3(T), 0, s,
                       reinterpret_cast<int32_t*>(own_c), (int64_t)nclaim, -1);
    const unsigned wb = (unsigned)((N + T / 64 - 1) / (T / 64));  // one wave per group
    hipLaunchKernelGGL(ccsp::group_claim, dim3(wb), dim3(T), 0, s, d, g, gc, p, lambda, gcen,
                       (const double2*)draws, done, N, off, cnt, mem, key, tmpm, tmpk, first, disp,
                       own_v, own_c);
    hipLaunchKernelGGL(ccsp::group_check, dim3(wb), dim3(T), 0, s, d, gc, p, gcen,
                       (const double2*)draws, done, N, off, cnt, mem, disp, own_v, own_c, won);
    hipLaunchKernelGGL(ccsp::zero_counter, dim3(1), dim3(64), 0, s, applied);
    hipLaunchKernelGGL(ccsp::group_apply, dim3((unsigned)N), dim3(ccsp::kWaveThreads), 0, s, d, p,
                       temperature,
                       (double2*)xy, N, off, cnt, mem, disp, u, won, rnd, done, delta, status,
                       members, round, applied);
    unsigned long long got = 0;
    e = hipMemcpyAsync(&got, applied, sizeof got, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "anneal_group: round");
    if (got == 0) return fail(CCSP_E_HIP, "anneal_group: no group could move in a round");
    remaining -= (int64_t)got;
  }
  e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_group: launch");
}

int anneal_moves(MovableMesh* mesh, double* xy, const ObjectiveParams* params, double temperature,
                 const int32_t* vid, const double* disp, const double* u, int64_t k, double* delta,
                 int32_t* status, void* stream) {
  if (!mesh || !xy || k < 0) return fail(CCSP_E_ARG, "anneal_moves: null argument or k < 0");
  if (k > 0 && (!vid || !disp || !u || !delta || !status))
    return fail(CCSP_E_ARG, "anneal_moves: null argument");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)disp & 15) != 0 || ((uintptr_t)u & 7) != 0 ||
      ((uintptr_t)delta & 7) != 0 || ((uintptr_t)vid & 3) != 0 || ((uintptr_t)status & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_moves: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_moves: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_moves: temperature must be finite and >= 0");
  if (k >= (int64_t(1) << 40)) return fail(CCSP_E_ARG, "anneal_moves: too many moves");
  if (int r = check_device(mesh)) return r;
  if (k == 0) return CCSP_OK;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  stage_edges(d, p, xy, s);
  const int64_t blocks = (k + ccsp::kThreads - 1) / ccsp::kThreads;
  hipLaunchKernelGGL(ccsp::anneal_moves, dim3((unsigned)blocks), dim3(ccsp::kThreads), 0, s, d, p,
                     temperature, (double2*)xy, vid, (const double2*)disp, u, k, delta, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_moves: launch");
}

int anneal_sweep(MovableMesh* mesh, double* xy, const ObjectiveParams* params, double temperature,
                 const double* disp, const double* u, double* delta, int32_t* status,
                 void* stream) {
  if (!mesh || !xy || !disp || !u || !delta || !status)
    return fail(CCSP_E_ARG, "anneal_sweep: null argument");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)disp & 15) != 0 || ((uintptr_t)u & 7) != 0 ||
      ((uintptr_t)delta & 7) != 0 || ((uintptr_t)status & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_sweep: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_sweep: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_sweep: temperature must be finite and >= 0");
  if (int r = check_device(mesh)) return r;
  if (int r = ensure_classes(mesh)) return r;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  stage_edges(d, p, xy, s);
  const std::vector<int64_t>& off = mesh->class_off;
  for (size_t c = 0; c + 1 < off.size(); ++c) {
    const int n = (int)(off[c + 1] - off[c]);
    if (n == 0) continue;
    hipLaunchKernelGGL(ccsp::anneal_class, dim3((unsigned)n), dim3(ccsp::kWaveThreads), 0, s,
                       d, p, temperature, 0.0,
                       (int)CCSP_PROPOSE_DISPLACE, (double2*)xy, mesh->class_dev + off[c],
                       (const double2*)disp + off[c], u + off[c], n, delta + off[c],
                       status + off[c], (unsigned long long*)nullptr);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_sweep: launch");
}

int anneal_propose(MovableMesh* mesh, double* xy, const ObjectiveParams* params, double temperature,
                   int32_t kind, const double* draws, const double* u, double* delta,
                   int32_t* status, void* stream) {
  if (!mesh || !xy || !draws || !u || !delta || !status)
    return fail(CCSP_E_ARG, "anneal_propose: null argument");
  if (kind != CCSP_PROPOSE_RESAMPLE && kind != CCSP_PROPOSE_SWAP && kind != CCSP_PROPOSE_CONTRACT)
    return fail(CCSP_E_ARG, "anneal_propose: unknown proposal kind");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)draws & 15) != 0 || ((uintptr_t)u & 7) != 0 ||
      ((uintptr_t)delta & 7) != 0 || ((uintptr_t)status & 3) != 0)
    return fail(CCSP_E_ARG, "anneal_propose: misaligned buffer");
  if (!check_params(params)) return fail(CCSP_E_ARG, "anneal_propose: invalid parameters");
  if (!(temperature >= 0) || !std::isfinite(temperature))
    return fail(CCSP_E_ARG, "anneal_propose: temperature must be finite and >= 0");
  if (int r = check_device(mesh)) return r;
  if (int r = ensure_classes(mesh)) return r;
  const ccsp::MeshDev& d = mesh->d;
  const ccsp::Par p = to_par(params);
  hipStream_t s = (hipStream_t)stream;
  stage_edges(d, p, xy, s);
  const std::vector<int64_t>& off = mesh->class_off;
  for (size_t c = 0; c + 1 < off.size(); ++c) {
    const int n = (int)(off[c + 1] - off[c]);
    if (n == 0) continue;
    hipLaunchKernelGGL(ccsp::anneal_class, dim3((unsigned)n), dim3(ccsp::kWaveThreads), 0, s,
                       d, p, temperature, 0.0, (int)kind,
                       (double2*)xy, mesh->class_dev + off[c],
                       (const double2*)draws + 2 * off[c], u + off[c], n, delta + off[c],
                       status + off[c], (unsigned long long*)nullptr);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CCSP_OK : hip_fail(e, "anneal_propose: launch");
}

int anneal_schedule(MovableMesh* mesh, double* xy, const ObjectiveParams* params, int32_t n_sweeps,
                    const double* temperature, const double* eps, double lambda0, double target,
                    const double* xi, const double* u, double* lambda_out, int64_t* accepted_out,
                    void* stream) {
  if (!mesh || !xy || !params || n_sweeps < 0)
    return fail(CCSP_E_ARG, "anneal_schedule: null argument or n_sweeps < 0");
  if (n_sweeps > 0 && (!temperature || !eps || !xi || !u || !lambda_out || !accepted_out))
    return fail(CCSP_E_ARG, "anneal_schedule: null argument");
  if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)xi & 15) != 0 || ((uintptr_t)u & 7) != 0)
    return fail(CCSP_E_ARG, "anneal_schedule: misaligned buffer");
  if (!(lambda0 > 0) || !std::isfinite(lambda0) || !(target > 0) || !(target < 1))
    return fail(CCSP_E_ARG, "anneal_schedule: lambda0 must be > 0 and target in (0, 1)");
  for (int32_t k = 0; k < n_sweeps; ++k) {
    ObjectiveParams pk = *params;
    pk.eps = eps[k];
    if (!check_params(&pk)) return fail(CCSP_E_ARG, "anneal_schedule: invalid parameters");
    if (!(temperature[k] >= 0) || !std::isfinite(temperature[k]))
      return fail(CCSP_E_ARG, "anneal_schedule: temperatures must be finite and >= 0");
  }
  if (int r = check_device(mesh)) return r;
  if (int r = ensure_classes(mesh)) return r;
  const int64_t M = mesh->class_off.back();
  if (M == 0 || n_sweeps == 0) return CCSP_OK;
  const size_t need = 8 * (size_t)M + 4 * (size_t)M + 256;
  if (!mesh->sched) {
    hipError_t e = hipMalloc(&mesh->sched, need);
    if (e != hipSuccess) return fail(CCSP_E_OOM, "anneal_schedule: device allocation failed");
  }
  double* delta = (double*)mesh->sched;
  int32_t* status = (int32_t*)(delta + M);
  auto* counter = (unsigned long long*)((char*)mesh->sched + ((12 * (size_t)M + 255) & ~size_t(255)));
  const ccsp::MeshDev& d = mesh->d;
  hipStream_t s = (hipStream_t)stream;
  const std::vector<int64_t>& off = mesh->class_off;
  double lam = lambda0;
  for (int32_t k = 0; k < n_sweeps; ++k) {
    ObjectiveParams pk = *params;
    pk.eps = eps[k];
    const ccsp::Par p = to_par(&pk);
    stage_edges(d, p, xy, s);
    hipLaunchKernelGGL(ccsp::zero_counter, dim3(1), dim3(64), 0, s, counter);
    const double2* xk = (const double2*)xi + (size_t)k * M;
    const double* uk = u + (size_t)k * M;
    for (size_t c = 0; c + 1 < off.size(); ++c) {
      const int n = (int)(off[c + 1] - off[c]);
      if (n == 0) continue;
      hipLaunchKernelGGL(ccsp::anneal_class, dim3((unsigned)n), dim3(ccsp::kWaveThreads), 0,
                         s, d, p, temperature[k], lam,
                         (int)CCSP_PROPOSE_DISPLACE, (double2*)xy, mesh->class_dev + off[c],
                         xk + off[c], uk + off[c], n, delta + off[c], status + off[c], counter);
    }
    unsigned long long acc = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&acc, counter, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "anneal_schedule");
    lambda_out[k] = lam;
    accepted_out[k] = (int64_t)acc;
    // adaptive aggressiveness (Sec. 3.2): scale lambda by 1 + (acceptance - target), within [1/2, 2]
    const double a = (double)acc / (double)M;
    lam = lam * std::min(2.0, std::max(0.5, 1.0 + (a - target)));
  }
  return CCSP_OK;
}

void mesh_free(MovableMesh* mesh) {
  if (!mesh) return;
  if (mesh->sched) (void)hipFree(mesh->sched);
  if (mesh->order_ws) (void)hipFree(mesh->order_ws);
  if (mesh->joint_ws) (void)hipFree(mesh->joint_ws);
  if (mesh->class_dev) (void)hipFree(mesh->class_dev);
  if (mesh->mem) (void)hipFree(mesh->mem);
  delete mesh;
}

}  // extern "C"
