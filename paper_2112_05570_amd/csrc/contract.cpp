// Contraction of short edges: the step from the optimised fuzzy topology to a true topology
// (paper Sec. 3.4.1), the C-ABI mesh_contract of ccsp_objective.h. Sequential host code, as the
// paper's step is: each contraction changes the neighbourhood the next one is decided in.
//
// Passes: each lists the edges shorter than eps at its start in increasing (length, lower id,
// higher id) and tries each that is still an edge and still shorter; passes repeat until one
// contracts nothing. A contraction of (a, b) needs: the original geometry to allow it; the common
// neighbours of a and b to be exactly the vertices opposite the edge (otherwise the result would
// not be a triangulation); not both ends on the hull for an interior edge; no remaining triangle
// with all three vertices on one original edge (zero area in intent, whatever rounding makes of
// the constrained vertices' positions); and a position of the
// survivor at which every remaining triangle around it is strictly counter-clockwise (exact).
// The survivor is the vertex with fewer degrees of freedom (original over constrained over free),
// kept where it is; two vertices of one kind merge into the lower id at a + t (b - a), t tried as
// 1/2, 1/4, 3/4, 0, 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <tuple>
#include <vector>

#include "ccsp_objective.h"
#include "exact.hpp"
#include "walk.hpp"

namespace {

using ccsp::orient_exact;

int fail(int code, const char* msg) {
  ccsp::set_last_error(msg);
  return code;
}

// binary64 filter (error bound (3 + 16u) u of this evaluation, below 2^-51), then exact
int orient_pts(const double* a, const double* b, const double* c) {
  const double l = (b[0] - a[0]) * (c[1] - a[1]);
  const double r = (b[1] - a[1]) * (c[0] - a[0]);
  const double det = l - r, sum = std::fabs(l) + std::fabs(r);
  if (std::fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return orient_exact(a[0], a[1], b[0], b[1], c[0], c[1]);
}

struct Contractor {
  std::vector<std::array<int32_t, 3>> tri;
  std::vector<uint8_t> tri_alive;
  std::vector<std::vector<int32_t>> star;  // triangles of each vertex, unordered
  std::vector<int32_t> kind, line, merged_into;
  std::vector<std::array<int32_t, 2>> prim;
  std::vector<std::array<double, 2>> xy;

  double len(int a, int b) const {
    const double dx = xy[b][0] - xy[a][0], dy = xy[b][1] - xy[a][1];
    return std::sqrt(dx * dx + dy * dy);
  }

  bool kinds_allow(int a, int b) const {
    const int ka = kind[a], kb = kind[b];
    if (ka == CCSP_VERTEX_ORIGINAL && kb == CCSP_VERTEX_ORIGINAL) return false;
    if (ka == CCSP_VERTEX_ORIGINAL && kb == CCSP_VERTEX_CONSTRAINED)
      return prim[line[b]][0] == a || prim[line[b]][1] == a;
    if (kb == CCSP_VERTEX_ORIGINAL && ka == CCSP_VERTEX_CONSTRAINED)
      return prim[line[a]][0] == b || prim[line[a]][1] == b;
    if (ka == CCSP_VERTEX_CONSTRAINED && kb == CCSP_VERTEX_CONSTRAINED) return line[a] == line[b];
    return true;
  }

  // Neighbours of v, each with the number of v's triangles that hold it (sorted by id).
  std::vector<std::pair<int32_t, int>> neighbours(int v) const {
    std::vector<int32_t> w;
    for (int t : star[v])
      for (int x : tri[t])
        if (x != v) w.push_back(x);
    std::sort(w.begin(), w.end());
    std::vector<std::pair<int32_t, int>> out;
    for (size_t i = 0; i < w.size();) {
      size_t j = i;
      while (j < w.size() && w[j] == w[i]) ++j;
      out.push_back({w[i], (int)(j - i)});
      i = j;
    }
    return out;
  }

  bool on_hull(int v) const {
    for (const auto& p : neighbours(v))
      if (p.second == 1) return true;
    return false;
  }

  std::vector<int32_t> shared_triangles(int a, int b) const {
    std::vector<int32_t> s;
    for (int t : star[a])
      for (int x : tri[t])
        if (x == b) {
          s.push_back(t);
          break;
        }
    std::sort(s.begin(), s.end());
    return s;
  }

  bool on_edge(int v, int k) const {
    if (kind[v] == CCSP_VERTEX_CONSTRAINED) return line[v] == k;
    return kind[v] == CCSP_VERTEX_ORIGINAL && (prim[k][0] == v || prim[k][1] == v);
  }

  // Whether triangle t, with a and b read as s, would have all three vertices on one original edge.
  bool flat_on_original(int t, int a, int b, int s) const {
    int tv[3];
    for (int k = 0; k < 3; ++k) tv[k] = (tri[t][k] == a || tri[t][k] == b) ? s : tri[t][k];
    for (int k = 0; k < 3; ++k) {
      if (kind[tv[k]] != CCSP_VERTEX_CONSTRAINED) continue;
      const int ln = line[tv[k]];
      if (on_edge(tv[0], ln) && on_edge(tv[1], ln) && on_edge(tv[2], ln)) return true;
    }
    return false;
  }

  bool try_edge(int a, int b) {
    if (!kinds_allow(a, b)) return false;
    const std::vector<int32_t> shared = shared_triangles(a, b);
    std::vector<int32_t> opp;
    for (int t : shared)
      for (int x : tri[t])
        if (x != a && x != b) opp.push_back(x);
    std::sort(opp.begin(), opp.end());
    opp.erase(std::unique(opp.begin(), opp.end()), opp.end());
    // link condition: common neighbours are exactly the opposite vertices
    const auto na = neighbours(a), nb = neighbours(b);
    std::vector<int32_t> common;
    for (size_t i = 0, j = 0; i < na.size() && j < nb.size();) {
      if (na[i].first < nb[j].first) {
        ++i;
      } else if (nb[j].first < na[i].first) {
        ++j;
      } else {
        common.push_back(na[i].first);
        ++i;
        ++j;
      }
    }
    if (common != opp) return false;
    if (shared.size() == 2 && on_hull(a) && on_hull(b)) return false;
    int s, r;
    std::vector<std::array<double, 2>> cands;
    const bool a_fixed = kind[a] == CCSP_VERTEX_ORIGINAL ||
                         (kind[a] == CCSP_VERTEX_CONSTRAINED && kind[b] == CCSP_VERTEX_FREE);
    const bool b_fixed = kind[b] == CCSP_VERTEX_ORIGINAL ||
                         (kind[b] == CCSP_VERTEX_CONSTRAINED && kind[a] == CCSP_VERTEX_FREE);
    if (a_fixed) {
      s = a;
      r = b;
      cands.push_back(xy[a]);
    } else if (b_fixed) {
      s = b;
      r = a;
      cands.push_back(xy[b]);
    } else {
      s = a;
      r = b;
      const double ax = xy[a][0], ay = xy[a][1];
      const double dx = xy[b][0] - ax, dy = xy[b][1] - ay;
      for (double t : {0.5, 0.25, 0.75, 0.0, 1.0}) cands.push_back({ax + t * dx, ay + t * dy});
    }
    std::vector<int32_t> rest;
    for (int v : {a, b})
      for (int t : star[v])
        if (!std::binary_search(shared.begin(), shared.end(), t)) rest.push_back(t);
    std::sort(rest.begin(), rest.end());
    rest.erase(std::unique(rest.begin(), rest.end()), rest.end());
    for (int t : rest)
      if (flat_on_original(t, a, b, s)) return false;
    for (const auto& P : cands) {
      bool ok = true;
      for (int t : rest) {
        const double* p[3];
        for (int k = 0; k < 3; ++k) {
          const int x = tri[t][k];
          p[k] = (x == a || x == b) ? P.data() : xy[x].data();
        }
        if (orient_pts(p[0], p[1], p[2]) <= 0) {
          ok = false;
          break;
        }
      }
      if (!ok) continue;
      for (int t : shared) {
        tri_alive[t] = 0;
        for (int x : tri[t]) {
          auto& st = star[x];
          st.erase(std::remove(st.begin(), st.end(), t), st.end());
        }
      }
      for (int t : star[r]) {
        for (auto& x : tri[t])
          if (x == r) x = s;
        star[s].push_back(t);
      }
      star[r].clear();
      xy[s] = P;
      merged_into[r] = s;
      return true;
    }
    return false;
  }

  int64_t run(double eps) {
    int64_t total = 0;
    for (;;) {
      std::vector<std::tuple<double, int32_t, int32_t>> cand;
      for (size_t t = 0; t < tri.size(); ++t) {
        if (!tri_alive[t]) continue;
        for (int i = 0; i < 3; ++i) {
          const int a = tri[t][i], b = tri[t][(i + 1) % 3];
          const double l = len(a, b);
          if (l < eps) cand.emplace_back(l, std::min(a, b), std::max(a, b));
        }
      }
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      int64_t done = 0;
      for (const auto& c : cand) {
        const int a = std::get<1>(c), b = std::get<2>(c);
        if (star[a].empty() || star[b].empty() || shared_triangles(a, b).empty()) continue;
        if (!(len(a, b) < eps)) continue;
        if (try_edge(a, b)) ++done;
      }
      total += done;
      if (done == 0) break;
    }
    return total;
  }
};

}  // namespace

extern "C" int mesh_contract(const MeshDesc* desc, const double* xy, double eps, int32_t* tri_out,
                             int64_t* n_triangles_out, int32_t* kind_out, int32_t* line_out,
                             double* xy_out, int64_t* n_vertices_out, int32_t* old_to_new,
                             int64_t* n_contracted) {
  if (!desc || !xy || !tri_out || !n_triangles_out || !kind_out || !line_out || !xy_out ||
      !n_vertices_out || !old_to_new || !n_contracted)
    return fail(CCSP_E_ARG, "mesh_contract: null argument");
  const int64_t V = desc->n_vertices, T = desc->n_triangles, P = desc->n_prims;
  if (V <= 0 || T <= 0 || P < 0 || !desc->kind || !desc->line || !desc->tri_v ||
      (P > 0 && !desc->prim_v))
    return fail(CCSP_E_ARG, "mesh_contract: null array or empty mesh");
  if (V >= (int64_t(1) << 31) || T >= (int64_t(1) << 31))
    return fail(CCSP_E_ARG, "mesh_contract: mesh too large for 32-bit ids");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(CCSP_E_ARG, "mesh_contract: eps must be > 0");
  Contractor c;
  c.kind.assign(desc->kind, desc->kind + V);
  c.line.assign(desc->line, desc->line + V);
  c.prim.resize(P);
  for (int64_t k = 0; k < P; ++k) {
    const int32_t a = desc->prim_v[2 * k], b = desc->prim_v[2 * k + 1];
    if (a < 0 || a >= V || b < 0 || b >= V)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_contract: original edge vertex out of range");
    c.prim[k] = {a, b};
  }
  for (int64_t v = 0; v < V; ++v) {
    const int k = c.kind[v];
    if (k != CCSP_VERTEX_ORIGINAL && k != CCSP_VERTEX_CONSTRAINED && k != CCSP_VERTEX_FREE)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_contract: unknown vertex kind");
    if (k == CCSP_VERTEX_CONSTRAINED && (c.line[v] < 0 || c.line[v] >= P))
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_contract: constrained vertex without edge");
    if (!std::isfinite(xy[2 * v]) || !std::isfinite(xy[2 * v + 1]))
      return fail(CCSP_E_ARG, "mesh_contract: position not finite");
  }
  c.xy.resize(V);
  for (int64_t v = 0; v < V; ++v) c.xy[v] = {xy[2 * v], xy[2 * v + 1]};
  c.tri.resize(T);
  c.tri_alive.assign(T, 1);
  c.star.assign(V, {});
  for (int64_t t = 0; t < T; ++t) {
    for (int k = 0; k < 3; ++k) {
      const int32_t v = desc->tri_v[3 * t + k];
      if (v < 0 || v >= V) return fail(CCSP_E_BAD_TRIANGULATION, "mesh_contract: vertex out of range");
      c.tri[t][k] = v;
    }
    const auto& tv = c.tri[t];
    if (orient_pts(c.xy[tv[0]].data(), c.xy[tv[1]].data(), c.xy[tv[2]].data()) <= 0)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_contract: triangle not counter-clockwise");
    for (int k = 0; k < 3; ++k) c.star[tv[k]].push_back((int32_t)t);
  }
  c.merged_into.resize(V);
  for (int64_t v = 0; v < V; ++v) c.merged_into[v] = (int32_t)v;
  *n_contracted = c.run(eps);
  std::vector<int32_t> new_id(V, -1);
  int64_t nv = 0;
  for (int64_t v = 0; v < V; ++v)
    if (!c.star[v].empty()) {
      new_id[v] = (int32_t)nv;
      kind_out[nv] = c.kind[v];
      line_out[nv] = c.line[v];
      xy_out[2 * nv] = c.xy[v][0];
      xy_out[2 * nv + 1] = c.xy[v][1];
      ++nv;
    }
  for (int64_t v = 0; v < V; ++v) {
    int32_t r = (int32_t)v;
    while (c.merged_into[r] != r) r = c.merged_into[r];
    old_to_new[v] = new_id[r];
  }
  int64_t nt = 0;
  for (int64_t t = 0; t < T; ++t)
    if (c.tri_alive[t]) {
      for (int k = 0; k < 3; ++k) tri_out[3 * nt + k] = new_id[c.tri[t][k]];
      ++nt;
    }
  *n_vertices_out = nv;
  *n_triangles_out = nt;
  return CCSP_OK;
}
