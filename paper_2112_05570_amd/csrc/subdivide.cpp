// Subdivision of a triangulation (paper Sec. 3.5.2): every triangle split into four at the
// midpoints of its edges, adding topological degrees of freedom before an optimisation. The
// C-ABI mesh_subdivide of ccsp_objective.h. Host code: one pass over the edges, linear in size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ccsp_objective.h"
#include "exact.hpp"
#include "walk.hpp"

namespace {

int fail(int code, const char* msg) {
  ccsp::set_last_error(msg);
  return code;
}

// binary64 filter (error bound (3 + 16u) u of this evaluation, below 2^-51), then exact
int orient3(const double* a, const double* b, const double* c) {
  const double l = (b[0] - a[0]) * (c[1] - a[1]);
  const double r = (b[1] - a[1]) * (c[0] - a[0]);
  const double det = l - r, sum = std::fabs(l) + std::fabs(r);
  if (std::fabs(det) > 0x1p-51 * sum && sum > 0x1p-900) return det > 0 ? 1 : -1;
  return ccsp::orient_exact(a[0], a[1], b[0], b[1], c[0], c[1]);
}

}  // namespace

extern "C" {

int mesh_subdivide(const MeshDesc* desc, const double* xy, int64_t* n_vertices_out,
                   int64_t* n_triangles_out, double* xy_out, int32_t* tri_out, int32_t* kind_out,
                   int32_t* line_out) {
  if (!desc || !xy || !n_vertices_out || !n_triangles_out)
    return fail(CCSP_E_ARG, "mesh_subdivide: null argument");
  const int64_t V = desc->n_vertices, T = desc->n_triangles, P = desc->n_prims;
  if (V <= 0 || T <= 0 || P < 0 || !desc->kind || !desc->line || !desc->tri_v ||
      (P > 0 && !desc->prim_v))
    return fail(CCSP_E_ARG, "mesh_subdivide: bad mesh description");
  if (4 * T >= (int64_t(1) << 31) || V + 3 * T >= (int64_t(1) << 31))
    return fail(CCSP_E_ARG, "mesh_subdivide: the result would exceed 2^31 vertices or triangles");
  const int32_t* tv = desc->tri_v;
  const int32_t* kind = desc->kind;
  const int32_t* line = desc->line;
  const int32_t* pv = desc->prim_v;
  for (int64_t i = 0; i < 3 * T; ++i)
    if (tv[i] < 0 || tv[i] >= V) return fail(CCSP_E_BAD_TRIANGULATION, "mesh_subdivide: vertex id out of range");
  for (int64_t v = 0; v < V; ++v) {
    if (kind[v] < CCSP_VERTEX_ORIGINAL || kind[v] > CCSP_VERTEX_FREE)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_subdivide: unknown vertex kind");
    if (kind[v] == CCSP_VERTEX_CONSTRAINED && (line[v] < 0 || line[v] >= P))
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_subdivide: constrained vertex without an original edge");
  }
  // edges by key min * V + max, increasing: edge e's midpoint is vertex V + e
  std::vector<int64_t> key(3 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) {
      const int64_t a = tv[3 * t + (i + 1) % 3], b = tv[3 * t + (i + 2) % 3];
      key[3 * t + i] = std::min(a, b) * V + std::max(a, b);
    }
  std::vector<int64_t> uniq(key);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  const int64_t E = (int64_t)uniq.size();
  *n_vertices_out = V + E;
  *n_triangles_out = 4 * T;
  if (!xy_out || !tri_out || !kind_out || !line_out) return CCSP_OK;  // sizes only
  // original edges by their ends, for midpoints of edges joining two ORIGINAL vertices
  std::vector<std::pair<int64_t, int32_t>> okey;
  okey.reserve(P);
  for (int64_t k = 0; k < P; ++k) {
    const int64_t a = pv[2 * k], b = pv[2 * k + 1];
    if (a < 0 || a >= V || b < 0 || b >= V)
      return fail(CCSP_E_BAD_TRIANGULATION, "mesh_subdivide: original edge end out of range");
    okey.emplace_back(std::min(a, b) * V + std::max(a, b), (int32_t)k);
  }
  std::sort(okey.begin(), okey.end());
  auto on_line = [&](int64_t v, int32_t L) {
    if (kind[v] == CCSP_VERTEX_CONSTRAINED) return line[v] == L;
    if (kind[v] == CCSP_VERTEX_ORIGINAL) return pv[2 * L] == v || pv[2 * L + 1] == v;
    return false;
  };
  for (int64_t v = 0; v < V; ++v) {
    xy_out[2 * v] = xy[2 * v];
    xy_out[2 * v + 1] = xy[2 * v + 1];
    kind_out[v] = kind[v];
    line_out[v] = line[v];
  }
  for (int64_t e = 0; e < E; ++e) {
    const int64_t a = uniq[e] / V, b = uniq[e] % V, m = V + e;
    xy_out[2 * m] = (xy[2 * a] + xy[2 * b]) * 0.5;
    xy_out[2 * m + 1] = (xy[2 * a + 1] + xy[2 * b + 1]) * 0.5;
    // the midpoint stays on the original edge that holds both ends, if one does
    int32_t L = -1;
    if (kind[a] == CCSP_VERTEX_CONSTRAINED) L = line[a];
    else if (kind[b] == CCSP_VERTEX_CONSTRAINED) L = line[b];
    else if (kind[a] == CCSP_VERTEX_ORIGINAL && kind[b] == CCSP_VERTEX_ORIGINAL) {
      auto it = std::lower_bound(okey.begin(), okey.end(), std::make_pair(uniq[e], (int32_t)-1));
      if (it != okey.end() && it->first == uniq[e]) L = it->second;
    }
    const bool cons = L >= 0 && on_line(a, L) && on_line(b, L);
    kind_out[m] = cons ? CCSP_VERTEX_CONSTRAINED : CCSP_VERTEX_FREE;
    line_out[m] = cons ? L : -1;
  }
  // sub-triangles: (v0, m2, m1), then (v1, m0, m2), (v2, m1, m0), (m0, m1, m2), each block over
  // every triangle in order; m_i is the midpoint of edge i (opposite v_i)
  for (int64_t t = 0; t < T; ++t) {
    int32_t v[3], mm[3];
    for (int i = 0; i < 3; ++i) {
      v[i] = tv[3 * t + i];
      mm[i] = (int32_t)(V + (std::lower_bound(uniq.begin(), uniq.end(), key[3 * t + i]) - uniq.begin()));
    }
    const int32_t sub[4][3] = {{v[0], mm[2], mm[1]}, {v[1], mm[0], mm[2]}, {v[2], mm[1], mm[0]},
                               {mm[0], mm[1], mm[2]}};
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 3; ++j) tri_out[3 * (k * T + t) + j] = sub[k][j];
  }
  for (int64_t t = 0; t < 4 * T; ++t) {
    const int32_t* s = tri_out + 3 * t;
    if (orient3(xy_out + 2 * s[0], xy_out + 2 * s[1], xy_out + 2 * s[2]) <= 0)
      return fail(CCSP_E_BAD_TRIANGULATION,
                  "mesh_subdivide: a sub-triangle is not strictly counter-clockwise (a midpoint "
                  "rounded across an edge)");
  }
  return CCSP_OK;
}

}  // extern "C"
