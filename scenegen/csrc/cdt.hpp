// Constrained Delaunay triangulation of a planar straight-line graph, built on the host.
//
// Points are inserted one at a time (Lawson's incremental Delaunay algorithm, points in Hilbert
// order, located by a walk from the previous triangle). Segments are then recovered by Sloan's
// (1993) flip method: every edge crossing the segment is flipped until the segment appears, after
// which Lawson flips restore the constrained Delaunay property across every unconstrained edge.
// All decisions use the exact predicates in predicates.hpp.
//
// Triangle layout: vertex ids v[3t+i] in counter-clockwise order; edge i of triangle t joins
// v[3t+i+1] and v[3t+i+2] (indices mod 3) and lies opposite v[3t+i]; nb[3t+i] is the triangle on
// the other side of edge i (-1 on the hull); pr[3t+i] is the primitive id of a constrained edge,
// -1 otherwise.
#pragma once
#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "predicates.hpp"

namespace sg {

struct Mesh {
  const double* xy = nullptr;  // 2 * nv
  int64_t nv = 0;
  std::vector<int32_t> v, nb, pr;
  std::vector<int32_t> vt;  // one triangle incident to each vertex (-1 if not yet inserted)

  int ntri() const { return (int)(v.size() / 3); }
  double X(int i) const { return xy[2 * (int64_t)i]; }
  double Y(int i) const { return xy[2 * (int64_t)i + 1]; }
  int orient(int a, int b, int c) const { return pred::orient(X(a), Y(a), X(b), Y(b), X(c), Y(c)); }
  int orient_pt(int a, int b, double px, double py) const {
    return pred::orient(X(a), Y(a), X(b), Y(b), px, py);
  }
  int incircle(int a, int b, int c, int d) const {
    return pred::incircle(X(a), Y(a), X(b), Y(b), X(c), Y(c), X(d), Y(d));
  }

  int new_tri() {
    v.resize(v.size() + 3, -1);
    nb.resize(nb.size() + 3, -1);
    pr.resize(pr.size() + 3, -1);
    return ntri() - 1;
  }
  int edge_to(int t, int other) const {  // local index i with nb[3t+i] == other
    for (int i = 0; i < 3; ++i)
      if (nb[3 * t + i] == other) return i;
    throw std::runtime_error("cdt: broken adjacency");
  }
  void replace_nb(int t, int old_t, int new_t) {
    if (t < 0) return;
    nb[3 * t + edge_to(t, old_t)] = new_t;
  }

  // Flip the edge i of triangle t. With t = (p,q,r), p = v[t][i], and its neighbour n = (s,r,q),
  // the result is t = (p,q,s) and n = (s,r,p); the new edge p-s is edge 1 of both.
  void flip(int t, int i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    const int p = v[3 * t + i], q = v[3 * t + i1], r = v[3 * t + i2];
    const int n = nb[3 * t + i];
    const int j = edge_to(n, t), j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    const int s = v[3 * n + j];
    const int n_rp = nb[3 * t + i1], c_rp = pr[3 * t + i1];
    const int n_pq = nb[3 * t + i2], c_pq = pr[3 * t + i2];
    const int n_qs = nb[3 * n + j1], c_qs = pr[3 * n + j1];
    const int n_sr = nb[3 * n + j2], c_sr = pr[3 * n + j2];
    v[3 * t + 0] = p; v[3 * t + 1] = q; v[3 * t + 2] = s;
    nb[3 * t + 0] = n_qs; pr[3 * t + 0] = c_qs;
    nb[3 * t + 1] = n;    pr[3 * t + 1] = -1;
    nb[3 * t + 2] = n_pq; pr[3 * t + 2] = c_pq;
    v[3 * n + 0] = s; v[3 * n + 1] = r; v[3 * n + 2] = p;
    nb[3 * n + 0] = n_rp; pr[3 * n + 0] = c_rp;
    nb[3 * n + 1] = t;    pr[3 * n + 1] = -1;
    nb[3 * n + 2] = n_sr; pr[3 * n + 2] = c_sr;
    replace_nb(n_qs, n, t);
    replace_nb(n_rp, t, n);
    vt[p] = t; vt[q] = t; vt[s] = t; vt[r] = n;
  }

  // The quad around edge i of t is strictly convex (the edge may be flipped).
  bool flippable(int t, int i) const {
    const int n = nb[3 * t + i];
    if (n < 0 || pr[3 * t + i] >= 0) return false;
    const int p = v[3 * t + i], q = v[3 * t + (i + 1) % 3], r = v[3 * t + (i + 2) % 3];
    const int s = v[3 * n + edge_to(n, t)];
    return orient(p, q, s) > 0 && orient(s, r, p) > 0;
  }

  // Lawson legalisation of the edges on the stack (t, local edge index). With `around_point`, every
  // stacked edge lies opposite a newly inserted point p and only the two edges opposite p need a
  // re-check after a flip; otherwise all four outer edges of the flipped quad are re-checked.
  void legalize(std::vector<std::pair<int, int>>& st, bool around_point) {
    while (!st.empty()) {
      auto [t, i] = st.back();
      st.pop_back();
      const int n = nb[3 * t + i];
      if (n < 0 || pr[3 * t + i] >= 0) continue;
      const int s = v[3 * n + edge_to(n, t)];
      if (incircle(v[3 * t], v[3 * t + 1], v[3 * t + 2], s) > 0) {
        flip(t, i);
        // After the flip, t = (p,q,s) and n = (s,r,p) with p the old apex of t.
        st.push_back({t, 0});
        st.push_back({n, 2});
        if (!around_point) {
          st.push_back({t, 2});
          st.push_back({n, 0});
        }
      }
    }
  }

  // Visibility walk from triangle t towards (px,py). Returns the triangle and sets `loc` to
  // -1 (strictly inside), 0..2 (on that edge) or 3 (on a vertex). Randomised edge order keeps the
  // walk from cycling in non-Delaunay triangulations.
  int locate(double px, double py, int t, int& loc, uint64_t& rng) const {
    const int64_t limit = 4 * (int64_t)ntri() + 64;
    for (int64_t it = 0; it < limit; ++it) {
      rng = rng * 6364136223846793005ull + 1442695040888963407ull;
      const int off = (int)((rng >> 33) % 3);
      bool moved = false;
      int zeros = 0, zedge = -1;
      for (int k = 0; k < 3; ++k) {
        const int e = (off + k) % 3;
        const int o = orient_pt(v[3 * t + (e + 1) % 3], v[3 * t + (e + 2) % 3], px, py);
        if (o < 0) {
          const int n = nb[3 * t + e];
          if (n < 0) {
            loc = -2;  // outside the triangulated domain
            return t;
          }
          t = n;
          moved = true;
          break;
        }
        if (o == 0) {
          ++zeros;
          zedge = e;
        }
      }
      if (!moved) {
        loc = zeros == 0 ? -1 : (zeros == 1 ? zedge : 3);
        return t;
      }
    }
    throw std::runtime_error("cdt: point location did not terminate");
  }

  void insert_in_triangle(int t, int p, std::vector<std::pair<int, int>>& st) {
    const int a = v[3 * t], b = v[3 * t + 1], c = v[3 * t + 2];
    const int n0 = nb[3 * t], n1 = nb[3 * t + 1], n2 = nb[3 * t + 2];
    const int c0 = pr[3 * t], c1 = pr[3 * t + 1], c2 = pr[3 * t + 2];
    const int t1 = new_tri(), t2 = new_tri();
    // t = (p,b,c), t1 = (a,p,c), t2 = (a,b,p)
    v[3 * t] = p; v[3 * t + 1] = b; v[3 * t + 2] = c;
    nb[3 * t] = n0; nb[3 * t + 1] = t1; nb[3 * t + 2] = t2;
    pr[3 * t] = c0; pr[3 * t + 1] = -1; pr[3 * t + 2] = -1;
    v[3 * t1] = a; v[3 * t1 + 1] = p; v[3 * t1 + 2] = c;
    nb[3 * t1] = t; nb[3 * t1 + 1] = n1; nb[3 * t1 + 2] = t2;
    pr[3 * t1 + 1] = c1;
    v[3 * t2] = a; v[3 * t2 + 1] = b; v[3 * t2 + 2] = p;
    nb[3 * t2] = t; nb[3 * t2 + 1] = t1; nb[3 * t2 + 2] = n2;
    pr[3 * t2 + 2] = c2;
    replace_nb(n1, t, t1);
    replace_nb(n2, t, t2);
    vt[p] = t; vt[a] = t1; vt[b] = t2; vt[c] = t;
    st.push_back({t, 0});
    st.push_back({t1, 1});
    st.push_back({t2, 2});
  }

  void insert_on_edge(int t, int i, int p, std::vector<std::pair<int, int>>& st) {
    const int n = nb[3 * t + i];
    if (n < 0) throw std::runtime_error("cdt: point on the hull");
    if (pr[3 * t + i] >= 0) throw std::runtime_error("cdt: point on a constrained edge");
    const int j = edge_to(n, t);
    const int a = v[3 * t + i], b = v[3 * t + (i + 1) % 3], c = v[3 * t + (i + 2) % 3];
    const int d = v[3 * n + j];
    const int nt_ca = nb[3 * t + (i + 1) % 3], ct_ca = pr[3 * t + (i + 1) % 3];  // edge (c,a)
    const int nt_ab = nb[3 * t + (i + 2) % 3], ct_ab = pr[3 * t + (i + 2) % 3];  // edge (a,b)
    const int nn_bd = nb[3 * n + (j + 1) % 3], cn_bd = pr[3 * n + (j + 1) % 3];  // edge (b,d)
    const int nn_dc = nb[3 * n + (j + 2) % 3], cn_dc = pr[3 * n + (j + 2) % 3];  // edge (d,c)
    const int tac = new_tri(), ndb = new_tri();
    // t = (a,b,p), tac = (a,p,c), n = (d,c,p), ndb = (d,p,b)
    v[3 * t] = a; v[3 * t + 1] = b; v[3 * t + 2] = p;
    nb[3 * t] = ndb; nb[3 * t + 1] = tac; nb[3 * t + 2] = nt_ab;
    pr[3 * t] = -1; pr[3 * t + 1] = -1; pr[3 * t + 2] = ct_ab;
    v[3 * tac] = a; v[3 * tac + 1] = p; v[3 * tac + 2] = c;
    nb[3 * tac] = n; nb[3 * tac + 1] = nt_ca; nb[3 * tac + 2] = t;
    pr[3 * tac + 1] = ct_ca;
    v[3 * n] = d; v[3 * n + 1] = c; v[3 * n + 2] = p;
    nb[3 * n] = tac; nb[3 * n + 1] = ndb; nb[3 * n + 2] = nn_dc;
    pr[3 * n] = -1; pr[3 * n + 1] = -1; pr[3 * n + 2] = cn_dc;
    v[3 * ndb] = d; v[3 * ndb + 1] = p; v[3 * ndb + 2] = b;
    nb[3 * ndb] = t; nb[3 * ndb + 1] = nn_bd; nb[3 * ndb + 2] = n;
    pr[3 * ndb + 1] = cn_bd;
    replace_nb(nt_ca, t, tac);
    replace_nb(nn_bd, n, ndb);
    vt[p] = t; vt[a] = t; vt[b] = t; vt[c] = tac; vt[d] = n;
    st.push_back({t, 2});
    st.push_back({tac, 1});
    st.push_back({n, 2});
    st.push_back({ndb, 1});
  }

  // Find the triangle with directed edge u->w (u = v[i+1], w = v[i+2]); returns (t, i) or (-1,-1).
  std::pair<int, int> find_edge(int u, int w) const {
    const int t0 = vt[u];
    int t = t0;
    do {
      int k = (v[3 * t] == u) ? 0 : (v[3 * t + 1] == u ? 1 : 2);
      if (v[3 * t + (k + 1) % 3] == w) return {t, (k + 2) % 3};
      if (v[3 * t + (k + 2) % 3] == w) return {t, (k + 1) % 3};
      t = nb[3 * t + (k + 1) % 3];  // rotate counter-clockwise about u
    } while (t >= 0 && t != t0);
    if (t < 0) {  // u on the hull: sweep clockwise from t0 as well
      t = t0;
      while (true) {
        int k = (v[3 * t] == u) ? 0 : (v[3 * t + 1] == u ? 1 : 2);
        if (v[3 * t + (k + 1) % 3] == w) return {t, (k + 2) % 3};
        if (v[3 * t + (k + 2) % 3] == w) return {t, (k + 1) % 3};
        t = nb[3 * t + (k + 2) % 3];
        if (t < 0 || t == t0) break;
      }
    }
    return {-1, -1};
  }

  static bool crosses(const Mesh& m, int a, int b, int p, int s) {
    if (p == a || p == b || s == a || s == b) return false;
    const int o1 = m.orient(a, b, p), o2 = m.orient(a, b, s);
    if ((int64_t)o1 * o2 >= 0) return false;
    const int o3 = m.orient(p, s, a), o4 = m.orient(p, s, b);
    return (int64_t)o3 * o4 < 0;
  }

  void insert_segment(int a, int b, int prim) {
    auto mark = [&](int u, int w) {
      auto e = find_edge(u, w);
      if (e.first < 0) throw std::runtime_error("cdt: segment edge missing after recovery");
      pr[3 * e.first + e.second] = prim;
      const int n = nb[3 * e.first + e.second];
      if (n >= 0) pr[3 * n + edge_to(n, e.first)] = prim;
    };
    if (find_edge(a, b).first >= 0 || find_edge(b, a).first >= 0) {
      mark(a, b);
      return;
    }
    // Triangle around a whose wedge contains b.
    int t = vt[a], k = -1;
    const int t0 = t;
    while (true) {
      k = (v[3 * t] == a) ? 0 : (v[3 * t + 1] == a ? 1 : 2);
      const int v1 = v[3 * t + (k + 1) % 3], v2 = v[3 * t + (k + 2) % 3];
      const int o1 = orient(a, v1, b), o2 = orient(a, v2, b);
      if (o1 > 0 && o2 < 0) break;
      if (o1 == 0 && (X(v1) - X(a)) * (X(b) - X(a)) + (Y(v1) - Y(a)) * (Y(b) - Y(a)) > 0)
        throw std::runtime_error("cdt: vertex lies on a segment");
      t = nb[3 * t + (k + 1) % 3];
      if (t < 0 || t == t0) throw std::runtime_error("cdt: cannot find segment start wedge");
    }
    // March along a->b collecting crossed edges (as vertex pairs).
    std::vector<std::pair<int, int>> q;
    int e = k;  // crossed edge of t
    while (true) {
      const int x = v[3 * t + (e + 1) % 3], y = v[3 * t + (e + 2) % 3];
      q.push_back({x, y});
      const int n = nb[3 * t + e];
      if (n < 0) throw std::runtime_error("cdt: segment leaves the domain");
      if (pr[3 * t + e] >= 0) throw std::runtime_error("cdt: segments intersect");
      const int j = edge_to(n, t);
      const int w = v[3 * n + j];
      if (w == b) break;
      const int o = orient(a, b, w);
      if (o == 0) throw std::runtime_error("cdt: vertex lies on a segment");
      t = n;
      e = (o > 0) ? (j + 1) % 3 : (j + 2) % 3;
    }
    // Sloan: flip crossing edges until none is left.
    std::vector<std::pair<int, int>> fresh;
    size_t head = 0;
    int64_t guard = 0;
    while (head < q.size()) {
      if (++guard > 100000000) throw std::runtime_error("cdt: segment recovery did not terminate");
      auto [x, y] = q[head++];
      auto te = find_edge(x, y);
      if (te.first < 0) continue;  // already removed by an earlier flip
      const int tt = te.first, ii = te.second;
      if (!flippable(tt, ii)) {
        q.push_back({x, y});
        continue;
      }
      flip(tt, ii);
      const int p = v[3 * tt + 0], s = v[3 * tt + 2];  // new edge p-s
      if (crosses(*this, a, b, p, s))
        q.push_back({p, s});
      else
        fresh.push_back({p, s});
    }
    mark(a, b);
    // Restore the constrained Delaunay property around the new edges.
    std::vector<std::pair<int, int>> st;
    for (auto [x, y] : fresh) {
      auto te = find_edge(x, y);
      if (te.first >= 0) st.push_back(te);
    }
    legalize(st, false);
  }
};

}  // namespace sg
