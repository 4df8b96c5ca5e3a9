// Seeded synthetic scenes, triangulations and rays (host side, C ABI for ctypes).
//
// Scenes follow the "lines" family of the paper's experiments (Sec. 4.2): non-crossing segments
// with uniform midpoints, uniform orientations and a range of lengths, inside a bounding square
// whose four sides are themselves constrained primitives. Triangulations are the constrained
// Delaunay triangulation (Sec. 3.5.1 starts from one) and, optionally, a flip-only annealed
// low-weight triangulation (the edge-flip perturbation of Sec. 3.2.7 under the Metropolis rule of
// Eq. 3.5, with the exponential cooling of Sec. 3.3 and the greedy flip sweep of Sec. 3.4.2).
// Rays follow the experimental setup of Sec. 5.4: origins uniform over the scene area with their
// containing triangle known, directions isotropic.
//
// Random numbers come from a counter-based generator: the SplitMix64 output function (Steele, Lea
// and Flood, OOPSLA 2014) applied to key + counter * golden ratio, so every ray can be drawn
// independently and in parallel.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "cdt.hpp"
#include "predicates.hpp"

namespace sg {

static thread_local std::string g_err;

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
static inline uint64_t key_of(uint64_t seed, uint64_t tag) { return mix64(seed * kGolden + tag + 1); }
static inline double u01(uint64_t key, uint64_t ctr) {  // uniform in [0,1), 53 bits
  return (double)(mix64(key + (ctr + 1) * kGolden) >> 11) * 0x1.0p-53;
}

// ------------------------------------------------------------------ segment sampling
// Closed segments intersect (touching counts).
static bool seg_intersect(const double* s, const double* t) {
  using pred::orient;
  const int o1 = orient(s[0], s[1], s[2], s[3], t[0], t[1]);
  const int o2 = orient(s[0], s[1], s[2], s[3], t[2], t[3]);
  const int o3 = orient(t[0], t[1], t[2], t[3], s[0], s[1]);
  const int o4 = orient(t[0], t[1], t[2], t[3], s[2], s[3]);
  if (o1 * o2 > 0 || o3 * o4 > 0) return false;
  if (o1 == 0 && o2 == 0) {  // collinear: overlap of the projections
    const bool usex = std::fabs(s[2] - s[0]) >= std::fabs(s[3] - s[1]);
    const int k = usex ? 0 : 1;
    const double a0 = std::min(s[k], s[k + 2]), a1 = std::max(s[k], s[k + 2]);
    const double b0 = std::min(t[k], t[k + 2]), b1 = std::max(t[k], t[k + 2]);
    return !(a1 < b0 || b1 < a0);
  }
  return true;
}

struct SegGrid {
  double lo, cell;
  int n;
  std::vector<std::vector<int32_t>> cells;
  SegGrid(double lo_, double hi_, double cell_) : lo(lo_), cell(cell_) {
    n = std::max(1, (int)std::ceil((hi_ - lo_) / cell_));
    cells.resize((size_t)n * n);
  }
  void range(const double* s, int& x0, int& x1, int& y0, int& y1) const {
    auto c = [&](double v) { return std::min(n - 1, std::max(0, (int)std::floor((v - lo) / cell))); };
    x0 = c(std::min(s[0], s[2])); x1 = c(std::max(s[0], s[2]));
    y0 = c(std::min(s[1], s[3])); y1 = c(std::max(s[1], s[3]));
  }
};

// Sequential rejection sampling of n non-crossing segments.
// Midpoints uniform in [mlo,mhi]^2, lengths uniform (or log-uniform) in [llo,lhi], angles
// uniform in [0,pi). A candidate is rejected if an endpoint is not strictly inside the open square
// (blo,bhi)^2 or if it touches or crosses an accepted segment.
static int64_t random_segments(uint64_t seed, int64_t n, double mlo, double mhi, double llo,
                               double lhi, int log_len, double blo, double bhi, double* out,
                               int64_t max_draws) {
  const uint64_t key = key_of(seed, 0x5e6);
  SegGrid grid(blo, bhi, std::max(lhi, (bhi - blo) / 4096.0));
  int64_t m = 0, draw = 0;
  while (m < n) {
    if (draw >= max_draws) break;
    const uint64_t c = 4 * (uint64_t)draw++;
    const double mx = mlo + (mhi - mlo) * u01(key, c);
    const double my = mlo + (mhi - mlo) * u01(key, c + 1);
    const double ul = u01(key, c + 2);
    const double len = log_len ? std::exp(std::log(llo) + (std::log(lhi) - std::log(llo)) * ul)
                               : llo + (lhi - llo) * ul;
    const double th = M_PI * u01(key, c + 3);
    const double hx = 0.5 * len * std::cos(th), hy = 0.5 * len * std::sin(th);
    double s[4] = {mx - hx, my - hy, mx + hx, my + hy};
    bool ok = true;
    for (int k = 0; k < 4; ++k)
      if (!(s[k] > blo && s[k] < bhi)) ok = false;
    if (!ok) continue;
    int x0, x1, y0, y1;
    grid.range(s, x0, x1, y0, y1);
    for (int gx = x0; gx <= x1 && ok; ++gx)
      for (int gy = y0; gy <= y1 && ok; ++gy)
        for (int32_t id : grid.cells[(size_t)gx * grid.n + gy])
          if (seg_intersect(s, out + 4 * (int64_t)id)) {
            ok = false;
            break;
          }
    if (!ok) continue;
    std::memcpy(out + 4 * m, s, sizeof(s));
    for (int gx = x0; gx <= x1; ++gx)
      for (int gy = y0; gy <= y1; ++gy) grid.cells[(size_t)gx * grid.n + gy].push_back((int32_t)m);
    ++m;
  }
  return m;
}

// ------------------------------------------------------------------ CDT construction
static uint64_t hilbert_key(uint32_t x, uint32_t y, int order) {
  // Position of (x,y) along the Hilbert curve of a 2^order grid (quadrant-rotation form).
  const uint32_t n = 1u << order;
  uint64_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
    d += (uint64_t)s * s * ((3 * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

static std::vector<int32_t> hilbert_order(const double* xy, const std::vector<int32_t>& ids) {
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int32_t i : ids) {
    x0 = std::min(x0, xy[2 * (int64_t)i]); x1 = std::max(x1, xy[2 * (int64_t)i]);
    y0 = std::min(y0, xy[2 * (int64_t)i + 1]); y1 = std::max(y1, xy[2 * (int64_t)i + 1]);
  }
  const double span = std::max(x1 - x0, y1 - y0) * (1 + 1e-9) + 1e-300;
  const int order = 16;
  const double sc = (double)((1u << order) - 1) / span;
  std::vector<std::pair<uint64_t, int32_t>> k(ids.size());
  for (size_t j = 0; j < ids.size(); ++j) {
    const int32_t i = ids[j];
    const uint32_t gx = (uint32_t)((xy[2 * (int64_t)i] - x0) * sc);
    const uint32_t gy = (uint32_t)((xy[2 * (int64_t)i + 1] - y0) * sc);
    k[j] = {hilbert_key(gx, gy, order), i};
  }
  std::sort(k.begin(), k.end());
  std::vector<int32_t> out(ids.size());
  for (size_t j = 0; j < ids.size(); ++j) out[j] = k[j].second;
  return out;
}

// Vertices 0..3 must be the corners of the bounding box in counter-clockwise order, and every
// other vertex strictly inside it. Segments (pairs of vertex ids) become constrained edges that
// carry their primitive id; the four box sides are added as constrained hull edges carrying
// box_prim0 .. box_prim0+3 (bottom, right, top, left).
static Mesh build_cdt(const double* xy, int64_t nv, const int32_t* segv, const int32_t* segp,
                      int64_t ns, int32_t box_prim0) {
  if (nv < 4) throw std::runtime_error("cdt: need the four box corners");
  Mesh m;
  m.xy = xy;
  m.nv = nv;
  m.vt.assign(nv, -1);
  const int64_t tri_est = 2 * nv;
  m.v.reserve(3 * tri_est); m.nb.reserve(3 * tri_est); m.pr.reserve(3 * tri_est);
  if (m.orient(0, 1, 2) <= 0 || m.orient(0, 2, 3) <= 0)
    throw std::runtime_error("cdt: box corners must be counter-clockwise");
  const int t0 = m.new_tri(), t1 = m.new_tri();
  m.v[0] = 0; m.v[1] = 1; m.v[2] = 2;  // edge 2 = (0,1) bottom, edge 0 = (1,2) right
  m.v[3] = 0; m.v[4] = 2; m.v[5] = 3;  // edge 0 = (2,3) top, edge 1 = (3,0) left
  m.nb[3 * t0 + 1] = t1;  // edge (2,0)
  m.nb[3 * t1 + 2] = t0;  // edge (0,2)
  m.pr[3 * t0 + 2] = box_prim0 + 0;
  m.pr[3 * t0 + 0] = box_prim0 + 1;
  m.pr[3 * t1 + 0] = box_prim0 + 2;
  m.pr[3 * t1 + 1] = box_prim0 + 3;
  m.vt[0] = t0; m.vt[1] = t0; m.vt[2] = t0; m.vt[3] = t1;
  std::vector<int32_t> ids(nv - 4);
  std::iota(ids.begin(), ids.end(), 4);
  const std::vector<int32_t> order = hilbert_order(xy, ids);
  std::vector<std::pair<int, int>> st;
  uint64_t rng = 0x243F6A8885A308D3ull;
  int hint = t0;
  for (int32_t p : order) {
    int loc;
    const int t = m.locate(m.X(p), m.Y(p), hint, loc, rng);
    if (loc == -2) throw std::runtime_error("cdt: vertex outside the bounding box");
    if (loc == 3) throw std::runtime_error("cdt: duplicate vertex");
    if (loc == -1)
      m.insert_in_triangle(t, p, st);
    else
      m.insert_on_edge(t, loc, p, st);
    m.legalize(st, true);
    hint = m.vt[p];
  }
  for (int64_t k = 0; k < ns; ++k) m.insert_segment(segv[2 * k], segv[2 * k + 1], segp[k]);
  return m;
}

// ------------------------------------------------------------------ flip annealing
static double edge_len(const Mesh& m, int a, int b) {
  return std::hypot(m.X(a) - m.X(b), m.Y(a) - m.Y(b));
}
static double total_weight(const Mesh& m) {
  double w = 0;
  const int T = m.ntri();
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) {
      const int n = m.nb[3 * t + i];
      if (n < 0 || n > t) w += edge_len(m, m.v[3 * t + (i + 1) % 3], m.v[3 * t + (i + 2) % 3]);
    }
  return w;
}
// Length change of flipping edge i of t (new diagonal minus old).
static double flip_gain(const Mesh& m, int t, int i) {
  const int n = m.nb[3 * t + i];
  const int p = m.v[3 * t + i], q = m.v[3 * t + (i + 1) % 3], r = m.v[3 * t + (i + 2) % 3];
  const int s = m.v[3 * n + m.edge_to(n, t)];
  return edge_len(m, p, s) - edge_len(m, q, r);
}
static int greedy_flips(Mesh& m) {
  int total = 0;
  while (true) {
    int flips = 0;
    const int T = m.ntri();
    for (int t = 0; t < T; ++t)
      for (int i = 0; i < 3; ++i) {
        const int n = m.nb[3 * t + i];
        if (n < 0 || n < t) continue;  // each interior edge once per sweep
        if (!m.flippable(t, i)) continue;
        if (flip_gain(m, t, i) < 0) {
          m.flip(t, i);
          ++flips;
        }
      }
    total += flips;
    if (flips == 0) break;
  }
  return total;
}

struct AnnealStats {
  double w_start, w_end;
  int64_t proposals, accepted, flips;
};

static AnnealStats anneal(Mesh& m, uint64_t seed, int64_t n_moves, double T0, double T1) {
  AnnealStats st{};
  st.w_start = total_weight(m);
  const uint64_t key = key_of(seed, 0xa22);
  const int T = m.ntri();
  int lambda = 1;
  int64_t window_acc = 0, window_n = 0;
  uint64_t ctr = 0;
  std::vector<std::pair<int, int>> done;
  for (int64_t mv = 0; mv < n_moves; ++mv) {
    const double temp = T0 * std::pow(T1 / T0, (double)mv / (double)std::max<int64_t>(1, n_moves - 1));
    done.clear();
    double dw = 0;
    for (int k = 0; k < lambda; ++k) {
      const double u = u01(key, ctr++);
      const int64_t slot = std::min<int64_t>((int64_t)(u * 3.0 * T), 3 * (int64_t)T - 1);
      const int t = (int)(slot / 3), i = (int)(slot % 3);
      if (!m.flippable(t, i)) continue;
      dw += flip_gain(m, t, i);
      m.flip(t, i);
      done.push_back({t, i});
    }
    ++st.proposals;
    const double ua = u01(key, ctr++);
    const bool acc = !done.empty() && (dw <= 0 || ua < std::exp(-dw / temp));
    if (acc) {
      ++st.accepted;
      ++window_acc;
      st.flips += (int64_t)done.size();
    } else {
      for (auto it = done.rbegin(); it != done.rend(); ++it) m.flip(it->first, 1);  // p-s is edge 1
    }
    if (++window_n == 256) {  // keep the acceptance rate near 23% by adapting the flips per move
      if (window_acc > 0.23 * window_n) lambda = std::min(lambda + 1, 8);
      else if (lambda > 1) --lambda;
      window_acc = window_n = 0;
    }
  }
  greedy_flips(m);
  st.w_end = total_weight(m);
  return st;
}

// ------------------------------------------------------------------ rays
static void sample_rays(const double* xy, int64_t T, const int32_t* tv, uint64_t seed, int64_t n,
                        double* o, double* d, int32_t* start) {
  std::vector<double> cdf(T);
  double acc = 0;
  for (int64_t t = 0; t < T; ++t) {
    const double* a = xy + 2 * (int64_t)tv[3 * t];
    const double* b = xy + 2 * (int64_t)tv[3 * t + 1];
    const double* c = xy + 2 * (int64_t)tv[3 * t + 2];
    acc += 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]));
    cdf[t] = acc;
  }
  const uint64_t key = key_of(seed, 0x7a1);
#pragma omp parallel for schedule(static, 4096)
  for (int64_t r = 0; r < n; ++r) {
    const uint64_t base = key_of(key, (uint64_t)r);
    for (uint64_t attempt = 0;; ++attempt) {
      const uint64_t c = 4 * attempt;
      const double u = u01(base, c) * acc;
      int64_t t = std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin();
      if (t >= T) t = T - 1;
      double r1 = u01(base, c + 1), r2 = u01(base, c + 2);
      if (r1 + r2 > 1.0) { r1 = 1.0 - r1; r2 = 1.0 - r2; }
      const double* a = xy + 2 * (int64_t)tv[3 * t];
      const double* b = xy + 2 * (int64_t)tv[3 * t + 1];
      const double* cc = xy + 2 * (int64_t)tv[3 * t + 2];
      const double px = a[0] + r1 * (b[0] - a[0]) + r2 * (cc[0] - a[0]);
      const double py = a[1] + r1 * (b[1] - a[1]) + r2 * (cc[1] - a[1]);
      if (pred::orient(a[0], a[1], b[0], b[1], px, py) <= 0) continue;
      if (pred::orient(b[0], b[1], cc[0], cc[1], px, py) <= 0) continue;
      if (pred::orient(cc[0], cc[1], a[0], a[1], px, py) <= 0) continue;
      const double th = 2.0 * M_PI * u01(base, c + 3);
      o[2 * r] = px; o[2 * r + 1] = py;
      d[2 * r] = std::cos(th); d[2 * r + 1] = std::sin(th);
      start[r] = (int32_t)t;
      break;
    }
  }
}

static Mesh mesh_from_arrays(const double* xy, int64_t nv, int64_t T, const int32_t* tv,
                             const int32_t* tn, const int32_t* tp) {
  Mesh m;
  m.xy = xy; m.nv = nv;
  m.v.assign(tv, tv + 3 * T);
  m.nb.assign(tn, tn + 3 * T);
  m.pr.assign(tp, tp + 3 * T);
  m.vt.assign(nv, -1);
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) m.vt[m.v[3 * t + i]] = (int32_t)t;
  return m;
}

}  // namespace sg

using namespace sg;

struct SgMesh {
  Mesh m;
};

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

int64_t sg_random_segments(uint64_t seed, int64_t n, double mlo, double mhi, double llo, double lhi,
                           int log_len, double blo, double bhi, double* out, int64_t max_draws) {
  try {
    return random_segments(seed, n, mlo, mhi, llo, lhi, log_len, blo, bhi, out, max_draws);
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

void* sg_build_cdt(const double* xy, int64_t nv, const int32_t* segv, const int32_t* segp,
                   int64_t ns, int32_t box_prim0) {
  try {
    auto* h = new SgMesh;
    h->m = build_cdt(xy, nv, segv, segp, ns, box_prim0);
    return h;
  } catch (const std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

void* sg_mesh_from_arrays(const double* xy, int64_t nv, int64_t T, const int32_t* tv,
                          const int32_t* tn, const int32_t* tp) {
  auto* h = new SgMesh;
  h->m = mesh_from_arrays(xy, nv, T, tv, tn, tp);
  return h;
}

int64_t sg_mesh_ntri(void* h) { return static_cast<SgMesh*>(h)->m.ntri(); }

void sg_mesh_copy(void* h, int32_t* tv, int32_t* tn, int32_t* tp) {
  const Mesh& m = static_cast<SgMesh*>(h)->m;
  std::memcpy(tv, m.v.data(), m.v.size() * 4);
  std::memcpy(tn, m.nb.data(), m.nb.size() * 4);
  std::memcpy(tp, m.pr.data(), m.pr.size() * 4);
}

double sg_mesh_weight(void* h) { return total_weight(static_cast<SgMesh*>(h)->m); }

// Flip-only annealing followed by greedy flips; out = {w_start, w_end, proposals, accepted, flips}.
int sg_mesh_anneal(void* h, uint64_t seed, int64_t n_moves, double T0, double T1, double* out) {
  try {
    AnnealStats s = anneal(static_cast<SgMesh*>(h)->m, seed, n_moves, T0, T1);
    out[0] = s.w_start; out[1] = s.w_end;
    out[2] = (double)s.proposals; out[3] = (double)s.accepted; out[4] = (double)s.flips;
    return 0;
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

int sg_mesh_greedy(void* h) { return greedy_flips(static_cast<SgMesh*>(h)->m); }

// Locate points: out[k] = containing triangle, or -1 if the point lies on an edge or vertex or
// outside the triangulation. Triangles are bucketed by bounding box on a uniform grid and the
// candidates of the point's cell are tested exactly, which works for any valid triangulation.
int sg_mesh_locate(void* h, int64_t n, const double* pts, int32_t* out) {
  try {
    const Mesh& m = static_cast<SgMesh*>(h)->m;
    const int T = m.ntri();
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int64_t i = 0; i < m.nv; ++i) {
      x0 = std::min(x0, m.X(i)); x1 = std::max(x1, m.X(i));
      y0 = std::min(y0, m.Y(i)); y1 = std::max(y1, m.Y(i));
    }
    const int g = std::max(1, std::min(4096, (int)std::sqrt((double)T / 2.0)));
    const double sx = g / std::max(1e-300, x1 - x0), sy = g / std::max(1e-300, y1 - y0);
    auto cx = [&](double x) { return std::min(g - 1, std::max(0, (int)((x - x0) * sx))); };
    auto cy = [&](double y) { return std::min(g - 1, std::max(0, (int)((y - y0) * sy))); };
    std::vector<int64_t> cnt((size_t)g * g + 1, 0);
    auto for_cells = [&](int t, auto&& f) {
      double a0 = 1e300, a1 = -1e300, b0 = 1e300, b1 = -1e300;
      for (int k = 0; k < 3; ++k) {
        const int v = m.v[3 * t + k];
        a0 = std::min(a0, m.X(v)); a1 = std::max(a1, m.X(v));
        b0 = std::min(b0, m.Y(v)); b1 = std::max(b1, m.Y(v));
      }
      for (int i = cx(a0); i <= cx(a1); ++i)
        for (int j = cy(b0); j <= cy(b1); ++j) f((size_t)i * g + j);
    };
    for (int t = 0; t < T; ++t) for_cells(t, [&](size_t c) { ++cnt[c + 1]; });
    for (size_t c = 0; c < (size_t)g * g; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> ids(cnt.back());
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int t = 0; t < T; ++t) for_cells(t, [&](size_t c) { ids[fill[c]++] = t; });
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t k = 0; k < n; ++k) {
      const double px = pts[2 * k], py = pts[2 * k + 1];
      int32_t found = -1;
      if (px >= x0 && px <= x1 && py >= y0 && py <= y1) {
        const size_t c = (size_t)cx(px) * g + cy(py);
        for (int64_t q = cnt[c]; q < cnt[c + 1]; ++q) {
          const int t = ids[q];
          const int a = m.v[3 * t], b = m.v[3 * t + 1], cc = m.v[3 * t + 2];
          const int o0 = m.orient_pt(b, cc, px, py), o1 = m.orient_pt(cc, a, px, py),
                    o2 = m.orient_pt(a, b, px, py);
          if (o0 > 0 && o1 > 0 && o2 > 0) {
            found = t;
            break;
          }
          if (o0 >= 0 && o1 >= 0 && o2 >= 0) break;  // on the boundary of t: not strictly inside any
        }
      }
      out[k] = found;
    }
    return 0;
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

void sg_mesh_free(void* h) { delete static_cast<SgMesh*>(h); }

void sg_sample_rays(const double* xy, int64_t T, const int32_t* tv, uint64_t seed, int64_t n,
                    double* o, double* d, int32_t* start, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  sample_rays(xy, T, tv, seed, n, o, d, start);
}

// Exact orientation signs for a batch of point triples (6 doubles per query: a, b, c).
void sg_orient_batch(int64_t n, const double* abc, int32_t* out) {
  for (int64_t k = 0; k < n; ++k) {
    const double* q = abc + 6 * k;
    out[k] = pred::orient(q[0], q[1], q[2], q[3], q[4], q[5]);
  }
}

}  // extern "C"
