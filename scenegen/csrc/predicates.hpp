// Exact geometric predicates for the host-side scene and triangulation builder.
//
// orient(a,b,c) = sign of (b-a) x (c-a); incircle(a,b,c,d) > 0 iff d lies strictly inside the
// circumcircle of the counter-clockwise triangle (a,b,c). Both are evaluated exactly on the double
// inputs: a floating-point evaluation with a forward error bound decides the sign when it is
// certain, and otherwise the determinant is expanded into a nonoverlapping floating-point
// expansion (error-free transforms: Knuth's TwoSum, an FMA-based TwoProduct, Shewchuk's
// Grow-Expansion and Compress, 1997) whose leading component carries the exact sign.
//
// This copy belongs to the input builder only; the walk library and the checker each have their
// own, written independently, so that the three can be checked against each other.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace sg {
namespace pred {

static constexpr double kU = 0x1.0p-53;  // unit roundoff of binary64

static inline void two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  y = (a - av) + (b - bv);
}
static inline void fast_two_sum(double a, double b, double& x, double& y) {  // |a| >= |b|
  x = a + b;
  y = b - (x - a);
}
static inline void two_prod(double a, double b, double& x, double& y) {
  x = a * b;
  y = std::fma(a, b, -x);
}

// Expansion: nonoverlapping components, increasing magnitude, zeros eliminated.
using Exp = std::vector<double>;

static inline Exp grow(const Exp& e, double b) {
  Exp h;
  h.reserve(e.size() + 1);
  double q = b;
  for (double ei : e) {
    double s, t;
    two_sum(q, ei, s, t);
    if (t != 0.0) h.push_back(t);
    q = s;
  }
  if (q != 0.0 || h.empty()) h.push_back(q);
  return h;
}
static inline Exp compress(const Exp& e) {
  const int m = (int)e.size();
  if (m <= 1) return e;
  std::vector<double> g(m);
  double Q = e[m - 1];
  int bottom = m - 1;
  for (int i = m - 2; i >= 0; --i) {
    double Qn, q;
    fast_two_sum(Q, e[i], Qn, q);
    if (q != 0.0) {
      g[bottom--] = Qn;
      Q = q;
    } else {
      Q = Qn;
    }
  }
  g[bottom] = Q;
  Exp h;
  for (int i = bottom + 1; i < m; ++i) {
    double Qn, q;
    fast_two_sum(g[i], Q, Qn, q);
    if (q != 0.0) h.push_back(q);
    Q = Qn;
  }
  h.push_back(Q);
  return h;
}
static inline Exp add(const Exp& e, const Exp& f) {
  Exp h = e;
  for (double x : f) h = grow(h, x);
  return compress(h);
}
static inline Exp neg(Exp e) {
  for (double& x : e) x = -x;
  return e;
}
static inline Exp mul(const Exp& e, const Exp& f) {
  Exp h{0.0};
  for (double a : e)
    for (double b : f) {
      double x, y;
      two_prod(a, b, x, y);
      h = grow(grow(h, y), x);
    }
  return compress(h);
}
static inline Exp diff(double a, double b) {
  double x, y;
  two_sum(a, -b, x, y);
  Exp h;
  if (y != 0.0) h.push_back(y);
  h.push_back(x);
  return h;
}
static inline int sign_of(const Exp& e) {
  for (int i = (int)e.size() - 1; i >= 0; --i)
    if (e[i] != 0.0) return e[i] > 0 ? 1 : -1;
  return 0;
}

// Grow-Expansion on a fixed-size buffer: h (length n) += b, zero components dropped.
static inline int grow_fixed(double* h, int n, double b) {
  double q = b;
  int k = 0;
  for (int i = 0; i < n; ++i) {
    double s, t;
    two_sum(q, h[i], s, t);
    if (t != 0.0) h[k++] = t;
    q = s;
  }
  h[k++] = q;
  return k;
}

static int orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  // (bx-ax)(cy-ay) - (by-ay)(cx-ax) expanded into six raw products.
  const double p[6][2] = {{bx, cy}, {ax, by}, {cx, ay}, {bx, ay}, {cx, by}, {ax, cy}};
  const int s[6] = {+1, +1, +1, -1, -1, -1};
  double h[16];
  int n = 0;
  for (int k = 0; k < 6; ++k) {
    double x, y;
    two_prod(p[k][0], p[k][1], x, y);
    if (s[k] < 0) {
      x = -x;
      y = -y;
    }
    n = grow_fixed(h, n, y);
    n = grow_fixed(h, n, x);
  }
  for (int i = n - 1; i >= 0; --i)
    if (h[i] != 0.0) return h[i] > 0 ? 1 : -1;
  return 0;
}

static inline int orient(double ax, double ay, double bx, double by, double cx, double cy) {
  const double l = (bx - ax) * (cy - ay);
  const double r = (by - ay) * (cx - ax);
  const double det = l - r;
  const double sum = std::fabs(l) + std::fabs(r);
  // Two rounded differences, two rounded products, one rounded difference: error < 3u(1+4u)sum.
  if (std::fabs(det) > 4.0 * kU * sum && sum > 1e-280) return det > 0 ? 1 : -1;
  return orient_exact(ax, ay, bx, by, cx, cy);
}

static int incircle_exact(double ax, double ay, double bx, double by, double cx, double cy,
                          double dx, double dy) {
  const Exp adx = diff(ax, dx), ady = diff(ay, dy);
  const Exp bdx = diff(bx, dx), bdy = diff(by, dy);
  const Exp cdx = diff(cx, dx), cdy = diff(cy, dy);
  const Exp alift = add(mul(adx, adx), mul(ady, ady));
  const Exp blift = add(mul(bdx, bdx), mul(bdy, bdy));
  const Exp clift = add(mul(cdx, cdx), mul(cdy, cdy));
  const Exp bc = add(mul(bdx, cdy), neg(mul(cdx, bdy)));
  const Exp ca = add(mul(cdx, ady), neg(mul(adx, cdy)));
  const Exp ab = add(mul(adx, bdy), neg(mul(bdx, ady)));
  const Exp det = add(add(mul(alift, bc), mul(blift, ca)), mul(clift, ab));
  return sign_of(det);
}

static inline int incircle(double ax, double ay, double bx, double by, double cx, double cy,
                           double dx, double dy) {
  const double adx = ax - dx, ady = ay - dy;
  const double bdx = bx - dx, bdy = by - dy;
  const double cdx = cx - dx, cdy = cy - dy;
  const double bdxcdy = bdx * cdy, cdxbdy = cdx * bdy;
  const double alift = adx * adx + ady * ady;
  const double cdxady = cdx * ady, adxcdy = adx * cdy;
  const double blift = bdx * bdx + bdy * bdy;
  const double adxbdy = adx * bdy, bdxady = bdx * ady;
  const double clift = cdx * cdx + cdy * cdy;
  const double det = alift * (bdxcdy - cdxbdy) + blift * (cdxady - adxcdy) + clift * (adxbdy - bdxady);
  const double perm = (std::fabs(bdxcdy) + std::fabs(cdxbdy)) * alift +
                      (std::fabs(cdxady) + std::fabs(adxcdy)) * blift +
                      (std::fabs(adxbdy) + std::fabs(bdxady)) * clift;
  // Shewchuk's bound for this evaluation order is (10 + 96u)u * perm; 12u leaves margin.
  if (std::fabs(det) > 12.0 * kU * perm && perm > 1e-250) return det > 0 ? 1 : -1;
  return incircle_exact(ax, ay, bx, by, cx, cy, dx, dy);
}

}  // namespace pred
}  // namespace sg
