/*
 * Checker for the stackless triangulation ray walk (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, obviously correct CPU code. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the walk library never does, and the two share no code.
 *
 * What the walk computes (paper, Sec. 5.1 "Ray Traversal"): a ray that starts inside a known
 * triangle finds the edge of that triangle it leaves through; if that edge belongs to the scene
 * geometry the closest hit is found, if no triangle lies across it the ray leaves the structure
 * (no hit), otherwise the walk continues in the triangle across the edge. Sec. 5.4 counts one
 * operation per visited triangle: picking the exit edge. So for a ray R(s) = o + s d:
 *
 *   hit_prim = the primitive whose constrained edge the ray crosses first at s > 0
 *              (-1 if it first leaves through an unconstrained hull edge),
 *   t        = the crossing parameter, computed from the primitive's own segment (a, b) as
 *              t = ((ax-ox)*ey - (ay-oy)*ex) / (dx*ey - dy*ex),  e = b - a,
 *              in IEEE binary64 in exactly this order with no fused operations,
 *   steps    = 1 + the number of interior unconstrained edges crossed before that.
 *
 * The paper only asks for consistent, stable decisions (Sec. 5.1). This checker takes them
 * exactly: side(v) = sign of D(v) = dx*(vy-oy) - dy*(vx-ox) on the binary64 inputs, with D = 0
 * counted as LEFT (the ray shifted infinitesimally to its right; a symbolic perturbation that
 * leaves every other decision unchanged). All signs are decided with exact integer arithmetic:
 * every binary64 number is m * 2^e with an integer m < 2^53, so a sum of products of such numbers
 * is an integer times a power of two, summed here limb by limb.
 *
 * Entry points:
 *   oracle_walk        the walk itself, step by step in the paper's order, with a step limit:
 *                      a ray whose walk would enter more than max_steps triangles (at most
 *                      the triangle count, which an exact walk never exceeds) stops with -2 and
 *                      steps = max_steps (a guard the library exposes; not in the paper);
 *   oracle_brute_edges the definition above, by brute force over every triangulation edge;
 *   oracle_brute_prims hit_prim and t by brute force over every primitive (no triangulation);
 *   oracle_validate    triangulation checks (orientation, adjacency, Euler, constrained
 *                      Delaunay, constrained edges covering their primitives).
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ exact arithmetic */

#define MAXF 4          /* factors per product */
#define LIMBS 300       /* 32-bit limbs: enough for 4-factor products over the full exponent range */

typedef struct {
  int sign;             /* +1 or -1 */
  int k;                /* number of factors */
  double f[MAXF];
} term_t;

/* x = m * 2^e with integer 0 <= m < 2^53 (x finite). */
static void split_double(double x, uint64_t *m, int *e) {
  int ex;
  double fr = frexp(fabs(x), &ex); /* |x| = fr * 2^ex, fr in [0.5, 1) or 0 */
  *m = (uint64_t)ldexp(fr, 53);    /* exact: a binary64 significand has at most 53 bits */
  *e = ex - 53;
}

/* a (na limbs) *= small (< 2^32); returns new length */
static int bn_mul_small(uint32_t *a, int na, uint32_t small) {
  uint64_t carry = 0;
  for (int i = 0; i < na; ++i) {
    uint64_t p = (uint64_t)a[i] * small + carry;
    a[i] = (uint32_t)p;
    carry = p >> 32;
  }
  if (carry) a[na++] = (uint32_t)carry;
  return na;
}

/* acc (nacc limbs) += a (na limbs) << shift bits */
static void bn_add_shifted(uint32_t *acc, int nacc, const uint32_t *a, int na, int shift) {
  const int lw = shift / 32, lb = shift % 32;
  uint64_t carry = 0;
  for (int i = 0; i <= na; ++i) {
    const uint64_t cur = i < na ? a[i] : 0;
    const uint64_t prev = i > 0 ? a[i - 1] : 0;
    const uint32_t limb = lb ? (uint32_t)((cur << lb) | (prev >> (32 - lb))) : (uint32_t)cur;
    const uint64_t s = (uint64_t)acc[lw + i] + limb + carry;
    acc[lw + i] = (uint32_t)s;
    carry = s >> 32;
  }
  for (int i = lw + na + 1; carry && i < nacc; ++i) {
    const uint64_t s = (uint64_t)acc[i] + carry;
    acc[i] = (uint32_t)s;
    carry = s >> 32;
  }
}

static int bn_cmp(const uint32_t *a, const uint32_t *b, int n) {
  for (int i = n - 1; i >= 0; --i) {
    if (a[i] != b[i]) return a[i] > b[i] ? 1 : -1;
  }
  return 0;
}

/* Exact sign of sum_i sign_i * prod_j f_ij. */
static int exact_sign(const term_t *terms, int nterms) {
  uint32_t mant[64][8];
  int nl[64], ex[64], neg[64];
  int emin = 1 << 30, used = 0;
  if (nterms > 64) abort();
  for (int i = 0; i < nterms; ++i) {
    int zero = 0, e = 0, s = terms[i].sign;
    uint32_t *a = mant[used];
    int na = 1;
    a[0] = 1;
    for (int j = 0; j < terms[i].k; ++j) {
      double f = terms[i].f[j];
      if (f == 0.0) { zero = 1; break; }
      if (f < 0) s = -s;
      uint64_t m; int fe;
      split_double(f, &m, &fe);
      /* a *= m, with m split into two 32-bit halves: a*lo + (a*hi << 32) */
      uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
      uint32_t t1[8] = {0}, t2[9] = {0};
      memcpy(t1, a, sizeof(uint32_t) * na);
      memcpy(t2 + 1, a, sizeof(uint32_t) * na);
      int n1 = bn_mul_small(t1, na, lo);
      int n2 = bn_mul_small(t2 + 1, na, hi) + 1;
      uint32_t r[9] = {0};
      uint64_t c = 0;
      int nr = n1 > n2 ? n1 : n2;
      for (int q = 0; q < nr; ++q) {
        uint64_t sum = (uint64_t)(q < n1 ? t1[q] : 0) + (q < n2 ? t2[q] : 0) + c;
        r[q] = (uint32_t)sum;
        c = sum >> 32;
      }
      if (c) r[nr++] = (uint32_t)c;
      while (nr > 1 && r[nr - 1] == 0) --nr;
      memcpy(a, r, sizeof(uint32_t) * nr);
      na = nr;
      e += fe;
    }
    if (zero) continue;
    nl[used] = na;
    ex[used] = e;
    neg[used] = s < 0;
    if (e < emin) emin = e;
    ++used;
  }
  if (used == 0) return 0;
  int top = 0;
  for (int i = 0; i < used; ++i) {
    int bits = (ex[i] - emin) + 32 * nl[i];
    if (bits > top) top = bits;
  }
  int n = top / 32 + 3;
  if (n > LIMBS) abort();
  uint32_t pos[LIMBS], negs[LIMBS];
  memset(pos, 0, sizeof(uint32_t) * n);
  memset(negs, 0, sizeof(uint32_t) * n);
  for (int i = 0; i < used; ++i)
    bn_add_shifted(neg[i] ? negs : pos, n, mant[i], nl[i], ex[i] - emin);
  return bn_cmp(pos, negs, n);
}

static term_t T2(int s, double a, double b) { term_t t = {s, 2, {a, b, 0, 0}}; return t; }
static term_t T4(int s, double a, double b, double c, double d) {
  term_t t = {s, 4, {a, b, c, d}};
  return t;
}

/* sign of D(v) = dx*(vy-oy) - dy*(vx-ox) = dx*vy - dx*oy - dy*vx + dy*ox */
int oracle_side_sign(const double *o, const double *d, const double *v) {
  term_t t[4] = {T2(+1, d[0], v[1]), T2(-1, d[0], o[1]), T2(-1, d[1], v[0]), T2(+1, d[1], o[0])};
  return exact_sign(t, 4);
}

/* sign of (b-a) x (c-a) = bx*cy - bx*ay - ax*cy - by*cx + by*ax + ay*cx */
int oracle_orient(const double *a, const double *b, const double *c) {
  term_t t[6] = {T2(+1, b[0], c[1]), T2(-1, b[0], a[1]), T2(-1, a[0], c[1]),
                 T2(-1, b[1], c[0]), T2(+1, b[1], a[0]), T2(+1, a[1], c[0])};
  return exact_sign(t, 6);
}

/* Lifted 4x4 determinant |x y x^2+y^2 1| over rows a,b,c,d: positive iff d lies inside the
 * circle through the counter-clockwise triangle a,b,c. Expanded along the column of ones into
 * four 3x3 minors, each a sum of twelve degree-4 monomials. */
static int minor3(term_t *out, int sgn, const double *p1, const double *p2, const double *p3) {
  const double x1 = p1[0], y1 = p1[1], x2 = p2[0], y2 = p2[1], x3 = p3[0], y3 = p3[1];
  /* x1(y2 l3 - y3 l2) - y1(x2 l3 - x3 l2) + l1(x2 y3 - x3 y2), l = x^2 + y^2 */
  term_t t[12] = {
      T4(+sgn, x1, y2, x3, x3), T4(+sgn, x1, y2, y3, y3), T4(-sgn, x1, y3, x2, x2), T4(-sgn, x1, y3, y2, y2),
      T4(-sgn, y1, x2, x3, x3), T4(-sgn, y1, x2, y3, y3), T4(+sgn, y1, x3, x2, x2), T4(+sgn, y1, x3, y2, y2),
      T4(+sgn, x1, x1, x2, y3), T4(+sgn, y1, y1, x2, y3), T4(-sgn, x1, x1, x3, y2), T4(-sgn, y1, y1, x3, y2)};
  memcpy(out, t, sizeof(t));
  return 12;
}
int oracle_incircle(const double *a, const double *b, const double *c, const double *d) {
  term_t t[48];
  int n = 0;
  /* cofactor signs (-1)^(r+3) for rows r = 0..3 of the column of ones */
  n += minor3(t + n, -1, b, c, d); /* delete row a */
  n += minor3(t + n, +1, a, c, d); /* delete row b */
  n += minor3(t + n, -1, a, b, d); /* delete row c */
  n += minor3(t + n, +1, a, b, c); /* delete row d */
  return exact_sign(t, n);
}

/* An edge p->q crossed by the ray, oriented from its RIGHT endpoint p to its LEFT endpoint q.
 * The crossing parameter is s = num/den with num = (px-ox)(qy-py) - (py-oy)(qx-px) and
 * den = dx(qy-py) - dy(qx-px) > 0. Under the rightward shift by eps the parameter becomes
 * s - eps * (d.(q-p)) / den, which orders crossings that coincide at eps = 0. */
typedef struct { const double *p, *q; } xedge_t;

/* num*den' as monomials of degree 4: num has 6 monomials, den' has 4 */
static int num_den(term_t *out, int sgn, const double *o, const xedge_t *a, const double *d,
                   const xedge_t *b) {
  const double *p = a->p, *q = a->q;
  /* num(a) = px*qy - ox*qy + ox*py - py*qx + oy*qx - oy*px */
  const double nm[6][2] = {{p[0], q[1]}, {o[0], q[1]}, {o[0], p[1]}, {p[1], q[0]}, {o[1], q[0]}, {o[1], p[0]}};
  const int ns[6] = {+1, -1, +1, -1, +1, -1};
  /* den(b) = dx*qy - dx*py - dy*qx + dy*px */
  const double dn[4][2] = {{d[0], b->q[1]}, {d[0], b->p[1]}, {d[1], b->q[0]}, {d[1], b->p[0]}};
  const int ds[4] = {+1, -1, -1, +1};
  int n = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 4; ++j) out[n++] = T4(sgn * ns[i] * ds[j], nm[i][0], nm[i][1], dn[j][0], dn[j][1]);
  return n;
}
/* dot(d, q-p) * den' as degree-4 monomials */
static int dot_den(term_t *out, int sgn, const double *d, const xedge_t *a, const xedge_t *b) {
  const double dt[4][2] = {{d[0], a->q[0]}, {d[0], a->p[0]}, {d[1], a->q[1]}, {d[1], a->p[1]}};
  const int dts[4] = {+1, -1, +1, -1};
  const double dn[4][2] = {{d[0], b->q[1]}, {d[0], b->p[1]}, {d[1], b->q[0]}, {d[1], b->p[0]}};
  const int ds[4] = {+1, -1, -1, +1};
  int n = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[n++] = T4(sgn * dts[i] * ds[j], dt[i][0], dt[i][1], dn[j][0], dn[j][1]);
  return n;
}
/* -1 if the perturbed ray crosses a before b, +1 if after, 0 if the same crossing. */
static int cross_order(const double *o, const double *d, const xedge_t *a, const xedge_t *b) {
  term_t t[48];
  int n = 0;
  n += num_den(t + n, +1, o, a, d, b); /* num_a den_b - num_b den_a  ~  s_a - s_b */
  n += num_den(t + n, -1, o, b, d, a);
  int s = exact_sign(t, n);
  if (s != 0) return s;
  /* equal at eps = 0: s_a(eps) - s_b(eps) ~ -(dot_a den_b - dot_b den_a) */
  n = 0;
  n += dot_den(t + n, +1, d, a, b);
  n += dot_den(t + n, -1, d, b, a);
  return -exact_sign(t, n);
}

static int is_left(const double *o, const double *d, const double *v) {
  return oracle_side_sign(o, d, v) >= 0;
}

/* The fixed hit-distance formula (no contraction: the file is built with -ffp-contract=off). */
double oracle_t(const double *o, const double *d, const double *seg) {
  const double ex = seg[2] - seg[0];
  const double ey = seg[3] - seg[1];
  const double num = (seg[0] - o[0]) * ey - (seg[1] - o[1]) * ex;
  const double den = d[0] * ey - d[1] * ex;
  return num / den;
}

/* ------------------------------------------------------------------ the walk (Sec. 5.1) */

static const double *VX(const oracle_tri_t *m, int v) { return m->xy + 2 * (int64_t)v; }

static void walk_one(const oracle_tri_t *m, const double *o, const double *d, int32_t start,
                     int64_t max_steps, int32_t *prim, double *t, int32_t *steps) {
  *prim = -3;
  *t = INFINITY;
  *steps = 0;
  if (start < 0 || start >= m->nt) return;
  int tri = start;
  const int32_t *tv = m->tri_v + 3 * (int64_t)tri;
  /* precondition: the origin lies strictly inside the start triangle */
  for (int i = 0; i < 3; ++i)
    if (oracle_orient(VX(m, tv[(i + 1) % 3]), VX(m, tv[(i + 2) % 3]), o) <= 0) return;
  /* first triangle: the exit edge i has its first endpoint RIGHT and its second LEFT */
  int left[3], exit_edge = -1;
  for (int i = 0; i < 3; ++i) left[i] = is_left(o, d, VX(m, tv[i]));
  for (int i = 0; i < 3; ++i)
    if (!left[(i + 1) % 3] && left[(i + 2) % 3]) exit_edge = i;
  if (exit_edge < 0) return;
  int64_t count = 1;
  for (;;) {
    const int64_t slot = 3 * (int64_t)tri + exit_edge;
    if (m->tri_prim[slot] >= 0) { /* the exit edge is scene geometry: closest hit */
      *prim = m->tri_prim[slot];
      *t = oracle_t(o, d, m->prim + 4 * (int64_t)*prim);
      break;
    }
    const int32_t nb = m->tri_nbr[slot];
    if (nb < 0) { /* no triangle across: the ray leaves the structure */
      *prim = -1;
      break;
    }
    /* the step guard: the walk would enter triangle max_steps + 1 */
    if (count >= max_steps) {
      *prim = -2;
      break;
    }
    /* continue in the neighbour, entered through its edge back to tri */
    int back = -1;
    for (int j = 0; j < 3; ++j)
      if (m->tri_nbr[3 * (int64_t)nb + j] == tri) back = j;
    if (back < 0) return;
    tri = nb;
    ++count;
    tv = m->tri_v + 3 * (int64_t)tri;
    /* the entry edge's endpoints are LEFT (first) and RIGHT (second); only the vertex across
     * decides between the two remaining edges */
    exit_edge = is_left(o, d, VX(m, tv[back])) ? (back + 1) % 3 : (back + 2) % 3;
  }
  *steps = (int32_t)count;
}

int oracle_walk(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                const int32_t *start, int64_t max_steps, int32_t *prim, double *t,
                int32_t *steps, int nthreads) {
  const int64_t limit = (max_steps <= 0 || max_steps > m->nt) ? m->nt : max_steps;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static, 4096)
#endif
  for (int64_t r = 0; r < n; ++r)
    walk_one(m, o + 2 * r, d + 2 * r, start[r], limit, prim + r, t + r, steps + r);
  (void)nthreads;
  return 0;
}

/* ------------------------------------------------------------------ continuation (Sec. 5.2) */

/* Specular reflection at a hit of primitive seg = (a, b) at parameter t: the new origin is
 * o + t d, the new direction d - k n with n = (-ey, ex), e = b - a, the segment's normal, and
 * k = 2 (d . n) / (n . n); binary64, in exactly this order, no fused operations. */
static void reflect(const double *o, const double *d, const double *seg, double t, double *o2,
                    double *d2) {
  const double ex = seg[2] - seg[0], ey = seg[3] - seg[1];
  const double nx = -ey, ny = ex;
  const double dn = d[0] * nx + d[1] * ny;
  const double nn = nx * nx + ny * ny;
  const double k = (2.0 * dn) / nn;
  o2[0] = o[0] + t * d[0];
  o2[1] = o[1] + t * d[1];
  d2[0] = d[0] - k * nx;
  d2[1] = d[1] - k * ny;
}

/* The walk of oracle_walk, continued at hits: while fewer than max_bounces reflections have been
 * made, a hit reflects the ray off its primitive and the walk goes on from the hit point in the
 * triangle it ended in (the final triangle of a traversal starts the secondary ray), which the
 * reflected ray enters through the hit edge, so only the vertex across that edge decides the
 * exit. Outputs: the last segment's primitive (-1 miss, -2 a segment longer than the step guard,
 * -3 bad start), its t, the triangles visited over all segments (the hit triangle counts in both
 * segments), the reflections made and the last segment's hit face (4 * triangle + edge, -1 if
 * it did not hit). */
static void bounce_one(const oracle_tri_t *m, const double *o_in, const double *d_in,
                       int32_t start, int32_t max_bounces, int64_t max_steps, int32_t *prim,
                       double *t, int32_t *steps, int32_t *hits, int32_t *face) {
  *prim = -3;
  *t = INFINITY;
  *steps = 0;
  *hits = 0;
  *face = -1;
  if (start < 0 || start >= m->nt) return;
  double o[2] = {o_in[0], o_in[1]}, d[2] = {d_in[0], d_in[1]};
  int tri = start;
  const int32_t *tv = m->tri_v + 3 * (int64_t)tri;
  for (int i = 0; i < 3; ++i)
    if (oracle_orient(VX(m, tv[(i + 1) % 3]), VX(m, tv[(i + 2) % 3]), o) <= 0) return;
  int left[3], exit_edge = -1;
  for (int i = 0; i < 3; ++i) left[i] = is_left(o, d, VX(m, tv[i]));
  for (int i = 0; i < 3; ++i)
    if (!left[(i + 1) % 3] && left[(i + 2) % 3]) exit_edge = i;
  if (exit_edge < 0) return;
  int64_t count = 1, seg_count = 1;
  const int64_t guard = max_steps;
  int32_t nb = 0;
  for (;;) {
    const int64_t slot = 3 * (int64_t)tri + exit_edge;
    if (m->tri_prim[slot] >= 0) {
      const int32_t p = m->tri_prim[slot];
      const double *seg = m->prim + 4 * (int64_t)p;
      const double th = oracle_t(o, d, seg);
      if (nb < max_bounces) {
        double o2[2], d2[2];
        reflect(o, d, seg, th, o2, d2);
        o[0] = o2[0];
        o[1] = o2[1];
        d[0] = d2[0];
        d[1] = d2[1];
        ++nb;
        ++count;
        seg_count = 1;
        /* the reflected ray enters this triangle through the hit edge */
        exit_edge = is_left(o, d, VX(m, tv[exit_edge])) ? (exit_edge + 1) % 3 : (exit_edge + 2) % 3;
        continue;
      }
      *prim = p;
      *t = th;
      *face = (int32_t)(4 * (int64_t)tri + exit_edge);
      break;
    }
    const int32_t nbr = m->tri_nbr[slot];
    if (nbr < 0) {
      *prim = -1;
      break;
    }
    if (seg_count >= guard) { /* this segment would enter triangle max_steps + 1 */
      *prim = -2;
      break;
    }
    int back = -1;
    for (int j = 0; j < 3; ++j)
      if (m->tri_nbr[3 * (int64_t)nbr + j] == tri) back = j;
    if (back < 0) return;
    tri = nbr;
    ++count;
    ++seg_count;
    tv = m->tri_v + 3 * (int64_t)tri;
    exit_edge = is_left(o, d, VX(m, tv[back])) ? (back + 1) % 3 : (back + 2) % 3;
  }
  *steps = (int32_t)count;
  *hits = nb;
}

int oracle_bounce(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                  const int32_t *start, int32_t max_bounces, int64_t max_steps, int32_t *prim,
                  double *t, int32_t *steps, int32_t *hits, int32_t *face, int nthreads) {
  const int64_t limit = (max_steps <= 0 || max_steps > m->nt) ? m->nt : max_steps;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
  for (int64_t r = 0; r < n; ++r)
    bounce_one(m, o + 2 * r, d + 2 * r, start[r], max_bounces, limit, prim + r, t + r,
               steps + r, hits + r, face + r);
  (void)nthreads;
  return 0;
}

/* ------------------------------------------------------------------ point location (Sec. 5.2) */

/* The triangle containing q, by definition: q is in the closed triangle (a, b, c) (counter-
 * clockwise) iff orient(b, c, q), orient(c, a, q) and orient(a, b, q) are all >= 0, and strictly
 * inside iff all are > 0. Every triangle is tried in index order; a bounding-box comparison
 * (exact: coordinates are only compared) skips the ones that cannot contain q. */
int oracle_locate(const oracle_tri_t *m, int64_t n, const double *q, int32_t *tri,
                  int32_t *status, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n; ++k) {
    const double *p = q + 2 * k;
    tri[k] = -1;
    status[k] = -1;
    if (!isfinite(p[0]) || !isfinite(p[1])) {
      status[k] = -2;
      continue;
    }
    for (int64_t t = 0; t < m->nt; ++t) {
      const double *a = m->xy + 2 * (int64_t)m->tri_v[3 * t];
      const double *b = m->xy + 2 * (int64_t)m->tri_v[3 * t + 1];
      const double *c = m->xy + 2 * (int64_t)m->tri_v[3 * t + 2];
      if (p[0] < fmin(a[0], fmin(b[0], c[0])) || p[0] > fmax(a[0], fmax(b[0], c[0])) ||
          p[1] < fmin(a[1], fmin(b[1], c[1])) || p[1] > fmax(a[1], fmax(b[1], c[1])))
        continue;
      const int s0 = oracle_orient(b, c, p), s1 = oracle_orient(c, a, p), s2 = oracle_orient(a, b, p);
      if (s0 >= 0 && s1 >= 0 && s2 >= 0) {
        tri[k] = (int32_t)t;
        status[k] = (s0 > 0 && s1 > 0 && s2 > 0) ? 0 : 1;
        break;
      }
    }
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ brute force */

/* Classify edge (a,b) against the ray: returns 1 and fills e (oriented RIGHT -> LEFT) if the
 * perturbed ray crosses it ahead of the origin, 0 if not, -1 if the origin lies on it. */
static int crossing(const double *o, const double *d, const double *a, const double *b,
                    xedge_t *e) {
  const int la = is_left(o, d, a), lb = is_left(o, d, b);
  if (la == lb) return 0;
  e->p = la ? b : a;
  e->q = la ? a : b;
  const int s = oracle_orient(o, e->p, e->q); /* sign of num: the crossing is ahead iff > 0 */
  if (s == 0) return -1;
  return s > 0;
}

int oracle_brute_edges(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                       int32_t *prim, double *t, int32_t *steps, int nthreads) {
  int status = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : status)
#endif
  for (int64_t r = 0; r < n; ++r) {
    const double *ro = o + 2 * r, *rd = d + 2 * r;
    xedge_t best = {0, 0};
    int64_t best_slot = -1;
    /* first terminating edge (constrained, or unconstrained on the hull) */
    for (int64_t s = 0; s < 3 * m->nt; ++s) {
      const int64_t tri = s / 3;
      const int i = (int)(s % 3);
      const int32_t nb = m->tri_nbr[s];
      if (!(m->tri_prim[s] >= 0 || nb < 0)) continue;
      if (nb >= 0 && nb < tri) continue; /* a constrained interior edge is visited once */
      const int32_t *tv = m->tri_v + 3 * tri;
      xedge_t e;
      const int c = crossing(ro, rd, VX(m, tv[(i + 1) % 3]), VX(m, tv[(i + 2) % 3]), &e);
      if (c < 0) status |= 1;
      if (c <= 0) continue;
      if (best_slot < 0 || cross_order(ro, rd, &e, &best) < 0) {
        best = e;
        best_slot = s;
      }
    }
    int64_t count = 1;
    for (int64_t s = 0; s < 3 * m->nt; ++s) {
      const int64_t tri = s / 3;
      const int i = (int)(s % 3);
      const int32_t nb = m->tri_nbr[s];
      if (m->tri_prim[s] >= 0 || nb < 0 || nb < tri) continue; /* interior unconstrained, once */
      const int32_t *tv = m->tri_v + 3 * tri;
      xedge_t e;
      const int c = crossing(ro, rd, VX(m, tv[(i + 1) % 3]), VX(m, tv[(i + 2) % 3]), &e);
      if (c < 0) status |= 1;
      if (c <= 0) continue;
      if (best_slot < 0 || cross_order(ro, rd, &e, &best) < 0) ++count;
    }
    steps[r] = (int32_t)count;
    if (best_slot < 0) { /* no terminating edge ahead: only possible for a malformed input */
      prim[r] = -3;
      t[r] = INFINITY;
      status |= 2;
    } else if (m->tri_prim[best_slot] >= 0) {
      prim[r] = m->tri_prim[best_slot];
      t[r] = oracle_t(ro, rd, m->prim + 4 * (int64_t)prim[r]);
    } else {
      prim[r] = -1;
      t[r] = INFINITY;
    }
  }
  return status;
}

int oracle_brute_prims(int64_t np, const double *pseg, int64_t n, const double *o,
                       const double *d, int32_t *prim, double *t, int nthreads) {
  int status = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : status)
#endif
  for (int64_t r = 0; r < n; ++r) {
    const double *ro = o + 2 * r, *rd = d + 2 * r;
    xedge_t best = {0, 0};
    int64_t bk = -1;
    for (int64_t k = 0; k < np; ++k) {
      xedge_t e;
      const int c = crossing(ro, rd, pseg + 4 * k, pseg + 4 * k + 2, &e);
      if (c < 0) status |= 1;
      if (c <= 0) continue;
      if (bk < 0 || cross_order(ro, rd, &e, &best) < 0) {
        best = e;
        bk = k;
      }
    }
    prim[r] = bk < 0 ? -1 : (int32_t)bk;
    t[r] = bk < 0 ? INFINITY : oracle_t(ro, rd, pseg + 4 * bk);
  }
  return status;
}

/* ------------------------------------------------------------------ triangulation checks */

static int fail(char *msg, int len, const char *what, int64_t a, int64_t b) {
  if (msg && len > 0) snprintf(msg, (size_t)len, "%s (%lld, %lld)", what, (long long)a, (long long)b);
  return 1;
}

int oracle_validate(const oracle_tri_t *m, int check_delaunay, char *msg, int msglen) {
  const int64_t T = m->nt, V = m->nv;
  int64_t e_int2 = 0, e_bnd = 0;
  char *used = calloc((size_t)V, 1);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t *tv = m->tri_v + 3 * t;
    for (int i = 0; i < 3; ++i) {
      if (tv[i] < 0 || tv[i] >= V) { free(used); return fail(msg, msglen, "vertex id out of range", t, i); }
      used[tv[i]] = 1;
    }
    if (oracle_orient(VX(m, tv[0]), VX(m, tv[1]), VX(m, tv[2])) <= 0) {
      free(used);
      return fail(msg, msglen, "triangle not counter-clockwise", t, 0);
    }
    for (int i = 0; i < 3; ++i) {
      const int32_t nb = m->tri_nbr[3 * t + i];
      const int32_t pr = m->tri_prim[3 * t + i];
      if (pr >= m->np || pr < -1) { free(used); return fail(msg, msglen, "primitive id out of range", t, i); }
      if (nb < 0) { ++e_bnd; continue; }
      if (nb >= T) { free(used); return fail(msg, msglen, "neighbour out of range", t, i); }
      ++e_int2;
      int back = -1, hits = 0;
      for (int j = 0; j < 3; ++j)
        if (m->tri_nbr[3 * (int64_t)nb + j] == t) { back = j; ++hits; }
      if (hits != 1) { free(used); return fail(msg, msglen, "adjacency not symmetric", t, i); }
      const int32_t *nv = m->tri_v + 3 * (int64_t)nb;
      if (nv[(back + 1) % 3] != tv[(i + 2) % 3] || nv[(back + 2) % 3] != tv[(i + 1) % 3]) {
        free(used);
        return fail(msg, msglen, "shared edge does not match", t, i);
      }
      if (m->tri_prim[3 * (int64_t)nb + back] != pr) {
        free(used);
        return fail(msg, msglen, "constraint differs across an edge", t, i);
      }
      if (check_delaunay && pr < 0) {
        if (oracle_incircle(VX(m, tv[0]), VX(m, tv[1]), VX(m, tv[2]), VX(m, nv[back])) > 0) {
          free(used);
          return fail(msg, msglen, "unconstrained edge not locally Delaunay", t, i);
        }
      }
    }
  }
  for (int64_t v = 0; v < V; ++v)
    if (!used[v]) { free(used); return fail(msg, msglen, "vertex not used", v, 0); }
  free(used);
  const int64_t E = e_int2 / 2 + e_bnd;
  if (e_int2 % 2 != 0) return fail(msg, msglen, "odd interior edge count", e_int2, 0);
  if (V - E + T != 1) return fail(msg, msglen, "Euler characteristic V - E + T != 1", V - E + T, 0);
  if (3 * T != e_int2 + e_bnd) return fail(msg, msglen, "3T != 2 E_int + E_bnd", 3 * T, e_int2 + e_bnd);
  /* constrained edges: collinear with and inside their primitive, covering it from end to end.
   * Edges are first grouped by primitive (counting sort), each edge listed once. */
  int64_t *first = calloc((size_t)m->np + 1, sizeof(int64_t));
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) {
      const int32_t pr = m->tri_prim[3 * t + i], nb = m->tri_nbr[3 * t + i];
      if (pr >= 0 && !(nb >= 0 && nb < t)) ++first[pr + 1];
    }
  for (int64_t k = 0; k < m->np; ++k) first[k + 1] += first[k];
  int64_t *slots = malloc(sizeof(int64_t) * (size_t)(first[m->np] + 1));
  int64_t *fill = malloc(sizeof(int64_t) * (size_t)(m->np + 1));
  memcpy(fill, first, sizeof(int64_t) * (size_t)(m->np + 1));
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) {
      const int32_t pr = m->tri_prim[3 * t + i], nb = m->tri_nbr[3 * t + i];
      if (pr >= 0 && !(nb >= 0 && nb < t)) slots[fill[pr]++] = 3 * t + i;
    }
  int bad = 0;
  for (int64_t k = 0; k < m->np && !bad; ++k) {
    const double *a = m->prim + 4 * k, *b = a + 2;
    double len = 0.0;
    int ends_a = 0, ends_b = 0;
    if (first[k + 1] == first[k]) { bad = fail(msg, msglen, "primitive not covered by constrained edges", k, 0); break; }
    for (int64_t q = first[k]; q < first[k + 1]; ++q) {
      const int64_t t = slots[q] / 3;
      const int i = (int)(slots[q] % 3);
      const double *p = VX(m, m->tri_v[3 * t + (i + 1) % 3]);
      const double *r = VX(m, m->tri_v[3 * t + (i + 2) % 3]);
      if (oracle_orient(a, b, p) != 0 || oracle_orient(a, b, r) != 0) {
        bad = fail(msg, msglen, "constrained edge off its primitive", k, t);
        break;
      }
      for (int w = 0; w < 2; ++w) {
        const double *x = w ? r : p;
        const double lo0 = fmin(a[0], b[0]), hi0 = fmax(a[0], b[0]);
        const double lo1 = fmin(a[1], b[1]), hi1 = fmax(a[1], b[1]);
        if (x[0] < lo0 || x[0] > hi0 || x[1] < lo1 || x[1] > hi1) {
          bad = fail(msg, msglen, "constrained edge outside its primitive", k, t);
          break;
        }
        if (x[0] == a[0] && x[1] == a[1]) ++ends_a;
        if (x[0] == b[0] && x[1] == b[1]) ++ends_b;
      }
      if (bad) break;
      len += hypot(r[0] - p[0], r[1] - p[1]);
    }
    if (bad) break;
    if (ends_a != 1 || ends_b != 1) { bad = fail(msg, msglen, "primitive ends not covered once", k, 0); break; }
    const double full = hypot(b[0] - a[0], b[1] - a[1]);
    if (fabs(len - full) > 1e-9 * (1.0 + full)) {
      bad = fail(msg, msglen, "constrained edges do not cover primitive", k, first[k + 1] - first[k]);
      break;
    }
  }
  free(first);
  free(slots);
  free(fill);
  if (bad) return 1;
  if (msg && msglen > 0) msg[0] = 0;
  return 0;
}
