/*
 * Checker for the 3D tetrahedral walk (TEST INFRASTRUCTURE ONLY): plain, slow CPU code that only
 * the tests and the benchmark's CPU leg may load. It shares no code with the walk library.
 *
 * The paper walks rays through triangulations in 2D and names the 3D case, a ray traversing a
 * constrained tetrahedralisation whose faces carry the scene's triangles, as the direction it
 * builds towards (Sec. 1.3: a CDT of triangle meshes; Sec. 1.4: one operation per tetrahedron,
 * four candidate exit faces, three once the entry face is discarded, and the number of
 * tetrahedra visited as the cost; Sec. 7.2). The 3D walk computes, for a ray R(s) = o + s d that
 * starts inside a known tetrahedron:
 *   hit_prim = the primitive triangle the ray crosses first at s > 0 (-1: it leaves through a
 *              hull face that is not a primitive),
 *   t        = its parameter, from the primitive's own vertices (a, b, c) as
 *              t = ((ax-ox)*nx + (ay-oy)*ny + (az-oz)*nz) / (dx*nx + dy*ny + dz*nz),
 *              n = (b - a) x (c - a), in IEEE binary64 in this order without fused operations,
 *   steps    = the number of tetrahedra visited, start and hit one included.
 * A ray off the grid below, with a zero direction, a start out of range or an origin not strictly
 * inside its start ends with code -3 and steps 0.
 *
 * Inputs live on an integer grid: vertex and origin coordinates in [0, 2^19), direction
 * components in [-2^19, 2^19], so every sign below is an exact int64 computation (a difference of
 * coordinates is below 2^20 in size, a cross product of two below 2^40, its dot product with a
 * third vector below 2^61).
 *
 * Decisions. The ray passes a directed edge (p, q) with Plücker sign pi(p, q) = sign of
 * d . ((p - o) x (q - o)). A face (a, b, c), ordered counter-clockwise as seen from outside its
 * tetrahedron, is the exit face iff pi(a,b), pi(b,c), pi(c,a) are all +. A zero value (the ray
 * meets the edge's line or runs parallel to it) is decided as for the line moved symbolically:
 * origin o + (e, e^2, e^3), direction d + (e^10, e^20, e^30) for an infinitesimal e > 0. With
 * a = q - p, c = d x a and W = (p - o) x (q - o), the value becomes
 *   d.W + e c_x + e^2 c_y + e^3 c_z + e^10 (W_x - e^2 a_z + e^3 a_y) + e^20 (W_y + e a_z - e^3 a_x)
 *   + ..., so its sign is that of the first nonzero of
 *   d.W, c_x, c_y, c_z, W_x, -a_z, a_y, W_y, a_z, -a_x,
 * which is never all zero for p != q (a_x = 0 then, and a_y or a_z is not) and stays
 * antisymmetric. The moved line is a real line, so every tetrahedron it enters has exactly one
 * exit face and the walk follows it as it would any line in general position.
 * - In the start tetrahedron the exit is the first face, in the order 0..3, whose three edges are
 *   all +.
 * - After entering through face e, w = v[e] and (p, q, r) = face e in its outside order: the exit
 *   face is the one holding w and the entry edge it shares, found with two signs as
 *   s_p = pi(w, p); if s_p = + then (pi(w, r) = - ? the face opposite q : the face opposite p)
 *   else (pi(w, q) = + ? the face opposite r : the face opposite p).
 * Faces of a positively oriented (v0, v1, v2, v3) in outside order, face i opposite v_i:
 * (1,2,3), (0,3,2), (0,1,3), (0,2,1).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t nv;
  const int32_t *xyz;      /* 3 nv */
  int64_t nt;
  const int32_t *tet_v;    /* 4 nt */
  const int32_t *tet_nbr;  /* 4 nt, -1 hull */
  const int32_t *tet_prim; /* 4 nt, -1 unless a primitive */
  int64_t np;
  const int32_t *prims;    /* 3 np vertex ids */
} oracle_tet_t;

static const int FACE[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

/* det[b - a; c - a; d - a], exact */
int64_t oracle3_orient(const int32_t *a, const int32_t *b, const int32_t *c, const int32_t *d) {
  const int64_t u0 = (int64_t)b[0] - a[0], u1 = (int64_t)b[1] - a[1], u2 = (int64_t)b[2] - a[2];
  const int64_t v0 = (int64_t)c[0] - a[0], v1 = (int64_t)c[1] - a[1], v2 = (int64_t)c[2] - a[2];
  const int64_t w0 = (int64_t)d[0] - a[0], w1 = (int64_t)d[1] - a[1], w2 = (int64_t)d[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

/* d . ((p - o) x (q - o)), exact */
int64_t oracle3_plucker(const int32_t *o, const int32_t *d, const int32_t *p, const int32_t *q) {
  const int64_t a0 = (int64_t)p[0] - o[0], a1 = (int64_t)p[1] - o[1], a2 = (int64_t)p[2] - o[2];
  const int64_t b0 = (int64_t)q[0] - o[0], b1 = (int64_t)q[1] - o[1], b2 = (int64_t)q[2] - o[2];
  const int64_t c0 = a1 * b2 - a2 * b1, c1 = a2 * b0 - a0 * b2, c2 = a0 * b1 - a1 * b0;
  return (int64_t)d[0] * c0 + (int64_t)d[1] * c1 + (int64_t)d[2] * c2;
}

static int sgn64(int64_t v) { return v > 0 ? 1 : (v < 0 ? -1 : 0); }

/* The walk's sign of the directed edge (a, b) under the symbolic move of the line (header);
 * *degen set when the unmoved value is zero. */
int oracle3_pi(const int32_t *o, const int32_t *d, const int32_t *P, const int32_t *Q, int *degen) {
  const int64_t v = oracle3_plucker(o, d, P, Q);
  if (v != 0) return sgn64(v);
  *degen = 1;
  const int64_t a0 = (int64_t)Q[0] - P[0], a1 = (int64_t)Q[1] - P[1], a2 = (int64_t)Q[2] - P[2];
  const int64_t c[3] = {(int64_t)d[1] * a2 - (int64_t)d[2] * a1, (int64_t)d[2] * a0 - (int64_t)d[0] * a2,
                        (int64_t)d[0] * a1 - (int64_t)d[1] * a0};
  for (int k = 0; k < 3; ++k)
    if (c[k] != 0) return sgn64(c[k]);
  const int64_t p0 = (int64_t)P[0] - o[0], p1 = (int64_t)P[1] - o[1], p2 = (int64_t)P[2] - o[2];
  const int64_t q0 = (int64_t)Q[0] - o[0], q1 = (int64_t)Q[1] - o[1], q2 = (int64_t)Q[2] - o[2];
  const int64_t seq[6] = {p1 * q2 - p2 * q1, -a2, a1, p2 * q0 - p0 * q2, a2, -a0};
  for (int k = 0; k < 6; ++k)
    if (seq[k] != 0) return sgn64(seq[k]);
  return 0; /* p == q */
}

static int pi_sign(const oracle_tet_t *m, const int32_t *o, const int32_t *d, int32_t a, int32_t b,
                   int *degen) {
  return oracle3_pi(o, d, m->xyz + 3 * (int64_t)a, m->xyz + 3 * (int64_t)b, degen);
}

double oracle3_t(const int32_t *o, const int32_t *d, const oracle_tet_t *m, int32_t prim) {
  const int32_t *A = m->xyz + 3 * (int64_t)m->prims[3 * (int64_t)prim];
  const int32_t *B = m->xyz + 3 * (int64_t)m->prims[3 * (int64_t)prim + 1];
  const int32_t *C = m->xyz + 3 * (int64_t)m->prims[3 * (int64_t)prim + 2];
  const double ax = A[0], ay = A[1], az = A[2];
  const double ux = B[0] - ax, uy = B[1] - ay, uz = B[2] - az;
  const double vx = C[0] - ax, vy = C[1] - ay, vz = C[2] - az;
  const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  const double num = (ax - o[0]) * nx + (ay - o[1]) * ny + (az - o[2]) * nz;
  const double den = (double)d[0] * nx + (double)d[1] * ny + (double)d[2] * nz;
  return num / den;
}

static void walk3_one(const oracle_tet_t *m, const int32_t *o, const int32_t *d, int32_t start,
                      int64_t max_steps, int32_t *prim, double *t, int32_t *steps, int32_t *degen) {
  *prim = -3;
  *t = INFINITY;
  *steps = 0;
  int dg = 0;
  int on_grid = 1;
  for (int k = 0; k < 3; ++k)
    on_grid = on_grid && o[k] >= 0 && o[k] < (1 << 19) && d[k] >= -(1 << 19) && d[k] <= (1 << 19);
  if (!on_grid || start < 0 || start >= m->nt || (d[0] == 0 && d[1] == 0 && d[2] == 0)) {
    *degen = 0;
    return;
  }
  int32_t tet = start;
  const int32_t *tv = m->tet_v + 4 * (int64_t)tet;
  /* precondition: the origin strictly inside the start tetrahedron */
  for (int i = 0; i < 4; ++i) {
    const int32_t *a = m->xyz + 3 * (int64_t)tv[FACE[i][0]], *b = m->xyz + 3 * (int64_t)tv[FACE[i][1]],
                  *c = m->xyz + 3 * (int64_t)tv[FACE[i][2]];
    if (oracle3_orient(a, b, c, o) >= 0) {
      *degen = 0;
      return;
    }
  }
  int exit_face = -1;
  for (int i = 0; i < 4 && exit_face < 0; ++i) {
    const int32_t a = tv[FACE[i][0]], b = tv[FACE[i][1]], c = tv[FACE[i][2]];
    if (pi_sign(m, o, d, a, b, &dg) > 0 && pi_sign(m, o, d, b, c, &dg) > 0 &&
        pi_sign(m, o, d, c, a, &dg) > 0)
      exit_face = i;
  }
  if (exit_face < 0) {
    *degen = dg;
    return;
  }
  int64_t count = 1;
  for (;;) {
    const int64_t slot = 4 * (int64_t)tet + exit_face;
    if (m->tet_prim[slot] >= 0) {
      *prim = m->tet_prim[slot];
      *t = oracle3_t(o, d, m, *prim);
      break;
    }
    const int32_t nb = m->tet_nbr[slot];
    if (nb < 0) {
      *prim = -1;
      break;
    }
    if (count >= max_steps) {
      *prim = -2;
      break;
    }
    int back = -1;
    for (int j = 0; j < 4; ++j)
      if (m->tet_nbr[4 * (int64_t)nb + j] == tet) back = j;
    if (back < 0) {
      *prim = -3;
      break;
    }
    tet = nb;
    ++count;
    tv = m->tet_v + 4 * (int64_t)tet;
    const int32_t w = tv[back];
    const int fp = FACE[back][0], fq = FACE[back][1], fr = FACE[back][2];
    if (pi_sign(m, o, d, w, tv[fp], &dg) > 0)
      exit_face = pi_sign(m, o, d, w, tv[fr], &dg) < 0 ? fq : fp;
    else
      exit_face = pi_sign(m, o, d, w, tv[fq], &dg) > 0 ? fr : fp;
  }
  *steps = (int32_t)count;
  *degen = dg;
}

int oracle3_walk(const oracle_tet_t *m, int64_t n, const int32_t *o, const int32_t *d,
                 const int32_t *start, int64_t max_steps, int32_t *prim, double *t, int32_t *steps,
                 int32_t *degen, int nthreads) {
  const int64_t limit = (max_steps <= 0 || max_steps > m->nt) ? m->nt : max_steps;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static, 1024)
#endif
  for (int64_t r = 0; r < n; ++r)
    walk3_one(m, o + 3 * r, d + 3 * r, start[r], limit, prim + r, t + r, steps + r, degen + r);
  (void)nthreads;
  return 0;
}

/* ---------------------------------------------------------------- brute force */

typedef struct {
  int32_t a, b, c;   /* outside order of the lower tetrahedron holding it */
  int32_t prim;      /* primitive id or -1 */
  int32_t interior;  /* 1 if a tetrahedron lies on both sides */
} face_t;

/* a / b < c / d for b, d > 0 (exact, 128-bit products) */
static int frac_less(int64_t a, int64_t b, int64_t c, int64_t d) {
  return (__int128)a * d < (__int128)c * b;
}

/*
 * The definition by brute force over every face: the ray crosses face (a, b, c) when its three
 * raw Plücker values d . ((p - o) x (q - o)) are all > 0 or all < 0, at s = num / den,
 * num = (a - o) . n, den = d . n, n = (b - a) x (c - a). hit = the primitive face crossed at the
 * smallest s > 0; steps = 1 + the interior non-primitive faces crossed at 0 < s < that. degen[r]
 * bit 0: the hit depends on how ties are broken (the ray touches a primitive's boundary ahead of
 * the origin, meets a primitive's plane at s = 0, or two primitives at the same s); bit 1: the
 * count does (the same for a face counted in steps). Only the walk's decisions define those.
 */
int oracle3_brute(const oracle_tet_t *m, int64_t n, const int32_t *o, const int32_t *d,
                  int32_t *prim, double *t, int32_t *steps, int32_t *degen, int nthreads) {
  int64_t nf = 0;
  for (int64_t k = 0; k < 4 * m->nt; ++k)
    if (m->tet_nbr[k] < 0 || m->tet_nbr[k] > k / 4) ++nf;
  face_t *f = (face_t *)malloc(sizeof(face_t) * (size_t)(nf > 0 ? nf : 1));
  if (!f) return -1;
  nf = 0;
  for (int64_t k = 0; k < 4 * m->nt; ++k) {
    const int32_t nb = m->tet_nbr[k];
    if (!(nb < 0 || nb > k / 4)) continue;
    const int32_t *tv = m->tet_v + 4 * (k / 4);
    const int i = (int)(k % 4);
    f[nf].a = tv[FACE[i][0]];
    f[nf].b = tv[FACE[i][1]];
    f[nf].c = tv[FACE[i][2]];
    f[nf].prim = m->tet_prim[k];
    f[nf].interior = nb >= 0;
    ++nf;
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t r = 0; r < n; ++r) {
    const int32_t *O = o + 3 * r, *D = d + 3 * r;
    int dg = 0;
    int64_t bn = 0, bd = 1;  /* best hit s = bn / bd, bd > 0 */
    int32_t best = -1;
    /* first pass: the nearest primitive */
    for (int64_t k = 0; k < nf; ++k) {
      const int32_t *A = m->xyz + 3 * (int64_t)f[k].a, *B = m->xyz + 3 * (int64_t)f[k].b,
                    *C = m->xyz + 3 * (int64_t)f[k].c;
      const int64_t p1 = oracle3_plucker(O, D, A, B), p2 = oracle3_plucker(O, D, B, C),
                    p3 = oracle3_plucker(O, D, C, A);
      const int pos = p1 > 0 && p2 > 0 && p3 > 0, neg = p1 < 0 && p2 < 0 && p3 < 0;
      if (!pos && !neg) {
        /* touching an edge or vertex (zeros, the rest one-signed) is a degenerate case */
        const int nz = (p1 == 0) + (p2 == 0) + (p3 == 0);
        if (nz > 0 && !((p1 > 0 || p2 > 0 || p3 > 0) && (p1 < 0 || p2 < 0 || p3 < 0))) {
          int64_t u0 = (int64_t)B[0] - A[0], u1 = (int64_t)B[1] - A[1], u2 = (int64_t)B[2] - A[2];
          int64_t v0 = (int64_t)C[0] - A[0], v1 = (int64_t)C[1] - A[1], v2 = (int64_t)C[2] - A[2];
          int64_t n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
          int64_t num = ((int64_t)A[0] - O[0]) * n0 + ((int64_t)A[1] - O[1]) * n1 + ((int64_t)A[2] - O[2]) * n2;
          int64_t den = (int64_t)D[0] * n0 + (int64_t)D[1] * n1 + (int64_t)D[2] * n2;
          if (den < 0) { den = -den; num = -num; }
          if (den != 0 && num > 0) dg |= f[k].prim >= 0 ? 1 : 2;
        }
        continue;
      }
      const int64_t u0 = (int64_t)B[0] - A[0], u1 = (int64_t)B[1] - A[1], u2 = (int64_t)B[2] - A[2];
      const int64_t v0 = (int64_t)C[0] - A[0], v1 = (int64_t)C[1] - A[1], v2 = (int64_t)C[2] - A[2];
      const int64_t n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
      int64_t num = ((int64_t)A[0] - O[0]) * n0 + ((int64_t)A[1] - O[1]) * n1 + ((int64_t)A[2] - O[2]) * n2;
      int64_t den = (int64_t)D[0] * n0 + (int64_t)D[1] * n1 + (int64_t)D[2] * n2;
      if (den < 0) { den = -den; num = -num; }
      if (num == 0) dg |= f[k].prim >= 0 ? 1 : 2;
      if (num <= 0 || f[k].prim < 0) continue;
      if (best < 0 || frac_less(num, den, bn, bd)) {
        best = k;
        bn = num;
        bd = den;
      } else if (!frac_less(bn, bd, num, den)) {
        dg |= 1;  /* two primitives at the same s */
      }
    }
    /* second pass: interior non-primitive faces crossed before it */
    int64_t cnt = 0;
    for (int64_t k = 0; k < nf; ++k) {
      if (f[k].prim >= 0 || !f[k].interior) continue;
      const int32_t *A = m->xyz + 3 * (int64_t)f[k].a, *B = m->xyz + 3 * (int64_t)f[k].b,
                    *C = m->xyz + 3 * (int64_t)f[k].c;
      const int64_t p1 = oracle3_plucker(O, D, A, B), p2 = oracle3_plucker(O, D, B, C),
                    p3 = oracle3_plucker(O, D, C, A);
      if (!((p1 > 0 && p2 > 0 && p3 > 0) || (p1 < 0 && p2 < 0 && p3 < 0))) continue;
      const int64_t u0 = (int64_t)B[0] - A[0], u1 = (int64_t)B[1] - A[1], u2 = (int64_t)B[2] - A[2];
      const int64_t v0 = (int64_t)C[0] - A[0], v1 = (int64_t)C[1] - A[1], v2 = (int64_t)C[2] - A[2];
      const int64_t n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
      int64_t num = ((int64_t)A[0] - O[0]) * n0 + ((int64_t)A[1] - O[1]) * n1 + ((int64_t)A[2] - O[2]) * n2;
      int64_t den = (int64_t)D[0] * n0 + (int64_t)D[1] * n1 + (int64_t)D[2] * n2;
      if (den < 0) { den = -den; num = -num; }
      if (num <= 0) continue;
      if (best < 0 || frac_less(num, den, bn, bd)) ++cnt;
      else if (!frac_less(bn, bd, num, den)) dg |= 2;
    }
    prim[r] = best >= 0 ? f[best].prim : -1;
    t[r] = best >= 0 ? oracle3_t(O, D, m, f[best].prim) : INFINITY;
    steps[r] = (int32_t)(1 + cnt);
    degen[r] = dg;
  }
  free(f);
  (void)nthreads;
  return 0;
}

/* ---------------------------------------------------------------- validation, location */

static int same_face(const int32_t *x, const int32_t *y) {
  /* the same three vertices, y in the reverse cyclic order of x */
  for (int s = 0; s < 3; ++s)
    if (x[0] == y[s] && x[1] == y[(s + 2) % 3] && x[2] == y[(s + 1) % 3]) return 1;
  return 0;
}

static int cmp64(const void *a, const void *b) {
  const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int oracle3_validate(const oracle_tet_t *m, char *msg, int msglen) {
  msg[0] = 0;
  for (int64_t v = 0; v < 3 * m->nv; ++v)
    if (m->xyz[v] < 0 || m->xyz[v] >= (1 << 19)) {
      snprintf(msg, msglen, "coordinate of vertex %lld out of [0, 2^19)", (long long)(v / 3));
      return 1;
    }
  for (int64_t t = 0; t < m->nt; ++t) {
    const int32_t *tv = m->tet_v + 4 * t;
    for (int i = 0; i < 4; ++i)
      if (tv[i] < 0 || tv[i] >= m->nv) {
        snprintf(msg, msglen, "tetrahedron %lld: vertex id out of range", (long long)t);
        return 1;
      }
    if (oracle3_orient(m->xyz + 3 * (int64_t)tv[0], m->xyz + 3 * (int64_t)tv[1],
                       m->xyz + 3 * (int64_t)tv[2], m->xyz + 3 * (int64_t)tv[3]) <= 0) {
      snprintf(msg, msglen, "tetrahedron %lld is not positively oriented", (long long)t);
      return 1;
    }
    for (int i = 0; i < 4; ++i) {
      const int32_t fi[3] = {tv[FACE[i][0]], tv[FACE[i][1]], tv[FACE[i][2]]};
      const int32_t nb = m->tet_nbr[4 * t + i], pr = m->tet_prim[4 * t + i];
      if (pr >= m->np || pr < -1) {
        snprintf(msg, msglen, "tetrahedron %lld face %d: primitive id out of range", (long long)t, i);
        return 1;
      }
      if (pr >= 0) {
        const int32_t *pv = m->prims + 3 * (int64_t)pr;
        int ok = 0;
        for (int s = 0; s < 3; ++s)
          for (int dir = 0; dir < 2; ++dir)
            if (pv[0] == fi[s] && pv[1] == fi[(s + (dir ? 2 : 1)) % 3] && pv[2] == fi[(s + (dir ? 1 : 2)) % 3]) ok = 1;
        if (!ok) {
          snprintf(msg, msglen, "tetrahedron %lld face %d is not the vertices of its primitive", (long long)t, i);
          return 1;
        }
      }
      if (nb < 0) continue;
      if (nb >= m->nt) {
        snprintf(msg, msglen, "tetrahedron %lld: neighbour out of range", (long long)t);
        return 1;
      }
      int found = 0;
      for (int j = 0; j < 4; ++j) {
        if (m->tet_nbr[4 * (int64_t)nb + j] != t) continue;
        const int32_t *nv = m->tet_v + 4 * (int64_t)nb;
        const int32_t fj[3] = {nv[FACE[j][0]], nv[FACE[j][1]], nv[FACE[j][2]]};
        if (!same_face(fi, fj)) continue;
        if (oracle3_orient(m->xyz + 3 * (int64_t)fi[0], m->xyz + 3 * (int64_t)fi[1], m->xyz + 3 * (int64_t)fi[2],
                           m->xyz + 3 * (int64_t)nv[j]) <= 0) {
          snprintf(msg, msglen, "tetrahedra %lld and %d overlap across their face", (long long)t, nb);
          return 1;
        }
        if (m->tet_prim[4 * (int64_t)nb + j] != pr) {
          snprintf(msg, msglen, "tetrahedra %lld and %d disagree on their face's primitive", (long long)t, nb);
          return 1;
        }
        found = 1;
      }
      if (!found) {
        snprintf(msg, msglen, "tetrahedron %lld face %d: neighbour %d does not share it back", (long long)t, i, nb);
        return 1;
      }
    }
  }
  /* Euler characteristic of a ball: V - E + F - T = 1 over the referenced vertices */
  int64_t *e = (int64_t *)malloc(sizeof(int64_t) * (size_t)(6 * m->nt));
  char *used = (char *)calloc((size_t)m->nv, 1);
  if (!e || !used) {
    free(e);
    free(used);
    snprintf(msg, msglen, "out of memory");
    return 1;
  }
  int64_t ne = 0, nf = 0, nv = 0;
  for (int64_t t = 0; t < m->nt; ++t) {
    const int32_t *tv = m->tet_v + 4 * t;
    for (int i = 0; i < 4; ++i) {
      used[tv[i]] = 1;
      for (int j = i + 1; j < 4; ++j) {
        const int64_t a = tv[i] < tv[j] ? tv[i] : tv[j], b = tv[i] < tv[j] ? tv[j] : tv[i];
        e[ne++] = a * m->nv + b;
      }
      if (m->tet_nbr[4 * t + i] < 0 || m->tet_nbr[4 * t + i] > t) ++nf;
    }
  }
  qsort(e, (size_t)ne, sizeof(int64_t), cmp64);
  int64_t ue = ne > 0 ? 1 : 0;
  for (int64_t k = 1; k < ne; ++k) ue += e[k] != e[k - 1];
  for (int64_t v = 0; v < m->nv; ++v) nv += used[v];
  free(e);
  free(used);
  if (nv - ue + nf - m->nt != 1) {
    snprintf(msg, msglen, "Euler characteristic V - E + F - T = %lld, not 1", (long long)(nv - ue + nf - m->nt));
    return 1;
  }
  return 0;
}

/* status 0 strictly inside tet[i] (the first such), 1 on the boundary of the first tetrahedron
 * holding q in its closure, -1 in none. */
int oracle3_locate(const oracle_tet_t *m, int64_t n, const int32_t *q, int32_t *tet,
                   int32_t *status, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t k = 0; k < n; ++k) {
    tet[k] = -1;
    status[k] = -1;
    for (int64_t t = 0; t < m->nt; ++t) {
      const int32_t *tv = m->tet_v + 4 * t;
      int inside = 1, strict = 1;
      for (int i = 0; i < 4 && inside; ++i) {
        const int64_t s = oracle3_orient(m->xyz + 3 * (int64_t)tv[FACE[i][0]], m->xyz + 3 * (int64_t)tv[FACE[i][1]],
                                         m->xyz + 3 * (int64_t)tv[FACE[i][2]], q + 3 * k);
        if (s > 0) inside = 0;
        if (s == 0) strict = 0;
      }
      if (inside) {
        tet[k] = (int32_t)t;
        status[k] = strict ? 0 : 1;
        break;
      }
    }
  }
  (void)nthreads;
  return 0;
}
