/*
 * Checker for the stackless triangulation ray walk: TEST INFRASTRUCTURE ONLY.
 * Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg; never by the walk
 * library. See oracle.c for the definitions each entry point follows.
 */
#ifndef CCSP_ORACLE_H
#define CCSP_ORACLE_H
#include <stdint.h>

typedef struct {
  int64_t nv;              /* vertices */
  const double *xy;        /* 2*nv: x, y */
  int64_t nt;              /* triangles */
  const int32_t *tri_v;    /* 3*nt, counter-clockwise; edge i is opposite vertex i */
  const int32_t *tri_nbr;  /* 3*nt, triangle across edge i, -1 on the hull */
  const int32_t *tri_prim; /* 3*nt, primitive id of a constrained edge i, -1 otherwise */
  int64_t np;              /* primitives */
  const double *prim;      /* 4*np: ax, ay, bx, by */
} oracle_tri_t;

/* exact signs */
int oracle_side_sign(const double *o, const double *d, const double *v); /* sign dx(vy-oy)-dy(vx-ox) */
int oracle_orient(const double *a, const double *b, const double *c);
int oracle_incircle(const double *a, const double *b, const double *c, const double *d);
double oracle_t(const double *o, const double *d, const double *seg);

/* Per ray: prim >= 0 hit, -1 left the triangulation, -2 step guard (the walk would enter
 * triangle max_steps + 1; then steps = max_steps; max_steps <= 0 or above the triangle count
 * means the triangle count), -3 origin not strictly inside the start triangle (walk) or
 * malformed input (brute force). t = +inf unless a hit. */
int oracle_walk(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                const int32_t *start, int64_t max_steps, int32_t *prim, double *t,
                int32_t *steps, int nthreads);
int oracle_brute_edges(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                       int32_t *prim, double *t, int32_t *steps, int nthreads);
int oracle_brute_prims(int64_t np, const double *pseg, int64_t n, const double *o,
                       const double *d, int32_t *prim, double *t, int nthreads);
int oracle_validate(const oracle_tri_t *m, int check_delaunay, char *msg, int msglen);
/* The walk continued by specular reflections at hits, up to max_bounces (see oracle.c); the
 * step limit max_steps (as in oracle_walk) applies to each segment. */
int oracle_bounce(const oracle_tri_t *m, int64_t n, const double *o, const double *d,
                  const int32_t *start, int32_t max_bounces, int64_t max_steps, int32_t *prim,
                  double *t, int32_t *steps, int32_t *hits, int32_t *face, int nthreads);
/* Point location by brute force: the first triangle (in index order) whose closure contains q;
 * status 0 strictly inside, 1 on an edge or vertex, -1 in no triangle, -2 not finite. */
int oracle_locate(const oracle_tri_t *m, int64_t n, const double *q, int32_t *tri,
                  int32_t *status, int nthreads);
int oracle_num_threads(void);
#endif
