/*
 * ccsp_objective: the low-weight objective with fuzzy contraction, and its change under
 * single-vertex moves, on AMD Instinct MI355X (Frederickx & Dutre, arXiv 2112.05570, Sec. 2.2 for
 * the objective; Sec. 3.2.1 and 3.2.2 for the local updates that simulated annealing samples).
 *
 * A movable mesh is a triangulation whose vertices have a kind: ORIGINAL (a vertex of the scene
 * geometry, fixed), CONSTRAINED (a Steiner vertex on original edge line[v], which moves along it)
 * or FREE (a Steiner vertex with two degrees of freedom). Positions are not part of the mesh: every
 * call takes the current positions, so a caller may move vertices between calls.
 *
 * For positions p and parameters (eps, delta, eps0, mu_angle, mu_len), all in binary64:
 *   |e|        = sqrt(dx*dx + dy*dy) for edge e = (a, b), a < b, dx = p[b].x - p[a].x, dy likewise;
 *   c(e)       = 0.5 + 0.5 * min(1, |e| / eps) if e is contractible, else 1            (Sec. 2.2.1)
 *   x(e)       = the product of c over the other edges of the one or two triangles holding e,
 *                taken in increasing triangle id, each triangle's two edges in its local order
 *                after e, multiplied left to right;
 *   w(e)       = x * M(x), with M(x) = 0 if x < 1/4, 4x - 1 if x <= 1/2, else 1. The equation of
 *                Sec. 2.2.1 writes M(x); its worked example (a merged pair weighs 1/2, an edge with
 *                two contracted neighbours 0) fixes the product x * M(x). In polishing, w(e) = 1;
 *   w_contr    = sum over edges of w(e) * |e|;
 *   P_angle    = sum over the three corners of every triangle of max(0, (-1 + delta) - cos)/delta,
 *                cos = (u.x*w.x + u.y*w.y) / (|u| * |w|) for the corner's edge vectors u, w; a
 *                corner with a zero-length edge adds 0. In polishing, max(0, cos - (1 - delta))/delta
 *                (Sec. 2.2.3);
 *   P_len      = sum over edges of max(0, eps0 - |e|) / eps0                               (Sec. 2.2.3)
 *   f          = w_contr + mu_angle * P_angle + mu_len * P_len                             (Sec. 2.2.4)
 * An edge is contractible (Sec. 2.2.2) unless
 *   - both ends are ORIGINAL; or one end is ORIGINAL and the other CONSTRAINED to an original edge
 *     that does not end at it; or both are CONSTRAINED to different original edges; or
 *   - the 1-hop rule: a common neighbour H of its ends that is not one of its opposite vertices
 *     lies at distance >= eps from every opposite vertex (distances computed as |e| above); or
 *   - conditioning: its ends have different degrees of freedom (ORIGINAL 0, CONSTRAINED 1, FREE 2)
 *     and some triangle of the end with more of them, h, that does not hold the other end l, with
 *     l in h's place, is badly conditioned for good. That is decided from positions no move
 *     changes: a triangle with a FREE vertex, or whose vertices all lie on one original edge,
 *     never is; three ORIGINAL vertices are when near-collinear; two ORIGINAL o1, o2 and a
 *     CONSTRAINED vertex on original edge (a, b) when (o1, o2, a), (o1, o2, b) and (o1, o2, mid)
 *     all are, mid = ((a.x + b.x) * 0.5, (a.y + b.y) * 0.5); otherwise when the ends of every
 *     CONSTRAINED vertex's original edge, and each ORIGINAL vertex, are near-collinear with the
 *     ends (a, b) of the first CONSTRAINED vertex's original edge (in triangle order). (p, q, r)
 *     is near-collinear when 16 * A / (P * P) < 0.01, A = 0.5 * |(q.x-p.x)*(r.y-p.y) -
 *     (q.y-p.y)*(r.x-p.x)|, P = (|pq| + |qr|) + |rp|, or P = 0; or
 *   - flat triangle: it joins a FREE F and a non-FREE C, and some triangle (F, X, Y) without C
 *     has X, Y and C on one original edge L, one of X, Y CONSTRAINED; then every CONSTRAINED one T
 *     of X, Y must reach C or an ORIGINAL end of L along L, through C and F's neighbours on L,
 *     by edges shorter than eps, else the edge is not contractible.
 * Edges are numbered by (lower vertex id, higher vertex id); mesh_info returns them.
 *
 * Errors are the CCSP_* codes of ccsp_walk.h, with last_error() describing the failure.
 * Scratch: a mesh owns per-edge scratch that its calls share, so calls on one mesh must be
 * ordered (issue them on one stream, or synchronise between streams). Different meshes are
 * independent.
 */
#ifndef CCSP_OBJECTIVE_H
#define CCSP_OBJECTIVE_H

#include <stdint.h>

#include "ccsp_walk.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { CCSP_VERTEX_ORIGINAL = 0, CCSP_VERTEX_CONSTRAINED = 1, CCSP_VERTEX_FREE = 2 };

/* Per-move status of objective_delta. */
enum {
  CCSP_MOVE_OK = 1,     /* valid: every triangle of the vertex stays strictly counter-clockwise */
  CCSP_MOVE_FOLDS = 0,  /* some triangle of the vertex would not (decided exactly); delta = +inf */
  CCSP_MOVE_FIXED = -1, /* the vertex is ORIGINAL; delta = +inf */
  CCSP_MOVE_BAD = -2,   /* vertex id out of range or a coordinate not finite; delta = +inf */
  CCSP_MOVE_REJECTED = 2, /* anneal_moves: valid, not accepted by the Metropolis rule */
  CCSP_MOVE_SKIPPED = 3   /* anneal_propose: the perturbation does not apply to the vertex (no
                             move tried); delta = +inf */
};

/* Proposal kinds of anneal_propose (CCSP_PROPOSE_DISPLACE is the displacement of anneal_sweep). */
enum {
  CCSP_PROPOSE_DISPLACE = 0,
  CCSP_PROPOSE_RESAMPLE = 1, /* Sec. 3.2.4: uniform by area over the vertex's triangles */
  CCSP_PROPOSE_SWAP = 2,     /* Sec. 3.2.5: near a neighbour, for a vertex on a short edge */
  CCSP_PROPOSE_CONTRACT = 3  /* Sec. 3.2.6: a resampling that changes the contracted state */
};

typedef struct MovableMesh MovableMesh; /* opaque; owns device memory */

/* HOST pointers, read during mesh_load only. */
typedef struct {
  int64_t n_vertices;
  const int32_t *kind;   /* n_vertices: CCSP_VERTEX_* */
  const int32_t *line;   /* n_vertices: for CONSTRAINED vertices the original edge (index into
                            prim_v), ignored for the others */
  int64_t n_triangles;
  const int32_t *tri_v;  /* 3 * n_triangles vertex ids, counter-clockwise */
  int64_t n_prims;
  const int32_t *prim_v; /* 2 * n_prims: the two ORIGINAL vertices ending each original edge */
} MeshDesc;

typedef struct {
  double eps;      /* contraction length, > 0 */
  double delta;    /* angle-cosine threshold, > 0 (the paper uses cos(179 deg) + 1) */
  double eps0;     /* minimum edge length of the length penalty, > 0 */
  double mu_angle; /* weight of P_angle */
  double mu_len;   /* weight of P_len */
  int32_t polish;  /* nonzero: fixed topology (w = 1, sharp-corner penalty) */
  int32_t reserved;/* must be 0 */
} ObjectiveParams;

/*
 * mesh_load (the triangulation with vertex kinds that the objective of Sec. 2.2 is defined on):
 * build the mesh's edges, adjacency and scratch on the current device. Fails with
 * CCSP_E_BAD_TRIANGULATION when an id is out of range, a triangle repeats a vertex, a kind is
 * unknown, a CONSTRAINED vertex names no original edge, an edge lies in more than two triangles,
 * or two triangles run through their shared edge in the same direction. Synchronous.
 */
int mesh_load(const MeshDesc *desc, MovableMesh **out);

/* mesh_info: number of edges, and (if edge_v is not NULL) their ends, 2 * n_edges HOST int32. */
int mesh_info(const MovableMesh *mesh, int64_t *n_edges, int32_t *edge_v);

/*
 * objective_eval (Sec. 2.2.4, f assembled from Secs. 2.2.1-2.2.3): f and its parts at positions
 * xy (DEVICE, 2 * n_vertices binary64, 16-byte aligned). out (DEVICE, 4 binary64) receives f, w_contr, P_angle, P_len. If not NULL,
 * contractible (DEVICE, n_edges bytes, 1 = contractible) and weight (DEVICE, n_edges binary64,
 * w(e)) receive the per-edge values. Sums are reduced in a fixed order: the result is
 * reproducible for a mesh. Every triangle is expected to be counter-clockwise at xy (not checked).
 * Asynchronous on `stream`.
 */
int objective_eval(MovableMesh *mesh, const double *xy, const ObjectiveParams *params,
                   double *out, uint8_t *contractible, double *weight, void *stream);

/*
 * objective_delta (Secs. 3.2.1-3.2.2, the change of f under single-vertex moves): for k proposed
 * moves, vertex vid[i] (DEVICE int32) to q_xy[2i..2i+1] (DEVICE binary64, 16-byte aligned), each against the positions xy as they are (the moves are independent
 * alternatives, not applied): delta[i] = f(xy with the vertex moved) - f(xy) (DEVICE binary64),
 * the sum of the differences of every term of f that the move changes, and status[i] (DEVICE
 * int32, CCSP_MOVE_*). A constrained vertex's new position is taken as given (the caller projects
 * it on its original edge). Asynchronous on `stream`; overwrites the mesh's scratch. Batches of
 * 4096 moves or more are evaluated in the order of their vertices (a radix sort of the move
 * indices, results still in input order), in a device buffer the mesh keeps: 16 bytes per move
 * plus the sort's temporaries, grown (after synchronising `stream`) when k exceeds every earlier
 * batch's.
 */
int objective_delta(MovableMesh *mesh, const double *xy, const ObjectiveParams *params,
                    const int32_t *vid, const double *q_xy, int64_t k, double *delta,
                    int32_t *status, void *stream);

/*
 * mesh_classes (the sweeps' parallel form of the sequential chain of Sec. 3.1): a partition of the
 * movable (non-ORIGINAL) vertices into classes whose members are pairwise more than four edges
 * apart. A move's change of f reads positions within four edges of
 * its vertex only, so the moves of one class do not interact: evaluating them all against the same
 * positions and applying the accepted ones gives what applying them one after another would, in
 * any order. Greedy colouring over the mesh's internal order, computed on the first call and kept.
 * *n_classes receives the number of classes; if class_off is not NULL it receives n_classes + 1
 * offsets into class_v, which (if not NULL) receives the caller's vertex ids of every movable
 * vertex, class by class (HOST arrays). Synchronous.
 */
int mesh_classes(MovableMesh *mesh, int32_t *n_classes, int64_t *class_off, int32_t *class_v);

/*
 * anneal_joint (the second variant of Sec. 3.2.2, which perturbs a fixed fraction of the movable
 * vertices in one go): one Metropolis step (Sec. 3.1) for one move of the k >= 1 distinct movable
 * vertices vid[0..k) (DEVICE int32, caller ids) together. Vertex vid[i] moves by
 * lambda * eta_i * xi[2i..2i+1] (xi DEVICE binary64, 16-byte aligned, unit draws; eta_i the
 * square root of the area of vid[i]'s triangles at the positions before the move, summed in the
 * caller's triangle order, as in anneal_schedule), projected on its original edge when
 * CONSTRAINED (as in anneal_moves). The move is valid when every triangle of every moved vertex
 * is strictly counter-clockwise afterwards. Its change of f is the sum over edges and triangles
 * of every term's new value minus its old one (each term as in objective_eval; a term the move
 * does not reach gives exactly 0), added per part in a fixed order and combined as f is. It is
 * accepted when valid and delta <= 0 or u < exp(-delta / temperature); xy (DEVICE) is then updated
 * in place. *delta_out (HOST) receives the change (+inf unless valid) and *status_out (HOST)
 * CCSP_MOVE_OK, CCSP_MOVE_REJECTED, CCSP_MOVE_FOLDS, or CCSP_MOVE_BAD when an id is out of range,
 * ORIGINAL or repeated, or a draw is not finite (nothing moves then). Synchronises `stream` once;
 * overwrites the mesh's scratch. Device memory kept by the mesh: 16 bytes per edge, 8 per
 * triangle, 4 per vertex and 16 per moved vertex (grown, after synchronising `stream`, when k
 * exceeds every earlier call's).
 */
int anneal_joint(MovableMesh *mesh, double *xy, const ObjectiveParams *params,
                 double temperature, double lambda, const int32_t *vid, int64_t k,
                 const double *xi, double u, double *delta_out, int32_t *status_out,
                 void *stream);

/*
 * anneal_joint_groups (the second variant of Sec. 3.2.3, which perturbs a fixed set of groups in
 * one go): one Metropolis step for the group moves of n >= 1 centres (DEVICE int32 caller ids)
 * made together. Centre i's group (as in anneal_group, at the positions before the move: d from
 * draws[4i+2], members within d) moves by (lambda * sqrt(group area)) * (draws[4i], draws[4i+1])
 * (draws DEVICE binary64, 16-byte aligned), projected per CONSTRAINED member; a vertex in several
 * groups moves with the displacement of the first of them in centre order (the paper does not say;
 * this is a reading). Validity, change of f, decision, outputs and the update of xy are those of
 * anneal_joint; CCSP_MOVE_BAD when a centre is out of range or ORIGINAL. Synchronises `stream`
 * three times; allocates its group scratch for the call (as anneal_group) and keeps anneal_joint's
 * workspace; overwrites the mesh's scratch.
 */
int anneal_joint_groups(MovableMesh *mesh, double *xy, const ObjectiveParams *params,
                        double temperature, double lambda, const int32_t *centres, int64_t n,
                        const double *draws, double u, double *delta_out, int32_t *status_out,
                        void *stream);

/*
 * anneal_moves: one Metropolis step (Sec. 3.1) for each of k single-vertex moves (Sec. 3.2.2), for
 * moves that do not interact (the vertices of one class of mesh_classes; for other sets, every
 * move is still evaluated against the positions before the call). Move i displaces vertex vid[i]
 * (DEVICE int32) by disp[2i..2i+1] (DEVICE binary64, 16-byte aligned); for a CONSTRAINED vertex the
 * displacement d is first projected on its original edge (a, b): d <- s * e with e = b - a and
 * s = (d.x*e.x + d.y*e.y) / (e.x*e.x + e.y*e.y). The move is accepted when it is valid (as in
 * objective_delta) and delta <= 0 or u[i] < exp(-delta / temperature) (u DEVICE binary64 in
 * [0, 1), temperature >= 0); accepted positions are written into xy (DEVICE, in place). delta
 * (DEVICE binary64) receives the change of f of each move and status (DEVICE int32) CCSP_MOVE_OK
 * for an accepted move, CCSP_MOVE_REJECTED for a valid one not accepted, or the objective_delta
 * codes. A vertex may appear at most once. Asynchronous on `stream`; overwrites the mesh's scratch.
 */
int anneal_moves(MovableMesh *mesh, double *xy, const ObjectiveParams *params, double temperature,
                 const int32_t *vid, const double *disp, const double *u, int64_t k, double *delta,
                 int32_t *status, void *stream);

/*
 * anneal_sweep (Sec. 3.1 acceptance, Sec. 3.2.2 displacements): one Metropolis step for every
 * movable vertex, class by class in the order of mesh_classes (classes computed on first use): the result is that of the sequential chain over
 * the vertices in the order mesh_classes lists them. Entry i of disp (DEVICE, 2 binary64 per
 * movable vertex, 16-byte aligned), u, delta and status (DEVICE, one per movable vertex) belongs to
 * the i-th vertex of that list; moves, acceptance, projection and status codes are those of
 * anneal_moves, and every move is evaluated against the positions its predecessors in the list
 * left. xy (DEVICE) is updated in place. One launch per class after one pass over the edges.
 * Asynchronous on `stream`; overwrites the mesh's scratch.
 */
int anneal_sweep(MovableMesh *mesh, double *xy, const ObjectiveParams *params, double temperature,
                 const double *disp, const double *u, double *delta, int32_t *status, void *stream);

/*
 * anneal_propose (Secs. 3.2.4-3.2.6: resampling, swap, contraction to a neighbour): one sweep as
 * anneal_sweep (class by class, equal to the sequential chain in the order of mesh_classes) with the proposals of Secs. 3.2.4-3.2.6 in place of displacements. The
 * i-th movable vertex v (mesh_classes order) uses draws[4i..4i+3] = r0, r1, r2, r3 (DEVICE
 * binary64, 16-byte aligned; r0, r1, r2 in [0, 1), and for SWAP (r2, r3) a point of the closed unit
 * disk) and u[i]; positions are the current ones, left by the vertices before it.
 *  - RESAMPLE: over v's triangles in increasing caller id, with areas
 *    0.5 * ((b.x-a.x)*(c.y-a.y) - (b.y-a.y)*(c.x-a.x)) on their stored vertices summed left to right,
 *    the first triangle whose running sum exceeds r0 times the total; in it (a, b, c) the point
 *    (1 - s) a + s (1 - r2) b + s r2 c, s = sqrt(r1), each coordinate summed left to right.
 *  - SWAP: l = (0.2 + 1.8 * r0) * eps; if no edge of v is shorter than l, the vertex is SKIPPED;
 *    otherwise w = the neighbour of rank min(floor(r1 * deg), deg - 1) in increasing caller id,
 *    and the point w + l * (r2, r3).
 *  - CONTRACT: the RESAMPLE point (after the projection below); SKIPPED unless exactly one of v's
 *    old and new positions has an edge of v shorter than eps.
 * The move d = point - v is projected as in anneal_moves for a CONSTRAINED vertex and the
 * proposal is v + d; acceptance, delta and status are those of anneal_moves, plus
 * CCSP_MOVE_SKIPPED. Edge lengths are sqrt(dx*dx + dy*dy). xy (DEVICE) is updated in place.
 * Asynchronous on `stream`; overwrites the mesh's scratch.
 */
int anneal_propose(MovableMesh *mesh, double *xy, const ObjectiveParams *params, double temperature,
                   int32_t kind, const double *draws, const double *u, double *delta,
                   int32_t *status, void *stream);

/*
 * anneal_group: group moves (Sec. 3.2.3) for the n centres (DEVICE int32 caller ids, movable
 * vertices; anything else gets status CCSP_MOVE_BAD or CCSP_MOVE_FIXED and round -1). Centre i
 * uses draws[4i..4i+3] = xi.x, xi.y, r, (unused) (DEVICE binary64, 16-byte aligned; r in [0, 1))
 * and u[i]:
 *  - d = (0.5 + 4.5 * r) * eps; the members are c and every vertex that is not ORIGINAL and lies
 *    within d of it (sqrt(dx*dx + dy*dy) <= d at the positions when the move is made), whether
 *    or not an edge joins it to c, with no limit on their number: c first, then by increasing
 *    caller id. They are found with a uniform grid of the positions, as the paper does;
 *  - area = the area of the triangles holding any member, each counted at the first member (in
 *    that order) it holds, a member's triangles in increasing caller id, each area as in
 *    anneal_schedule, summed left to right; the displacement is (lambda * sqrt(area)) * xi,
 *    projected as in anneal_moves for each CONSTRAINED member;
 *  - valid when every triangle of every member is strictly counter-clockwise afterwards (exact);
 *    delta[i] is the change of f of the whole move (+inf when not valid), accepted as in
 *    anneal_moves. status[i] is CCSP_MOVE_OK, CCSP_MOVE_REJECTED or CCSP_MOVE_FOLDS and
 *    members[i] (DEVICE int32) the group's size.
 * The moves are made in rounds; round[i] (DEVICE int32) receives the round of centre i. Moves of
 * one round are independent (more than five edges apart along paths that do not pass through an
 * ORIGINAL vertex of more than 32 neighbours, neither moving a vertex into or out of the other's
 * disc), so the result equals the sequential chain over the centres in the order of increasing
 * (round[i], i). xy (DEVICE) is updated in place. Allocates its scratch (about 30 bytes per
 * centre, 24 per member of the round's pending groups, 8 per vertex, 8 per cell of the query
 * grid and 4 per cell of the claims' grid, at most 64 MiB) and
 * synchronises `stream` once per round; overwrites the mesh's scratch.
 */
int anneal_group(MovableMesh *mesh, double *xy, const ObjectiveParams *params, double temperature,
                 double lambda, const int32_t *centres, int64_t n, const double *draws,
                 const double *u, double *delta, int32_t *status, int32_t *members,
                 int32_t *round, void *stream);

/*
 * anneal_schedule: n_sweeps sweeps (as anneal_sweep) of simulated annealing with both the
 * temperature and the contraction length lowered by the caller's schedule (Sec. 3.3.1: sweep k
 * uses temperature[k] and eps[k], HOST arrays; params supplies the other parameters) and an
 * adaptive step scale (Sec. 3.2): the move of the i-th movable vertex (in mesh_classes order) in
 * sweep k is lambda_k * eta * xi[k][i], with xi (DEVICE, n_sweeps x movable x 2 binary64, 16-byte
 * aligned) unit draws supplied by the caller and eta the square root of the area of the vertex's
 * triangles at the current positions, summed in the caller's triangle order, each area as
 * 0.5 * ((b.x-a.x)*(c.y-a.y) - (b.y-a.y)*(c.x-a.x)); the move is then (lambda_k * eta) * xi,
 * projected as in anneal_moves, and accepted with u[k][i] (DEVICE, n_sweeps x movable). lambda_0
 * = lambda0; after sweep k, with a the accepted fraction, lambda_{k+1} = lambda_k * f, f =
 * 1 + (a - target) limited to [1/2, 2] (the paper keeps acceptance near a target, 23%, without
 * giving the rule). lambda_out[k] and accepted_out[k] (HOST) receive lambda_k and the number of
 * accepted moves. xy (DEVICE) is updated in place. Synchronises `stream` after every sweep.
 */
int anneal_schedule(MovableMesh *mesh, double *xy, const ObjectiveParams *params, int32_t n_sweeps,
                    const double *temperature, const double *eps, double lambda0, double target,
                    const double *xi, const double *u, double *lambda_out, int64_t *accepted_out,
                    void *stream);

/*
 * mesh_subdivide: the subdivision of Sec. 3.5.2, every triangle split into four at the midpoints
 * of its edges. HOST code and HOST pointers. Input: desc (as mesh_load) and xy (2 * n_vertices
 * binary64). The vertices keep their ids, kinds and lines; edge e (edges numbered by
 * min * n_vertices + max of their ends, increasing) adds vertex n_vertices + e at
 * ((xa + xb) * 0.5, (ya + yb) * 0.5), CONSTRAINED to the original edge that holds both ends (the
 * line of a CONSTRAINED end, or the original edge joining two ORIGINAL ends) if there is one,
 * else FREE (line -1). Triangle t = (v0, v1, v2) with midpoints m_i of its edges opposite v_i gives
 * t, T + t, 2T + t, 3T + t = (v0, m2, m1), (v1, m0, m2), (v2, m1, m0), (m0, m1, m2). Sizes go to
 * *n_vertices_out = n_vertices + edges and *n_triangles_out = 4 * n_triangles; with xy_out,
 * tri_out, kind_out or line_out NULL only the sizes are computed, else those HOST arrays
 * (caller-allocated at these sizes) receive the result. Errors: CCSP_E_ARG,
 * CCSP_E_BAD_TRIANGULATION (ids, kinds or lines out of range, or a sub-triangle that rounding of a
 * midpoint leaves not strictly counter-clockwise, decided exactly). Thread-safe.
 */
int mesh_subdivide(const MeshDesc *desc, const double *xy, int64_t *n_vertices_out,
                   int64_t *n_triangles_out, double *xy_out, int32_t *tri_out, int32_t *kind_out,
                   int32_t *line_out);

/*
 * mesh_contract: contraction of the edges shorter than eps (Sec. 3.4.1), turning a triangulation
 * whose short edges stand for merged vertices into one where they are merged. HOST code and HOST
 * pointers throughout (sequential, as each contraction changes the next one's neighbourhood).
 * Input: desc (as mesh_load; triangles must be strictly counter-clockwise) and xy (2 * n_vertices
 * binary64). Contraction runs in passes; a pass lists the edges shorter than eps at its start in
 * increasing (length, lower id, higher id), lengths sqrt(dx*dx + dy*dy), and tries each that is
 * still an edge and still shorter; passes repeat until one contracts nothing. An edge (a, b) is
 * contracted only when
 *  - the original geometry allows it: not two ORIGINAL vertices, not an ORIGINAL vertex with a
 *    CONSTRAINED one whose original edge does not end at it, not two CONSTRAINED vertices on
 *    different original edges;
 *  - the common neighbours of a and b are exactly the vertices opposite the edge;
 *  - it is not an interior edge with both ends on the hull;
 *  - no remaining triangle around the survivor has all three vertices on one original edge (its
 *    ORIGINAL ends or vertices CONSTRAINED to it);
 *  - the survivor has a position where every remaining triangle around it is strictly
 *    counter-clockwise (exact): an ORIGINAL vertex survives where it is, as does a CONSTRAINED
 *    one against a FREE one; otherwise the lower id survives at a + t (b - a), t tried as 1/2,
 *    1/4, 3/4, 0, 1.
 * The edge's triangles are removed and the other vertex is replaced by the survivor. Output (HOST,
 * caller-allocated with the input's sizes): tri_out (3 per triangle), kind_out, line_out, xy_out
 * (2 per vertex) of the surviving vertices renumbered in increasing old id and the surviving
 * triangles in increasing old id, each with its vertex order; old_to_new[v] (n_vertices) the new
 * id of v's survivor (-1 for a vertex in no triangle); the counts and the number of contractions.
 * Errors: CCSP_E_ARG, CCSP_E_BAD_TRIANGULATION (ids out of range, a triangle not strictly
 * counter-clockwise). Allocates host memory for the call; thread-safe.
 */
int mesh_contract(const MeshDesc *desc, const double *xy, double eps, int32_t *tri_out,
                  int64_t *n_triangles_out, int32_t *kind_out, int32_t *line_out, double *xy_out,
                  int64_t *n_vertices_out, int32_t *old_to_new, int64_t *n_contracted);

/*
 * flip_anneal: simulated annealing of a constrained triangulation by edge flips (Sec. 3.2.7), the
 * energy being its weight (total edge length), in n_rounds rounds at temperature[r] (HOST). The
 * triangulation is given in the arrays of ccsp_walk.h, here DEVICE buffers updated in place:
 * tri_v, tri_nbr, tri_prim (3 * n_triangles int32 each) over positions xy (DEVICE, 2 * n_vertices
 * binary64, 16-byte aligned). A flip replaces the unconstrained interior edge (b, c) of
 * t = (a, b, c) and u = (d, c, b) by (a, d) when both (a, b, d) and (a, d, c) are strictly
 * counter-clockwise (exact); its change of weight is |ad| - |bc| (lengths as in the objective).
 * It is accepted when the change is < 0, or, at temperature T > 0, when u < exp(-change / T).
 * Round r: every unconstrained interior edge, named by its slot 3t + i in the triangle of lower
 * id, draws a 64-bit priority and u = (x >> 11) * 2^-53 as outputs k + 1 and k + 2 of the
 * SplitMix64 sequence from state seed, k = 2 * (r * 2^32 + slot); each is tested against the
 * triangulation as the round found it; among the accepted flips, one is applied when its
 * (priority, slot) beats every other accepted flip touching one of the triangles its flip touches
 * (its two triangles and their neighbours). The applied flips are independent, so the round is
 * the same as applying them one after another. After a flip, t holds (a, b, d) and u holds
 * (a, d, c), in that vertex order, with neighbours and primitive ids following their edges.
 * With vertex_line (DEVICE, n_vertices int32: the original edge of each Steiner vertex on one,
 * -1 for the other vertices) and prim_v (DEVICE, 2 * n_prims int32: the ends of each original
 * edge), a flip is also refused when one of its new triangles has all three vertices on one
 * original edge (its ends or Steiner vertices on it): zero area in intent, which the exact test
 * lets through when rounding leaves a Steiner vertex off its line (Sec. 3.2.7 asks for strict
 * convexity against exactly this). vertex_line NULL: no such test (prim_v and n_prims ignored).
 * flips_out[r] (HOST) receives the number of flips of round r; a round with none at T = 0 leaves
 * no flip that would lower the weight. The triangulation must be valid (as load_triangulation
 * checks); triangle and vertex ids read from it are range-checked. n_rounds <= 2^20. Allocates
 * device scratch for the call: 5 bytes per slot, 4 per triangle and 512 per round; the rounds are
 * queued on `stream` back to back and the call synchronises it once, at the end.
 */
int flip_anneal(int64_t n_vertices, const double *xy, int64_t n_triangles, int32_t *tri_v,
                int32_t *tri_nbr, int32_t *tri_prim, const int32_t *vertex_line, int64_t n_prims,
                const int32_t *prim_v, int32_t n_rounds, const double *temperature, uint64_t seed,
                int64_t *flips_out, void *stream);

/* mesh_free: release the mesh (after its calls have completed). NULL is ignored. */
void mesh_free(MovableMesh *mesh);

#ifdef __cplusplus
}
#endif

#endif
