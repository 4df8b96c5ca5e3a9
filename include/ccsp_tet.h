/*
 * ccsp_tet: stackless ray traversal of a 3D constrained tetrahedralisation on AMD Instinct MI355X.
 *
 * The operation is the 3D form of the triangulation walk (Frederickx & Dutre, arXiv 2112.05570):
 * the scene's triangles are faces of a tetrahedralisation (the 3D constrained triangulation of
 * Sec. 1.3), and a ray walks from the tetrahedron holding its origin through one tetrahedron after
 * another. One decision per tetrahedron picks the face the ray leaves through; once the entry face
 * is known three candidates remain (Sec. 1.4 counts four faces per tetrahedron and the cost as the
 * number of tetrahedra visited; Sec. 7.2 names the 3D case as the next step of the method). Per
 * ray the library returns
 *   hit_prim  the primitive triangle crossed first at s > 0 (>= 0), or a status below 0,
 *   hit_t     its parameter, from the primitive's own vertices (a, b, c) as
 *             ((ax-ox)*nx + (ay-oy)*ny + (az-oz)*nz) / (dx*nx + dy*ny + dz*nz),
 *             n = (b - a) x (c - a), in IEEE binary64 in exactly this order without fused
 *             operations (+inf without a hit),
 *   steps     the number of tetrahedra visited, start and hit tetrahedron included.
 *
 * Integer grid. Vertex and origin coordinates are integers in [0, 2^19), direction components
 * integers in [-2^19, 2^19], not all zero. Every decision is then exact (a coordinate difference
 * is below 2^20 in size and the largest product sum below 2^62), and hit_prim, hit_t and steps are
 * defined bit for bit.
 *
 * Decisions. The ray passes the directed edge (p, q) with Plücker sign pi(p, q) = sign of
 * d . ((p - o) x (q - o)). A face ordered counter-clockwise as seen from outside its tetrahedron
 * is the exit face iff its three directed edges have pi = +. In the start tetrahedron the exit is
 * the first face, in face order 0..3, passing that test. After entering through face e with apex
 * w (the vertex opposite e) and face e's vertices (p, q, r) in its outside order, two signs
 * decide: if pi(w, p) = + the exit is the face opposite q when pi(w, r) = -, else the face
 * opposite p; if pi(w, p) = - the exit is the face opposite r when pi(w, q) = +, else the face
 * opposite p. A zero value is decided as for the line moved symbolically, origin
 * o + (e, e^2, e^3) and direction d + (e^10, e^20, e^30) for an infinitesimal e > 0: with
 * a = q - p, c = d x a and W = (p - o) x (q - o), the sign is that of the first nonzero of
 * c_x, c_y, c_z, W_x, -a_z, a_y, W_y, a_z, -a_x. The moved line is a real line in general
 * position, so the walk never loops and never lacks an exit face.
 *
 * Conventions
 *   Tetrahedron t has vertices tet_v[4t+0..3] with det[v1 - v0; v2 - v0; v3 - v0] > 0. Face i is
 *   opposite tet_v[4t+i]; seen from outside it is ordered (1,2,3), (0,3,2), (0,1,3), (0,2,1) for
 *   i = 0..3. tet_nbr[4t+i] is the tetrahedron across face i (-1 on the hull); tet_prim[4t+i] the
 *   primitive lying on face i, -1 if none (both tetrahedra of an interior face name the same
 *   primitive). prims[3k+0..2] are primitive k's vertex ids, in the order t is computed from.
 *
 * Errors follow ccsp_walk.h: CCSP_OK or a negative code, last_error() describing it. Per-ray
 * outcomes: CCSP_RAY_MISS (-1) out through a hull face that is not a primitive; CCSP_RAY_GUARD
 * (-2) the walk would enter one tetrahedron more than the step limit (steps = the limit);
 * CCSP_RAY_BAD (-3) start out of range, a coordinate off the grid, a zero direction or an origin
 * not strictly inside the start tetrahedron (checked exactly for every ray; steps = 0).
 */
#ifndef CCSP_TET_H
#define CCSP_TET_H

#include <stdint.h>

#include "ccsp_walk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct TetMesh TetMesh; /* opaque; owns its device memory */

/* Host description of a tetrahedralisation; everything is copied at load. */
typedef struct {
  int64_t n_vertices;       /* 4 .. 2^31 - 1 */
  const int32_t *xyz;       /* 3*n_vertices grid coordinates in [0, 2^19) */
  int64_t n_tets;           /* 1 .. 2^29 - 1 */
  const int32_t *tet_v;     /* 4*n_tets */
  const int32_t *tet_nbr;   /* 4*n_tets */
  const int32_t *tet_prim;  /* 4*n_tets */
  int64_t n_prims;          /* 0 .. 2^29 */
  const int32_t *prims;     /* 3*n_prims vertex ids */
} TetMeshDesc;

/* load_tetmesh: validate and upload a tetrahedralisation whose faces carry the scene's triangles
 * (the 3D constrained triangulation of Sec. 1.3; host arrays; synchronous). Checks, exactly: ids and
 * coordinates in range, every tetrahedron positively oriented, every interior face shared with
 * the neighbour it names, whose fourth vertex lies strictly on the face's outer side, and every
 * primitive face named by both of its tetrahedra and made of its primitive's three vertices.
 * Returns CCSP_E_BAD_TRIANGULATION with the first failure in last_error(), CCSP_E_OOM if device
 * memory runs out. The library renumbers the tetrahedra internally along a Morton curve of their
 * centroids (callers keep using their own ids). Device memory: 128 bytes per tetrahedron: four
 * 16-byte face slots (the neighbour and its entry face, the neighbour's fourth vertex, the vertex
 * order across the face) and 64 bytes for its four vertices and internal id (read in the start
 * tetrahedron). */
int load_tetmesh(const TetMeshDesc *desc, TetMesh **out);

/* free_tetmesh: free a loaded tetrahedralisation (synchronises the device first). NULL is a no-op. */
int free_tetmesh(TetMesh *mesh);

/* tetmesh_info: tetrahedron count and device bytes of a loaded tetrahedralisation. */
int tetmesh_info(const TetMesh *mesh, int64_t *n_tets, int64_t *device_bytes);

/* Launch parameters of trace_rays3d; zero fields take the defaults. */
typedef struct {
  int32_t wg_size;        /* threads per workgroup: 64..512, multiple of 64 (default 256) */
  int32_t waves_per_cu;   /* persistent waves per compute unit, 1..64 (default 12) */
  int32_t rays_per_claim; /* rays a wave takes per global atomic, 64..65536, multiple of 64
                             (default 256); the wave stages them 64 at a time in LDS */
  int32_t refill_min;     /* refill a wave once this many lanes are idle, 1..64 (default 8) */
  int32_t bin_key;        /* binning key: 1 = the origin's cell of an 8x8x8 Morton-ordered grid,
                             2 = that cell and the octant of the direction (default 1) */
} Tune3d;

/* Walk n rays through `mesh` (Sec. 1.4's per-tetrahedron decision, the 3D form of Sec. 5.1's
 * walk). o, d: 3*n int32 (device), start: n int32 (device, the caller's tetrahedron ids), outputs
 * hit_prim (n int32), hit_t (n binary64), steps (n int32) on the device, all in input order;
 * every ray is independent, so the output arrays may not overlap the inputs.
 * flags: 0 or CCSP_TRACE_INPUT_ORDER (walk the rays in input order instead of binning them by
 * start tetrahedron first), optionally with CCSP_TRACE_TIMED (record stage events for
 * trace3d_stage_times). Binning is a counting sort by the origin's cell of an 8x8x8 grid in
 * Morton order (and the direction's octant, Tune3d.bin_key), so that the rays an XCD walks start
 * close together and the rays a wave walks also head the same way; it also decides every ray's
 * start tetrahedron (the precondition checks and the first exit face), so the walk proper starts
 * at the first exit. Results are the same in either order.
 * step_limit: 0 = the tetrahedron count, which the walk never exceeds; else a walk that would
 * enter one tetrahedron more ends with CCSP_RAY_GUARD. tune may be NULL. Asynchronous on `stream`
 * (hipStream_t, NULL = default stream); n = 0 is a no-op.
 * Device memory: a ring of 128 groups of 8 tile counters per device (at most 128 calls in flight
 * on one device at once), and ray scratch of 64 bytes per ray plus 16 KiB per 4096 rays, shared by the
 * device's traces, grown (after a device synchronisation) when n exceeds every earlier call's;
 * traces that bin on different streams of one device are ordered one after the other. */
int trace_rays3d(const TetMesh *mesh, const int32_t *o, const int32_t *d, const int32_t *start,
                 int64_t n, int32_t flags, int32_t step_limit, const Tune3d *tune,
                 int32_t *hit_prim, double *hit_t, int32_t *steps, void *stream);

/* trace3d_stage_times: stage durations of the device's most recent trace_rays3d with CCSP_TRACE_TIMED: binning and
 * the walk, in milliseconds (waits for that trace to finish). */
int trace3d_stage_times(float *bin_ms, float *walk_ms);

#ifdef __cplusplus
}
#endif

#endif
