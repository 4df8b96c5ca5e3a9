/*
 * ccsp_walk: stackless ray traversal of a 2D constrained triangulation on AMD Instinct MI355X.
 *
 * The operation (Frederickx & Dutre, arXiv 2112.05570, Sec. 5.1 "Ray Traversal", and the
 * operation count of Sec. 5.4): a ray R(s) = o + s*d starts inside a known triangle. In each
 * visited triangle one decision is taken: the edge the ray leaves through. If that edge is part
 * of the scene geometry (a constrained edge) the walk stops with a hit; if no triangle lies across
 * it the ray has left the triangulation (no hit); otherwise the walk continues in the neighbour.
 * Per ray the library returns
 *   hit_prim  the primitive id of the constrained edge hit (>= 0), or a status below 0,
 *   hit_t     the hit parameter t with R(t) on the primitive, computed from the primitive's own
 *             segment (a,b) as ((ax-ox)*ey - (ay-oy)*ex) / (dx*ey - dy*ex), e = b - a, in IEEE
 *             binary64 in exactly this order without fused operations (so t does not depend on the
 *             triangulation, nor on where a primitive is split into several edges),
 *   steps     the number of triangles visited, start and hit triangle included (Sec. 5.4).
 *
 * Decisions are exact: vertex v is LEFT of the ray iff dx*(vy-oy) - dy*(vx-ox) >= 0 evaluated
 * exactly on the binary64 inputs (zero counts as LEFT: the ray is shifted infinitesimally to its
 * right, a consistent symbolic perturbation). Sec. 5.1 requires consistent decisions to avoid
 * loops and missing exit edges; exactness makes hit_prim and steps independent of the precision
 * mode. In TRACE_FP32_FILTERED mode the sign is first taken from single-precision coordinates
 * and accepted only when a forward error bound proves it; otherwise the binary64 filter and, if
 * needed, an exact expansion decide. Both modes give identical hit_prim, hit_t and steps.
 *
 * Conventions
 *   Triangle t has counter-clockwise vertices tri_v[3t+0..2]; its edge i joins tri_v[3t+(i+1)%3]
 *   and tri_v[3t+(i+2)%3] and lies opposite tri_v[3t+i]. tri_nbr[3t+i] is the triangle across
 *   edge i (-1 on the hull). tri_prim[3t+i] is the primitive id of a constrained edge i, -1 for an
 *   unconstrained one. A primitive may be split over several collinear constrained edges.
 *
 * Errors: every call returns CCSP_OK (0) or a negative code; last_error() then describes the
 * failure (thread-local, valid until the next call on the same thread). Per-ray outcomes are
 * data: hit_prim >= 0 hit; CCSP_RAY_MISS (-1) left through an unconstrained hull edge, hit_t=+inf;
 * CCSP_RAY_GUARD (-2) the walk reached the step limit (by default the triangle count, which an
 * exact walk never exceeds; TuneParams.step_limit lowers it) with another triangle to enter; CCSP_RAY_BAD (-3) start_tri out of range or the origin is not strictly inside it (then
 * steps = 0). A ray whose origin is not strictly inside start_tri is a precondition violation;
 * without CCSP_TRACE_VALIDATE it may also end as a hit or miss along a wrong path, but never reads
 * out of bounds.
 *
 * Streams: every stream argument is a hipStream_t (NULL = the default stream). Calls are
 * asynchronous on that stream unless stated; results are valid once the stream has reached the
 * point of the call. A loaded triangulation is read-only, so traces on different streams may run
 * concurrently.
 */
#ifndef CCSP_WALK_H
#define CCSP_WALK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CCSP_OK = 0,
  CCSP_E_ARG = -1,               /* a null pointer, negative size, misaligned buffer, bad mode */
  CCSP_E_BAD_TRIANGULATION = -2, /* the descriptor fails validation (see load_triangulation) */
  CCSP_E_OOM = -3,               /* device or pinned host allocation failed */
  CCSP_E_HIP = -4,               /* a HIP runtime call failed */
  CCSP_E_BAD_RAY = -5            /* CCSP_TRACE_VALIDATE found a ray violating its precondition */
};

enum {
  CCSP_RAY_MISS = -1,
  CCSP_RAY_GUARD = -2,
  CCSP_RAY_BAD = -3
};

/* precision: one mode, optionally OR-ed with flags */
enum {
  CCSP_TRACE_FP64 = 0,          /* binary64 coordinates, binary64 filter, exact fallback */
  CCSP_TRACE_FP32_FILTERED = 1, /* binary32 coordinates + error-bound filter, then as FP64 */
  CCSP_TRACE_MODE_MASK = 0xff,
  CCSP_TRACE_VALIDATE = 1 << 8, /* check every ray's precondition exactly; synchronises the
                                   stream and returns CCSP_E_BAD_RAY if any ray fails it */
  CCSP_TRACE_COUNT = 1 << 9,    /* accumulate the counters read by read_counters() */
  CCSP_TRACE_INPUT_ORDER = 1 << 10, /* walk rays in input order instead of binning them first
                                       (see trace_rays) */
  CCSP_TRACE_TIMED = 1 << 11,       /* record HIP events on the stream around the stages of this
                                       trace, for read_stage_times() */
  CCSP_TRACE_GRAPH = 1 << 12        /* trace_batch only: replay the launch from a cached HIP graph */
};

typedef struct Triangulation Triangulation; /* opaque; owns its device memory */

/* Host description of a triangulation; everything is copied at load. */
typedef struct {
  int64_t n_vertices;
  const double *xy;        /* 2*n_vertices: x0,y0,x1,y1,... (binary64 is authoritative) */
  int64_t n_triangles;     /* < 2^29 */
  const int32_t *tri_v;    /* 3*n_triangles */
  const int32_t *tri_nbr;  /* 3*n_triangles */
  const int32_t *tri_prim; /* 3*n_triangles */
  int64_t n_prims;
  const double *prim_seg;  /* 4*n_prims: ax,ay,bx,by (t is computed from these) */
} TriangulationDesc;

/* Launch parameters of the persistent walk. A zero field takes the default. Passing NULL uses the
 * device's tuning cache entry for the workload's shape (see autotune), else the defaults. */
typedef struct {
  int32_t wg_size;         /* threads per workgroup: 64..512, multiple of 64 (default 256) */
  int32_t tile_rays;       /* rays a wave stages in LDS per tile: 64, 128 or 256 (default 64) */
  int32_t waves_per_cu;    /* persistent waves per compute unit, i.e. the grid (default 24) */
  int32_t refill_min;      /* refill a wave once this many of its 64 lanes are idle, 1..64
                              (default 16) */
  int32_t tiles_per_claim; /* tiles taken per global atomic, 1..4096 (default 4) */
  int32_t xcd_chunks;      /* 1: one tile counter for the whole launch; 8: one per XCD, each XCD
                              starting in its own eighth of the rays (default 8) */
  int32_t bin;             /* trace_rays ray order: 1 = bucket binning by origin cell (default),
                              2 = radix sort by start triangle; ignored by trace_batch */
  int32_t step_limit;      /* not a launch parameter: the step guard's limit. A walk that would
                              enter one triangle more than this ends with CCSP_RAY_GUARD and
                              steps = step_limit (trace_bounces: the limit applies to each segment
                              and steps still counts all segments). 0 or more than the triangle
                              count: the triangle count, which an exact walk never exceeds. Applies
                              to every item of a batch; never stored in the tuning cache, so a
                              TuneParams with only this field set takes the default launch. */
} TuneParams;

/*
 * load_triangulation: validate desc, pack it for the walk and copy it to the current device. The
 * packed form holds, per triangle and edge, what one step of the walk of Sec. 5.1 reads: the
 * neighbour, the edge it is entered through, the vertex the next decision needs and the
 * primitive of a constrained edge (Sec. 5.1: a constrained exit edge ends the walk).
 * Validation (exact): vertex ids in range, every triangle strictly counter-clockwise, coordinates
 * finite with magnitude < 2^64, neighbours in range and symmetric with the shared edge reversed,
 * the same primitive on both sides of an edge, primitive ids in range, every constrained edge
 * collinear with its primitive, V - E + T = 1 over the referenced vertices. Failure returns
 * CCSP_E_BAD_TRIANGULATION and names the first offending triangle. On success *out owns the
 * device copy until free_triangulation. Host pointers are not retained. Synchronises `stream`.
 */
int load_triangulation(const TriangulationDesc *desc, void *stream, Triangulation **out);

/*
 * trace_rays: walk n rays through one triangulation (Sec. 5.1: from the start triangle, one exit
 * decision per triangle, stopping at a constrained edge or the hull; Sec. 5.4: steps counts the
 * triangles visited; the first triangle has three candidate exit edges and every later one two,
 * Sec. 7.2's footnote). All array arguments are DEVICE pointers
 * owned by the caller: o_xy and d_xy hold n interleaved (x,y) binary64 pairs (16-byte aligned),
 * start_tri n triangle ids; the outputs hit_prim, hit_t (8-byte aligned) and steps receive n
 * values each. d must be nonzero and the origin strictly inside start_tri. The call is
 * asynchronous on `stream` (except with CCSP_TRACE_VALIDATE).
 * Ray binning: unless CCSP_TRACE_INPUT_ORDER is set, a trace of n >= 65,536 rays through a
 * triangulation of at least 262,144 triangles first groups the rays by the cell of their origin
 * (the results do not depend on it; only the order in which rays are walked, hence cache reuse,
 * does). It uses per-device scratch of about 48 bytes per ray, allocated on the first binned
 * trace larger than any before unless reserve_workspace() reserved it; binned traces on
 * different streams of one device are serialised on the device.
 */
int trace_rays(const Triangulation *tri, const double *o_xy, const double *d_xy,
               const int32_t *start_tri, int64_t n, int precision, int32_t *hit_prim,
               double *hit_t, int32_t *steps, void *stream);

/* trace_rays_tuned: trace_rays (the walk of Sec. 5.1) with explicit tuning of the persistent launch
 * (tune may be NULL); results do not depend on the tuning. */
int trace_rays_tuned(const Triangulation *tri, const double *o_xy, const double *d_xy,
                     const int32_t *start_tri, int64_t n, int precision, int32_t *hit_prim,
                     double *hit_t, int32_t *steps, const TuneParams *tune, void *stream);

/*
 * trace_bounces: trace_rays with rays continued at hits (secondary rays, paper Sec. 5.2: the
 * final triangle of a traversal is the start of the next). At a hit, while fewer than
 * max_bounces reflections have been made, the ray is reflected specularly off the hit primitive
 * and walks on from the hit point in the triangle it ended in, which the reflected ray enters
 * through the hit edge; no new point location and no self-intersection with the primitive just
 * hit. Reflection in binary64, in this order, without fused operations: o' = o + t d;
 * n = (-ey, ex) with e = b - a of the primitive; k = (2 (d.n)) / (n.n); d' = d - k n. Outputs
 * (DEVICE, n each): hit_prim, hit_t and steps as in trace_rays but for the LAST segment (prim and
 * t) and over ALL segments (steps, the hit triangle counting in both segments); bounces: the
 * reflections made; hit_face (may be NULL): 4 * (caller's triangle) + edge of the last hit, -1
 * if the last segment did not hit. The step guard applies per segment. precision: a mode with
 * CCSP_TRACE_COUNT / INPUT_ORDER / TIMED (no VALIDATE). Asynchronous on `stream`.
 */
int trace_bounces(const Triangulation *tri, const double *o_xy, const double *d_xy,
                  const int32_t *start_tri, int64_t n, int32_t max_bounces, int precision,
                  int32_t *hit_prim, double *hit_t, int32_t *steps, int32_t *bounces,
                  int32_t *hit_face, const TuneParams *tune, void *stream);

/* One batch item: a triangulation and its rays (device pointers, as in trace_rays). */
typedef struct {
  const Triangulation *scene;
  const double *o_xy;
  const double *d_xy;
  const int32_t *start_tri;
  int64_t n;
  int32_t *hit_prim;
  double *hit_t;
  int32_t *steps;
} TraceItem;

/*
 * trace_batch: the walk of Sec. 5.1, as in trace_rays, for the rays of n_items items (possibly
 * different triangulations of uneven sizes) in one persistent launch, then finish them in one
 * more. `items` is a HOST array, read
 * during the call. Results equal those of one trace_rays per item; rays are walked in input order
 * (no binning). The item table goes to the device through library-owned rings of pinned and device
 * tables (allocated at the first call and when n_items exceeds every earlier call's), so batches
 * may run concurrently on different streams. With CCSP_TRACE_GRAPH the launch is replayed from a
 * HIP graph cached per (item count, tile count, mode, launch parameters), with its own item table
 * and tile counters; replays of one graph on different streams are ordered one after the other.
 * Asynchronous on `stream` (the call may block briefly while a pinned table's previous upload
 * completes).
 */
int trace_batch(const TraceItem *items, int32_t n_items, int precision, const TuneParams *tune,
                void *stream);

/*
 * autotune: choose launch parameters by measurement. With n_items == 1 and no CCSP_TRACE_GRAPH it
 * tunes trace_rays on that item, otherwise trace_batch on all items. `precision` is a mode,
 * optionally with CCSP_TRACE_GRAPH (batches) or CCSP_TRACE_INPUT_ORDER (single traces). Every
 * candidate is run once untimed and then `reps` times between two HIP events on `stream`; the
 * search is coordinate-wise from the defaults over waves_per_cu {8..28}, refill_min {4..48},
 * tile_rays {64, 128, 256}, wg_size {64..512}, tiles_per_claim {1..16} and xcd_chunks {1, 8}, two
 * passes. The items' outputs are overwritten by every run (with the same, correct results). On
 * success *best and *best_ms (mean milliseconds per call) hold the winner, which is also stored
 * in the current device's tuning cache: later trace_rays/trace_batch calls with tune == NULL on a
 * workload of the same shape (item count, total rays and total triangles rounded up to powers of
 * two, mode and flags) use it. Synchronises `stream`.
 */
int autotune(const TraceItem *items, int32_t n_items, int precision, int32_t reps,
             TuneParams *best, float *best_ms, void *stream);

/* tune_cache_set: store launch parameters for a workload shape (as autotune would; for reloading
 * results saved earlier). Launch parameters only: the walk (Sec. 5.1) and its results do not
 * depend on them. */
int tune_cache_set(int32_t n_items, int64_t total_rays, int64_t total_triangles, int precision,
                   const TuneParams *tune);
/* tune_cache_get: 1 and *out if the shape has an entry, 0 if not. */
int tune_cache_get(int32_t n_items, int64_t total_rays, int64_t total_triangles, int precision,
                   TuneParams *out);

/*
 * locate_points: the triangle containing each of n points (paper Sec. 5.2). q_xy: n interleaved
 * (x,y) binary64 pairs (DEVICE, 16-byte aligned); tri_out receives the caller's triangle id and
 * status: 0 = strictly inside tri_out, 1 = on an edge or vertex of tri_out (a ray may not start
 * there), -1 = outside the triangulation (tri_out -1), -2 = a coordinate not finite (tri_out -1).
 * Each point is reached by a walk from a seed point of a grid built at load (a point strictly
 * inside a known triangle per cell, about one cell per four triangles) along the exact segment
 * from the seed to the point, through constrained edges as through the others; decisions are
 * exact, so strict inclusion is decided exactly. Asynchronous on `stream`.
 */
int locate_points(const Triangulation *tri, const double *q_xy, int64_t n, int32_t *tri_out,
                  int32_t *status, void *stream);

/*
 * trace_rays_static: trace_rays_tuned for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). It calls no hipMalloc,
 * hipFree or allocating library routine: its scratch (the launch's tile counters and the ray
 * binning records) lives in one fixed device array of 80 MiB per GPU, part of the library's code
 * object, which each GPU the call runs on holds until the process ends. Results equal
 * trace_rays_tuned's on the same arguments. Differences: at most CCSP_STATIC_MAX_RAYS rays per call
 * (more: CCSP_E_ARG); precision takes a mode and CCSP_TRACE_INPUT_ORDER only (VALIDATE, COUNT and
 * TIMED: CCSP_E_ARG); tune == NULL means the default launch (the tuning cache is not consulted).
 * Every call on one GPU shares that GPU's array: calls whose executions overlap on the device
 * (other streams, other host threads) race and give wrong results; order them on one stream or
 * with events. The array keeps the last call's contents; each call clears what must start at zero
 * (with a kernel, not a memset). Asynchronous on `stream`.
 */
#define CCSP_STATIC_MAX_RAYS (1 << 20)
int trace_rays_static(const Triangulation *tri, const double *o_xy, const double *d_xy,
                      const int32_t *start_tri, int64_t n, int precision, int32_t *hit_prim,
                      double *hit_t, int32_t *steps, const TuneParams *tune, void *stream);

/* reserve_workspace: reserve the ray binning scratch for traces of up to max_rays rays on the
 * current device, so that later traces allocate nothing. */
int reserve_workspace(int64_t max_rays);

/* free_triangulation: release the device copy (synchronises the device first). NULL is a no-op. */
void free_triangulation(Triangulation *tri);

/* last_error: description of the last failure on this thread ("" if none). */
const char *last_error(void);

/*
 * read_counters: out[0] steps walked, out[1] binary32 decisions deferred to binary64,
 * out[2] binary64 decisions deferred to the exact expansion, out[3] rays traced, accumulated
 * over every trace made with CCSP_TRACE_COUNT on the current device since the last reset.
 * Synchronises the device. reset != 0 clears them after reading.
 */
int read_counters(uint64_t out[4], int reset);

/*
 * read_stage_times: stage durations of the most recent traces made with CCSP_TRACE_TIMED on the
 * current device, oldest first, measured with HIP events on each trace's stream. bin_ms[i] runs
 * from the start of the trace to the start of the walk kernel (the ray binning; about zero for a
 * trace that does not bin; the item-table upload for trace_batch), walk_ms[i] covers the walk
 * kernel alone, finish_ms[i] the finishing pass that writes the caller's arrays (a copy of the
 * parked results for a binned trace; for trace_batch with CCSP_TRACE_GRAPH the whole replayed
 * graph counts as walk and finish_ms[i] is zero).
 * The library keeps the last 256 timed traces per device; this call writes up to max_records of
 * the most recent ones, sets *n_records to their number, and forgets all kept records. Blocks
 * until those traces finish.
 */
int read_stage_times(int32_t max_records, float *bin_ms, float *walk_ms, float *finish_ms,
                     int32_t *n_records);

/* triangulation_info: out[0] triangles, out[1] vertices, out[2] primitives, out[3] device bytes. */
int triangulation_info(const Triangulation *tri, int64_t out[4]);

/*
 * gather_roofline: a measurement, not part of the walk. Chases a buffer of working_set_bytes
 * (rounded down to a power of two of 16-byte records, each pointing to a pseudo-random next one)
 * with waves_per_cu waves of 64 lanes per compute unit, each lane doing steps_per_lane dependent
 * 16-byte loads, and stores the sustained loads per second in *out_loads_per_s. This is the
 * memory pattern of one walk step, so the walk's steps per second over this rate (at a matching
 * working set) is its fraction of the gather roofline. Allocates and frees its own buffer and
 * synchronises `stream`.
 */
int gather_roofline(int64_t working_set_bytes, int32_t waves_per_cu, int64_t steps_per_lane,
                    double *out_loads_per_s, void *stream);

/* ------------------------------------------------------------------------------ request server
 *
 * Continuous batching of walk requests over resident triangulations, for callers that receive
 * rays on the host. Each request names a triangulation and brings host arrays (pinned memory,
 * e.g. from hipHostMalloc, lets its copies overlap other work; pageable memory works but
 * serialises the server). A worker thread admits pending requests in arrival order while a
 * launch slot is free and their device memory fits the server's pool, coalesces the admitted
 * requests (of any triangulations) into one trace_batch launch on the slot's stream between
 * their copies in and out, and reports each request once its results are in its host arrays.
 * Requests that arrive while launches are in flight are admitted as slots and memory free up,
 * so up to `slots` launches overlap on the device. Results are those of trace_rays on the same
 * rays (without binning, which does not change them). Errors go to last_error().
 */
typedef struct Server Server;

typedef struct {
  int32_t slots;         /* launches in flight at once, each on its own stream: 1..16 (0: 4) */
  int32_t max_items;     /* requests coalesced into one launch: 1..4096 (0: 256) */
  int64_t max_rays;      /* rays per launch; a single larger request still runs (0: 2^22) */
  int64_t memory_bytes;  /* device memory for admitted requests, >= 1 MiB (0: 1 GiB); a request
                            of n rays takes about 52 n bytes */
  int32_t precision;     /* a precision mode, without flags */
  int32_t reserved;
} ServerConfig;

/* server_create: allocate the pool and the slot streams on the current device and start the
 * worker thread. cfg may be NULL (defaults, binary64 mode). */
int server_create(const ServerConfig *cfg, Server **out);

/* server_submit: queue a request of n rays through `scene` (which must stay loaded until the
 * request completes). o_xy, d_xy, start_tri and the result arrays are HOST pointers that must
 * stay valid until server_poll reports the request. *id receives its id (ids increase from 1).
 * A request that could never fit the pool is rejected with CCSP_E_ARG. Thread-safe. */
int server_submit(Server *s, const Triangulation *scene, const double *o_xy, const double *d_xy,
                  const int32_t *start_tri, int64_t n, int32_t *hit_prim, double *hit_t,
                  int32_t *steps, uint64_t *id);

/* server_poll: take up to max completed requests, in completion order, waiting up to timeout_s
 * seconds for the first one: ids, status (CCSP_OK or an error code), and the submission and
 * completion times in seconds of CLOCK_MONOTONIC. *n_out receives the number taken. */
int server_poll(Server *s, int32_t max, uint64_t *ids, int32_t *status, double *t_submit,
                double *t_done, int32_t *n_out, double timeout_s);

/* server_stats: out[0] launches, out[1] requests admitted, out[2] rays admitted, out[3] most
 * requests in one launch, out[4] peak pool bytes in use, out[5] admission attempts stopped by a
 * full pool, out[6] most slots busy at once, out[7] requests pending now. */
int server_stats(Server *s, int64_t out[8]);

/* server_destroy: finish every queued and in-flight request, stop the worker, free the server
 * (completed requests not yet polled are dropped). NULL is a no-op. */
void server_destroy(Server *s);

#ifdef __cplusplus
}
#endif
#endif /* CCSP_WALK_H */
