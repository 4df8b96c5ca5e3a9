"""Seeded synthetic workloads for the triangulation ray walk.

This module only *produces inputs*: scenes of non-crossing line segments inside a bounding square,
their constrained Delaunay triangulation (plus an optional flip-annealed low-weight variant) and
rays with a known start triangle. It serves both the checker under ``oracle/`` and the walk
library, and contains none of the walk's arithmetic. The heavy lifting is C++ in ``csrc/``
(``libscenegen.so``, built by :func:`build`).

Workloads (paper: the "lines" scenes of Sec. 4.2 and the ray experiment of Sec. 5.4):

* ``tiny``   unit square + 64 segments, lengths U[0.02, 0.1]; 65,536 rays.
* ``grid``   256 x 256 lattice of unit segments trimmed to [0.1, 0.9], rotated 30 degrees about the
             centre; CDT and a flip-annealed triangulation; 2^22 rays.
* ``large``  10^6 segments, midpoints U[0,1000]^2, lengths log-U[0.01, 1]; box [-1,1001]^2; 2^26 rays.
* ``batch``  256 scenes as ``large`` with log-U[100, 10^5] segments and log-U[1024, 2^20] rays.
* ``serve``  64 resident scenes with log-U[10^3, 5*10^5] segments.

Conventions: vertices 0..3 are the box corners (counter-clockwise from the lower left); segment k
joins vertices 4+2k and 5+2k and is primitive k; the box sides bottom, right, top, left are
primitives S..S+3. Triangle arrays follow the walk library's descriptor: ``tri_v[t, i]`` counter-
clockwise, edge i opposite vertex i, ``tri_nbr[t, i]`` the triangle across edge i (-1 on the hull)
and ``tri_prim[t, i]`` the primitive of a constrained edge (-1 otherwise).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libscenegen.so")
_lib = None


def build() -> str:
    """Compile libscenegen.so with g++ (host code only)."""
    src = os.path.join(_HERE, "csrc", "scenegen.cpp")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB_PATH + ".tmp", src]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        P, I64, U64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        lib.sg_last_error.restype = ctypes.c_char_p
        lib.sg_random_segments.argtypes = [U64, I64, D, D, D, D, ctypes.c_int, D, D, P, I64]
        lib.sg_random_segments.restype = I64
        lib.sg_build_cdt.argtypes = [P, I64, P, P, I64, I32]
        lib.sg_build_cdt.restype = P
        lib.sg_mesh_from_arrays.argtypes = [P, I64, I64, P, P, P]
        lib.sg_mesh_from_arrays.restype = P
        lib.sg_mesh_ntri.argtypes = [P]
        lib.sg_mesh_ntri.restype = I64
        lib.sg_mesh_copy.argtypes = [P, P, P, P]
        lib.sg_mesh_weight.argtypes = [P]
        lib.sg_mesh_weight.restype = D
        lib.sg_mesh_anneal.argtypes = [P, U64, I64, D, D, P]
        lib.sg_mesh_anneal.restype = ctypes.c_int
        lib.sg_mesh_greedy.argtypes = [P]
        lib.sg_mesh_locate.argtypes = [P, I64, P, P]
        lib.sg_mesh_locate.restype = ctypes.c_int
        lib.sg_mesh_free.argtypes = [P]
        lib.sg_sample_rays.argtypes = [P, I64, P, U64, I64, P, P, P, ctypes.c_int]
        lib.sg_orient_batch.argtypes = [I64, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _err(msg):
    raise RuntimeError(f"{msg}: {_L().sg_last_error().decode()}")


# Per-purpose seed tags: every draw stream is derived from (seed, tag), so the scene, the rays
# and any later stream of the same workload never share random numbers.
TAG_SCENE, TAG_RAYS, TAG_ANNEAL, TAG_CHOICE, TAG_MOVES = 1, 2, 3, 4, 5


def subseed(seed: int, tag: int, index: int = 0) -> int:
    return (int(seed) * 1_000_003 + tag * 7919 + index * 104_729) & ((1 << 64) - 1)


@dataclass
class Scene:
    """A scene and its triangulation (all host numpy arrays)."""

    xy: np.ndarray          # (V,2) float64
    prims: np.ndarray       # (P,4) float64: ax, ay, bx, by
    seg_v: np.ndarray       # (S,2) int32 vertex ids of segment k (primitive k)
    box: tuple              # (lo, hi) of the bounding square
    tri_v: np.ndarray = None
    tri_nbr: np.ndarray = None
    tri_prim: np.ndarray = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self):
        return int(self.xy.shape[0])

    @property
    def n_triangles(self):
        return int(self.tri_v.shape[0])

    @property
    def n_prims(self):
        return int(self.prims.shape[0])

    def copy_with(self, tri_v, tri_nbr, tri_prim, name=None):
        return Scene(self.xy, self.prims, self.seg_v, self.box, tri_v, tri_nbr, tri_prim,
                     name or self.name, dict(self.meta))


def scene_from_segments(seg: np.ndarray, lo: float, hi: float, name: str = "") -> Scene:
    """Vertices, primitives and segment ids for segments seg (S,4) inside the square [lo,hi]^2."""
    seg = np.ascontiguousarray(seg, dtype=np.float64).reshape(-1, 4)
    S = seg.shape[0]
    corners = np.array([[lo, lo], [hi, lo], [hi, hi], [lo, hi]], dtype=np.float64)
    xy = np.concatenate([corners, seg.reshape(-1, 2)], axis=0)
    seg_v = (4 + np.arange(2 * S, dtype=np.int32)).reshape(S, 2)
    sides = np.array([[lo, lo, hi, lo], [hi, lo, hi, hi], [hi, hi, lo, hi], [lo, hi, lo, lo]],
                     dtype=np.float64)
    prims = np.concatenate([seg, sides], axis=0)
    return Scene(np.ascontiguousarray(xy), np.ascontiguousarray(prims), seg_v, (lo, hi), name=name)


def split_segments(sc: Scene) -> Scene:
    """The same scene (same primitives) with every segment constrained as two sub-segments that
    meet at its midpoint, which must be exactly representable and exactly on the segment (true
    for integer coordinates); the result is not yet triangulated."""
    S = sc.seg_v.shape[0]
    a = sc.xy[sc.seg_v[:, 0]]
    b = sc.xy[sc.seg_v[:, 1]]
    m = 0.5 * (a + b)
    on = exact_orient(np.concatenate([a, b, m], axis=1)) == 0
    if not on.all() or ((m == a).all(axis=1) | (m == b).all(axis=1)).any():
        raise ValueError("a segment midpoint is not exactly on its segment")
    V = sc.xy.shape[0]
    xy = np.concatenate([sc.xy, m], axis=0)
    mid = V + np.arange(S, dtype=np.int32)
    seg_v = np.stack([np.stack([sc.seg_v[:, 0], mid], 1), np.stack([mid, sc.seg_v[:, 1]], 1)],
                     1).reshape(-1, 2).astype(np.int32)
    meta = dict(sc.meta, seg_prim=np.repeat(np.arange(S, dtype=np.int32), 2))
    return Scene(np.ascontiguousarray(xy), sc.prims, np.ascontiguousarray(seg_v), sc.box,
                 name=sc.name + "+split", meta=meta)


def open_hull(sc: Scene, sides=(0, 1, 2, 3)) -> Scene:
    """The same triangulation with the given box sides (0 bottom, 1 right, 2 top, 3 left) no
    longer scene geometry: their hull edges become unconstrained, so a ray reaching them leaves
    the triangulation without a hit. The opened sides are dropped from the primitives and the
    kept sides renumbered after the segments, in their order."""
    S = sc.n_prims - 4
    if S < 0 or sc.tri_prim is None:
        raise ValueError("open_hull needs a triangulated scene whose last four primitives are the box sides")
    opened = sorted(set(int(k) for k in sides))
    if any(k < 0 or k > 3 for k in opened):
        raise ValueError("box sides are numbered 0..3")
    kept = [k for k in range(4) if k not in opened]
    remap = np.arange(sc.n_prims + 1, dtype=np.int64) - 1  # index p + 1 -> new id of p (-1 -> -1)
    for k in opened:
        remap[S + k + 1] = -1
    for j, k in enumerate(kept):
        remap[S + k + 1] = S + j
    tp = remap[sc.tri_prim.astype(np.int64) + 1].astype(np.int32)
    prims = np.ascontiguousarray(np.concatenate([sc.prims[:S], sc.prims[S + np.array(kept, dtype=np.int64)]])
                                 if kept else sc.prims[:S])
    meta = dict(sc.meta, open_sides=tuple(opened))
    return Scene(sc.xy, prims, sc.seg_v, sc.box, sc.tri_v, sc.tri_nbr, np.ascontiguousarray(tp),
                 sc.name + "+open" + "".join(str(k) for k in opened), meta)


ORIGINAL, CONSTRAINED, FREE = 0, 1, 2


@dataclass
class MovableMesh:
    """A triangulation with Steiner vertices, the input of the low-weight objective: vertex
    positions, counter-clockwise triangles, each vertex's kind (ORIGINAL, CONSTRAINED to original
    edge line[v], or FREE) and the two original vertices ending each original edge (prim_v)."""

    xy: np.ndarray       # (V,2) float64
    tri_v: np.ndarray    # (T,3) int32
    kind: np.ndarray     # (V,) int32
    line: np.ndarray     # (V,) int32, -1 unless CONSTRAINED
    prim_v: np.ndarray   # (P,2) int32
    name: str = ""

    @property
    def n_vertices(self):
        return int(self.xy.shape[0])

    @property
    def n_triangles(self):
        return int(self.tri_v.shape[0])


def movable_input(sc: Scene) -> tuple:
    """A scene's triangulation as the input of the low-weight optimiser, before any subdivision:
    (xy, tri_v, kind, line, prim_v) with every vertex ORIGINAL (line -1) and the original edges
    being the scene's segments followed by the four box sides."""
    if "seg_prim" in sc.meta:
        raise ValueError("movable_input expects one constrained edge per segment, unsplit")
    prim_v = np.concatenate([sc.seg_v, [[0, 1], [1, 2], [2, 3], [3, 0]]]).astype(np.int32)
    if prim_v.shape[0] != sc.n_prims:
        raise ValueError("scene primitives are not its segments plus four box sides")
    V = sc.n_vertices
    return (np.ascontiguousarray(sc.xy), np.ascontiguousarray(sc.tri_v, dtype=np.int32),
            np.full(V, ORIGINAL, dtype=np.int32), np.full(V, -1, dtype=np.int32), prim_v)


def vertex_moves(mesh: MovableMesh, n: int, seed: int, lam: float) -> tuple:
    """n proposed single-vertex moves (vertex ids, new positions) drawn as in Sec. 3.2.2: a movable
    vertex chosen uniformly; a displacement lam * eta * xi, where xi is a point uniform in the unit
    disk with its radius scaled by a Pareto(1/2) draw (x >= 1) and eta is the square root of the
    area of the vertex's triangles; projected on the original edge for constrained vertices."""
    rng = np.random.default_rng(subseed(seed, TAG_MOVES))
    movable = np.nonzero(mesh.kind != ORIGINAL)[0]
    v = movable[rng.integers(0, movable.shape[0], n)]
    u = rng.random((n, 3))
    r = np.sqrt(u[:, 0]) * (1.0 - u[:, 2]) ** -2.0
    th = 2.0 * np.pi * u[:, 1]
    p = mesh.xy[mesh.tri_v]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    star = np.bincount(mesh.tri_v.ravel(), weights=np.repeat(area, 3), minlength=mesh.n_vertices)
    d = (lam * np.sqrt(star[v]) * r)[:, None] * np.stack([np.cos(th), np.sin(th)], 1)
    con = mesh.kind[v] == CONSTRAINED
    if con.any():
        ends = mesh.prim_v[mesh.line[v[con]]]
        e = mesh.xy[ends[:, 1]] - mesh.xy[ends[:, 0]]
        k = (d[con] * e).sum(1) / (e * e).sum(1)
        d[con] = k[:, None] * e
    return v.astype(np.int32), np.ascontiguousarray(mesh.xy[v] + d)


def vertex_displacements(mesh: MovableMesh, vid, seed: int, lam: float) -> np.ndarray:
    """Displacements lam * eta * xi for the given vertices, drawn as in vertex_moves (not yet
    projected on original edges)."""
    vid = np.asarray(vid, dtype=np.int64)
    rng = np.random.default_rng(subseed(seed, TAG_MOVES, 1))
    u = rng.random((vid.shape[0], 3))
    r = np.sqrt(u[:, 0]) * (1.0 - u[:, 2]) ** -2.0
    th = 2.0 * np.pi * u[:, 1]
    p = mesh.xy[mesh.tri_v]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    star = np.bincount(mesh.tri_v.ravel(), weights=np.repeat(area, 3), minlength=mesh.n_vertices)
    return np.ascontiguousarray((lam * np.sqrt(star[vid]) * r)[:, None]
                                * np.stack([np.cos(th), np.sin(th)], 1))


def random_segments(seed, n, mid_lo, mid_hi, len_lo, len_hi, log_len, box_lo, box_hi,
                    max_draws=None) -> np.ndarray:
    out = np.empty((n, 4), dtype=np.float64)
    max_draws = max_draws or max(1000, 100 * n)
    m = _L().sg_random_segments(int(seed) & ((1 << 64) - 1), n, mid_lo, mid_hi, len_lo, len_hi,
                                int(log_len), box_lo, box_hi, _ptr(out), max_draws)
    if m < 0:
        _err("segment sampling failed")
    if m < n:
        raise RuntimeError(f"segment sampling placed only {m} of {n} segments")
    return out


def triangulate(sc: Scene) -> Scene:
    """Constrained Delaunay triangulation of the scene (fills tri_v / tri_nbr / tri_prim)."""
    L = _L()
    S = sc.seg_v.shape[0]
    segp = np.ascontiguousarray(sc.meta.get("seg_prim", np.arange(S, dtype=np.int32)), np.int32)
    n_seg_prims = sc.prims.shape[0] - 4
    h = L.sg_build_cdt(_ptr(sc.xy), sc.xy.shape[0], _ptr(sc.seg_v), _ptr(segp), S, n_seg_prims)
    if not h:
        _err("triangulation failed")
    try:
        T = L.sg_mesh_ntri(h)
        tv = np.empty((T, 3), np.int32)
        tn = np.empty((T, 3), np.int32)
        tp = np.empty((T, 3), np.int32)
        L.sg_mesh_copy(h, _ptr(tv), _ptr(tn), _ptr(tp))
    finally:
        L.sg_mesh_free(h)
    sc.tri_v, sc.tri_nbr, sc.tri_prim = tv, tn, tp
    return sc


def _mesh(sc: Scene):
    return _L().sg_mesh_from_arrays(_ptr(sc.xy), sc.xy.shape[0], sc.n_triangles, _ptr(sc.tri_v),
                                    _ptr(sc.tri_nbr), _ptr(sc.tri_prim))


def weight(sc: Scene) -> float:
    """Total edge length of the triangulation (the paper's weight)."""
    h = _mesh(sc)
    try:
        return float(_L().sg_mesh_weight(h))
    finally:
        _L().sg_mesh_free(h)


def anneal_flips(sc: Scene, seed: int, moves_per_edge: float = 6.0, t0_rel: float = 0.02,
                 t1_rel: float = 1e-4) -> tuple:
    """Flip-only simulated annealing of the triangulation, then greedy flips.

    Temperatures are relative to the box side (the paper normalises scenes to the unit square).
    Returns (annealed Scene, stats dict). If annealing ends heavier than greedy flipping of the
    input alone, the greedy result is returned instead, so the weight never exceeds the input's.
    """
    L = _L()
    side = sc.box[1] - sc.box[0]
    n_edges = (3 * sc.n_triangles) // 2
    n_moves = int(moves_per_edge * n_edges)
    out = np.zeros(5, np.float64)
    h = _mesh(sc)
    try:
        if L.sg_mesh_anneal(h, subseed(seed, TAG_ANNEAL), n_moves, t0_rel * side, t1_rel * side,
                            _ptr(out)) != 0:
            _err("annealing failed")
        T = L.sg_mesh_ntri(h)
        tv, tn, tp = (np.empty((T, 3), np.int32) for _ in range(3))
        L.sg_mesh_copy(h, _ptr(tv), _ptr(tn), _ptr(tp))
    finally:
        L.sg_mesh_free(h)
    stats = dict(w_start=out[0], w_end=out[1], proposals=out[2], accepted=out[3], flips=out[4])
    res = sc.copy_with(tv, tn, tp, name=sc.name + "/annealed")
    h = _mesh(sc)
    try:
        L.sg_mesh_greedy(h)
        w_greedy = float(L.sg_mesh_weight(h))
        if w_greedy < stats["w_end"]:
            T = L.sg_mesh_ntri(h)
            tv, tn, tp = (np.empty((T, 3), np.int32) for _ in range(3))
            L.sg_mesh_copy(h, _ptr(tv), _ptr(tn), _ptr(tp))
            res = sc.copy_with(tv, tn, tp, name=sc.name + "/greedy")
            stats["w_end"] = w_greedy
            stats["fallback"] = "greedy"
    finally:
        L.sg_mesh_free(h)
    return res, stats


def locate(sc: Scene, pts: np.ndarray) -> np.ndarray:
    """Triangle strictly containing each point, -1 if on an edge, vertex or outside."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    out = np.empty(pts.shape[0], np.int32)
    h = _mesh(sc)
    try:
        if _L().sg_mesh_locate(h, pts.shape[0], _ptr(pts), _ptr(out)) != 0:
            _err("point location failed")
    finally:
        _L().sg_mesh_free(h)
    return out


@dataclass
class Rays:
    o: np.ndarray       # (N,2) float64 origins
    d: np.ndarray       # (N,2) float64 directions (cos, sin), not renormalised
    start: np.ndarray   # (N,) int32 start triangle (origin strictly inside)

    @property
    def n(self):
        return int(self.start.shape[0])

    def slice(self, a, b):
        return Rays(self.o[a:b], self.d[a:b], self.start[a:b])

    def take(self, idx):
        return Rays(np.ascontiguousarray(self.o[idx]), np.ascontiguousarray(self.d[idx]),
                    np.ascontiguousarray(self.start[idx]))


def sample_rays(sc: Scene, n: int, seed: int, threads: int = 0) -> Rays:
    """Area-weighted start triangle, origin uniform inside it (strictly), angle U[0, 2pi)."""
    o = np.empty((n, 2), np.float64)
    d = np.empty((n, 2), np.float64)
    st = np.empty(n, np.int32)
    _L().sg_sample_rays(_ptr(sc.xy), sc.n_triangles, _ptr(sc.tri_v), subseed(seed, TAG_RAYS), n,
                        _ptr(o), _ptr(d), _ptr(st), int(threads))
    return Rays(o, d, st)


def exact_orient(abc: np.ndarray) -> np.ndarray:
    abc = np.ascontiguousarray(abc, dtype=np.float64).reshape(-1, 6)
    out = np.empty(abc.shape[0], np.int32)
    _L().sg_orient_batch(abc.shape[0], _ptr(abc), _ptr(out))
    return out


# ----------------------------------------------------------------------------- workloads
def _rot30(p, c):
    cs, sn = math.cos(math.radians(30.0)), math.sin(math.radians(30.0))
    x, y = p[..., 0] - c, p[..., 1] - c
    return np.stack([c + cs * x - sn * y, c + sn * x + cs * y], axis=-1)


def grid_segments(n: int = 256, trim: float = 0.1) -> tuple:
    """Unit segments between 4-neighbours of the n x n lattice, trimmed to [trim, 1-trim] of
    their span and rotated 30 degrees about the lattice centre. Horizontal segments first (row
    by row), then vertical ones (column by column). Returns (segments (S,4), box lo, box hi)."""
    i = np.arange(n - 1, dtype=np.float64)
    j = np.arange(n, dtype=np.float64)
    J, I = np.meshgrid(j, i, indexing="ij")           # horizontal: row j, column i
    h = np.stack([I + trim, J, I + 1 - trim, J], axis=-1).reshape(-1, 4)
    I2, J2 = np.meshgrid(j, i, indexing="ij")          # vertical: column I2, row J2
    v = np.stack([I2, J2 + trim, I2, J2 + 1 - trim], axis=-1).reshape(-1, 4)
    seg = np.concatenate([h, v], axis=0)
    c = (n - 1) / 2.0
    a = _rot30(seg[:, 0:2], c)
    b = _rot30(seg[:, 2:4], c)
    seg = np.concatenate([a, b], axis=1)
    half = 0.5 * (n - 1) * (math.cos(math.radians(30)) + math.sin(math.radians(30))) + 1.0
    return np.ascontiguousarray(seg), c - half, c + half


WORKLOADS = {
    "tiny": dict(kind="random", n_seg=64, mid=(0.0, 1.0), length=(0.02, 0.1), log_len=False,
                 box=(0.0, 1.0), rays=65536),
    "grid": dict(kind="grid", n=256, rays=1 << 22),
    "large": dict(kind="random", n_seg=1_000_000, mid=(0.0, 1000.0), length=(0.01, 1.0),
                  log_len=True, box=(-1.0, 1001.0), rays=1 << 26),
    "batch": dict(kind="multi", n_scenes=256, n_seg=(100, 100_000), rays=(1024, 1 << 20),
                  mid=(0.0, 1000.0), length=(0.01, 1.0), box=(-1.0, 1001.0)),
    "serve": dict(kind="multi", n_scenes=64, n_seg=(1000, 500_000), rays=(256, 262_144),
                  mid=(0.0, 1000.0), length=(0.01, 1.0), box=(-1.0, 1001.0)),
}


def log_uniform_int(u: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """round(exp(U[ln lo, ln hi])) for uniforms u in [0,1)."""
    return np.rint(np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)).astype(np.int64)


def make_scene(name: str, seed: int = 0, n_seg: int | None = None, index: int = 0) -> Scene:
    """Build the scene of a workload (without rays) and its CDT."""
    w = WORKLOADS[name]
    if w["kind"] == "grid":
        seg, lo, hi = grid_segments(w["n"])
        sc = scene_from_segments(seg, lo, hi, name=name)
    else:
        n = int(n_seg if n_seg is not None else w["n_seg"])
        seg = random_segments(subseed(seed, TAG_SCENE, index), n, w["mid"][0], w["mid"][1],
                              w["length"][0], w["length"][1], w.get("log_len", True),
                              w["box"][0], w["box"][1])
        sc = scene_from_segments(seg, w["box"][0], w["box"][1], name=f"{name}[{index}]")
    return triangulate(sc)


def multi_workload(name: str, seed: int = 0, count: int | None = None,
                   max_seg: int | None = None, max_rays: int | None = None):
    """Yield (index, Scene, Rays) for the scenes of a multi-scene workload, in order. Scene i uses
    the segment stream of index i and the ray stream subseed(seed, TAG_RAYS, i + 1); max_seg and
    max_rays cap the drawn sizes (for small tests)."""
    segs, nrays = multi_sizes(name, seed)
    for i in range(len(segs) if count is None else count):
        ns = int(segs[i] if max_seg is None else min(segs[i], max_seg))
        nr = int(nrays[i] if max_rays is None else min(nrays[i], max_rays))
        sc = make_scene(name, seed, n_seg=ns, index=i)
        yield i, sc, sample_rays(sc, nr, seed=subseed(seed, TAG_RAYS, i + 1))


def multi_sizes(name: str, seed: int = 0) -> tuple:
    """Segment and ray counts of the scenes of a multi-scene workload (log-uniform draws)."""
    w = WORKLOADS[name]
    rng = np.random.default_rng(np.random.SeedSequence([seed, TAG_CHOICE]))
    u = rng.random((w["n_scenes"], 2))
    segs = log_uniform_int(u[:, 0], *w["n_seg"])
    rays = log_uniform_int(u[:, 1], *w["rays"])
    return segs, rays


# ---------------------------------------------------------------- 3D: tetrahedralisations
#
# Inputs of the 3D walk: vertices on the integer grid 0 <= x, y, z < 2^19, ray origins on the same
# grid and integer directions with |components| <= 2^19, so that every orientation and Plücker
# sign of the walk is an exact int64 computation. The tetrahedralisation is the Delaunay one of
# seeded random grid points (scipy/Qhull), each tetrahedron positively oriented (checked exactly);
# the scene's primitives are faces of it: every hull face and a seeded fraction of the interior
# faces, so that the tetrahedralisation is a constrained one for them without a constrained
# builder.

GRID3 = 1 << 19


@dataclass
class TetScene:
    xyz: np.ndarray       # (V,3) int32 grid coordinates
    tet_v: np.ndarray     # (T,4) int32, orient3d(v0, v1, v2, v3) > 0
    tet_nbr: np.ndarray   # (T,4) int32, the tetrahedron across face i (opposite v[i]); -1 hull
    tet_prim: np.ndarray  # (T,4) int32, primitive of face i, -1 if not scene geometry
    prims: np.ndarray     # (P,3) int32 vertex ids of each primitive triangle
    name: str = ""

    @property
    def n_vertices(self):
        return int(self.xyz.shape[0])

    @property
    def n_tets(self):
        return int(self.tet_v.shape[0])

    @property
    def n_prims(self):
        return int(self.prims.shape[0])


# the faces of a tetrahedron, opposite v[i], as seen from outside when v0..v3 is positive
TET_FACES = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))


def orient3_int(a, b, c, d):
    """det[b - a; c - a; d - a] over int64 rows (exact for grid coordinates)."""
    a, b, c, d = (np.asarray(x, dtype=np.int64) for x in (a, b, c, d))
    # contiguous columns: strided column views make the products several times slower
    (u0, u1, u2), (v0, v1, v2), (w0, w1, w2) = (
        [np.ascontiguousarray(x[..., k] - a[..., k]) for k in range(3)] for x in (b, c, d))
    return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0)


def make_tet_scene(n_points: int, seed: int, frac_prims: float = 0.15, open_hull=False) -> TetScene:
    """The Delaunay tetrahedralisation of n_points seeded grid points with every hull face and a
    seeded fraction of the interior faces as primitives (open_hull: hull faces are not)."""
    from scipy.spatial import Delaunay
    for attempt in range(20):
        rng = np.random.default_rng(np.random.SeedSequence([seed, TAG_SCENE, 3, attempt]))
        pts = np.unique(rng.integers(0, GRID3, (n_points, 3)), axis=0)
        rng.shuffle(pts)
        dl = Delaunay(pts.astype(np.float64))
        tv = dl.simplices.astype(np.int64)
        nb = dl.neighbors.astype(np.int64)
        o = orient3_int(*(pts[tv[:, i]].astype(np.int64) for i in range(4)))
        if (o == 0).any():
            continue  # a flat tetrahedron: draw the points again
        neg = o < 0
        tv[neg] = tv[neg][:, [1, 0, 2, 3]]
        nb[neg] = nb[neg][:, [1, 0, 2, 3]]
        break
    else:
        raise RuntimeError("no tetrahedralisation without flat tetrahedra")
    T = tv.shape[0]
    # faces named by (tet, i), each interior face once (from its lower tetrahedron), in row order;
    # one uniform draw per interior face decides whether it is a primitive
    t_idx, i_idx = np.nonzero((nb < 0) | (nb > np.arange(T)[:, None]))
    n_idx = nb[t_idx, i_idx]
    face_rng = np.random.default_rng(np.random.SeedSequence([seed, TAG_SCENE, 4]))
    u = face_rng.random(t_idx.shape[0])
    chosen = np.where(n_idx < 0, not open_hull, u < frac_prims)
    t_c, i_c, n_c = t_idx[chosen], i_idx[chosen], n_idx[chosen]
    k = np.arange(t_c.shape[0])
    prim = -np.ones((T, 4), dtype=np.int64)
    prim[t_c, i_c] = k
    inner = n_c >= 0
    j = np.argmax(nb[n_c[inner]] == t_c[inner][:, None], axis=1)
    prim[n_c[inner], j] = k[inner]
    faces = np.array(TET_FACES)
    plist = np.stack([tv[t_c, faces[i_c, 0]], tv[t_c, faces[i_c, 1]], tv[t_c, faces[i_c, 2]]], 1)
    return TetScene(np.ascontiguousarray(pts, dtype=np.int32), np.ascontiguousarray(tv, dtype=np.int32),
                    np.ascontiguousarray(nb, dtype=np.int32), np.ascontiguousarray(prim, dtype=np.int32),
                    np.ascontiguousarray(plist, dtype=np.int32).reshape(-1, 3),
                    name=f"tets[{n_points}]" + ("+open" if open_hull else ""))


@dataclass
class Rays3:
    o: np.ndarray       # (n,3) int32 grid points
    d: np.ndarray       # (n,3) int32 nonzero
    start: np.ndarray   # (n,) int32

    @property
    def n(self):
        return int(self.start.shape[0])

    def slice(self, a, b):
        return Rays3(self.o[a:b], self.d[a:b], self.start[a:b])


def sample_rays3(sc: TetScene, n: int, seed: int) -> Rays3:
    """Rays with a start tetrahedron drawn by volume, an origin uniform inside it rounded to the
    grid (drawn again until strictly inside, decided exactly), and an isotropic direction scaled
    to 2^19 and rounded (never zero)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, TAG_RAYS, 3]))
    P = sc.xyz.astype(np.int64)
    vol = orient3_int(*(P[sc.tet_v[:, i]] for i in range(4))).astype(np.float64)
    cdf = np.cumsum(vol) / vol.sum()
    o = np.empty((n, 3), dtype=np.int64)
    st = np.empty(n, dtype=np.int64)
    todo = np.arange(n)
    while todo.size:
        k = todo.size
        t = np.minimum(np.searchsorted(cdf, rng.random(k), side="right"), sc.n_tets - 1)
        b = -np.log(rng.random((k, 4)))  # uniform barycentric coordinates
        b /= b.sum(axis=1, keepdims=True)
        V = P[sc.tet_v[t]]
        q = np.rint(np.einsum("ki,kij->kj", b, V.astype(np.float64))).astype(np.int64)
        inside = np.ones(k, dtype=bool)
        for i in range(4):
            f = TET_FACES[i]
            inside &= orient3_int(V[:, f[0]], V[:, f[1]], V[:, f[2]], q) < 0
        o[todo[inside]] = q[inside]
        st[todo[inside]] = t[inside]
        todo = todo[~inside]
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    d = np.rint(g * (GRID3 - 1)).astype(np.int64)
    zero = (d == 0).all(axis=1)
    d[zero] = [1, 0, 0]
    return Rays3(o.astype(np.int32), d.astype(np.int32), st.astype(np.int32))
