"""Stackless ray walk through 2D constrained triangulations on MI355X (arXiv 2112.05570, Sec. 5).

Thin Python layer over libccsp_walk.so: :class:`Scene` owns a loaded triangulation, :func:`trace`
walks rays held in torch CUDA tensors, :func:`trace_batch` walks many scenes in one persistent
launch. PyTorch only provides device memory and streams; the walk itself runs in HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import binding as B
from .binding import (CCSP_RAY_BAD, CCSP_RAY_GUARD, CCSP_RAY_MISS, CCSP_TRACE_COUNT,
                      CCSP_TRACE_FP32_FILTERED, CCSP_TRACE_FP64, CCSP_TRACE_GRAPH,
                      CCSP_TRACE_INPUT_ORDER, CCSP_TRACE_TIMED, CCSP_TRACE_VALIDATE, CcspError,
                      TuneParams, read_stage_times, reserve_workspace)

PRECISION = {"fp64": CCSP_TRACE_FP64, "fp32": CCSP_TRACE_FP32_FILTERED}


def _mode(precision) -> int:
    return PRECISION[precision] if isinstance(precision, str) else int(precision)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Scene:
    """A triangulation resident on the current device."""

    def __init__(self, xy, tri_v, tri_nbr, tri_prim, prims, stream=None):
        xy, prims = _c(xy, np.float64), _c(prims, np.float64)
        tv, tn, tp = _c(tri_v, np.int32), _c(tri_nbr, np.int32), _c(tri_prim, np.int32)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
        desc = B.TriangulationDesc(xy.reshape(-1, 2).shape[0], p(xy), tv.reshape(-1, 3).shape[0],
                                   p(tv), p(tn), p(tp), prims.reshape(-1, 4).shape[0], p(prims))
        self.handle = None
        self.handle = B.load_triangulation(desc, _stream(stream) if stream is not None else 0)
        self.n_triangles, self.n_vertices, self.n_prims, self.device_bytes = \
            B.triangulation_info(self.handle)

    @classmethod
    def from_arrays(cls, scene, stream=None):
        """From any object with xy, tri_v, tri_nbr, tri_prim and prims arrays."""
        return cls(scene.xy, scene.tri_v, scene.tri_nbr, scene.tri_prim, scene.prims, stream)

    def free(self):
        if self.handle:
            B.free_triangulation(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


class TetMesh:
    """A 3D tetrahedralisation resident on the current device (include/ccsp_tet.h): integer grid
    coordinates in [0, 2^19), positively oriented tetrahedra, primitives among their faces."""

    def __init__(self, xyz, tet_v, tet_nbr, tet_prim, prims):
        xyz, tv, tn, tp, pr = (_c(a, np.int32) for a in (xyz, tet_v, tet_nbr, tet_prim, prims))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
        desc = B.TetMeshDesc(xyz.reshape(-1, 3).shape[0], p(xyz), tv.reshape(-1, 4).shape[0],
                             p(tv), p(tn), p(tp), pr.reshape(-1, 3).shape[0], p(pr))
        self.handle = None
        self.handle = B.load_tetmesh(desc)
        self.n_tets, self.device_bytes = B.tetmesh_info(self.handle)

    @classmethod
    def from_arrays(cls, scene):
        """From any object with xyz, tet_v, tet_nbr, tet_prim and prims arrays."""
        return cls(scene.xyz, scene.tet_v, scene.tet_nbr, scene.tet_prim, scene.prims)

    def free(self):
        if self.handle:
            B.free_tetmesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def trace3d_stage_times():
    """(binning ms, walk ms) of the device's last timed trace3d."""
    return B.trace3d_stage_times()


def trace3d(mesh: TetMesh, o, d, start, out: "Result | None" = None, step_limit: int = 0,
            tune: "B.Tune3d | None" = None, stream=None, input_order=False, timed=False):
    """Walk rays through a tetrahedralisation: o, d (n, 3) int32 and start (n,) int32 CUDA
    tensors. Returns a Result (hit_prim, hit_t, steps) in input order. Rays are binned by start
    tetrahedron first unless input_order; timed records stage events (trace3d_stage_times)."""
    import torch
    n = start.shape[0]
    for name, x, shape in (("o", o, (n, 3)), ("d", d, (n, 3)), ("start", start, (n,))):
        if not x.is_cuda or x.dtype != torch.int32 or tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous int32 CUDA tensor of shape {shape}")
    res = _outputs(n, start.device, out)
    flags = (B.CCSP_TRACE_INPUT_ORDER if input_order else 0) | (B.CCSP_TRACE_TIMED if timed else 0)
    B.trace_rays3d(mesh.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n, flags,
                   int(step_limit), tune, res.hit_prim.data_ptr(), res.hit_t.data_ptr(), res.steps.data_ptr(),
                   _stream(stream))
    return res


@dataclass
class Result:
    hit_prim: "torch.Tensor"
    hit_t: "torch.Tensor"
    steps: "torch.Tensor"


def _outputs(n, device, out):
    import torch
    if out is not None:
        return out
    return Result(torch.empty(n, dtype=torch.int32, device=device),
                  torch.empty(n, dtype=torch.float64, device=device),
                  torch.empty(n, dtype=torch.int32, device=device))


def _check_rays(o, d, start):
    import torch
    n = start.shape[0]
    for name, x, dt, shape in (("o", o, torch.float64, (n, 2)), ("d", d, torch.float64, (n, 2)),
                               ("start", start, torch.int32, (n,))):
        if not x.is_cuda or x.dtype != dt or tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of shape {shape}")
    return n


def trace(scene: Scene, o, d, start, precision="fp32", out: Result | None = None, stream=None,
          tune: TuneParams | None = None, validate=False, count=False,
          input_order=False, timed=False) -> Result:
    """Walk rays (o, d: (n,2) float64; start: (n,) int32 CUDA tensors). Asynchronous.
    input_order=True walks the rays in the given order instead of binning them spatially;
    timed=True records the stage durations read by read_stage_times()."""
    n = _check_rays(o, d, start)
    res = _outputs(n, o.device, out)
    mode = (_mode(precision) | (CCSP_TRACE_VALIDATE if validate else 0)
            | (CCSP_TRACE_COUNT if count else 0) | (CCSP_TRACE_INPUT_ORDER if input_order else 0)
            | (CCSP_TRACE_TIMED if timed else 0))
    B.trace_rays_tuned(scene.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n, mode,
                       res.hit_prim.data_ptr(), res.hit_t.data_ptr(), res.steps.data_ptr(), tune,
                       _stream(stream))
    return res


def trace_static(scene: Scene, o, d, start, out: Result, precision="fp32", stream=None,
                 tune: TuneParams | None = None, input_order=False) -> Result:
    """:func:`trace` through the entry point that allocates nothing (``trace_rays_static`` in the
    C header): at most CCSP_STATIC_MAX_RAYS rays, outputs passed in, one call at a time per GPU."""
    n = _check_rays(o, d, start)
    mode = _mode(precision) | (CCSP_TRACE_INPUT_ORDER if input_order else 0)
    B.trace_rays_static(scene.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n, mode,
                        out.hit_prim.data_ptr(), out.hit_t.data_ptr(), out.steps.data_ptr(), tune,
                        _stream(stream))
    return out


def _items(jobs):
    items, results = [], []
    for job in jobs:
        scene, o, d, start = job[:4]
        n = _check_rays(o, d, start)
        res = _outputs(n, o.device, job[4] if len(job) > 4 else None)
        results.append(res)
        items.append(B.TraceItem(scene.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n,
                                 res.hit_prim.data_ptr(), res.hit_t.data_ptr(),
                                 res.steps.data_ptr()))
    return items, results


def trace_batch(jobs, precision="fp32", tune: TuneParams | None = None, stream=None,
                graph=False, count=False, timed=False):
    """jobs: list of (Scene, o, d, start[, Result]). Returns the list of Results. tune=None uses
    the autotuned parameters for this workload shape if there are any."""
    items, results = _items(jobs)
    B.trace_batch(items, _mode(precision) | (CCSP_TRACE_COUNT if count else 0)
                  | (CCSP_TRACE_TIMED if timed else 0) | (CCSP_TRACE_GRAPH if graph else 0),
                  tune, _stream(stream))
    return results


def autotune(jobs, precision="fp32", graph=False, input_order=False, reps=3, stream=None,
             cache_path=None):
    """Launch parameters for this workload, chosen by measurement in the library (see
    ``autotune`` in the C header) and kept in its per-device cache, so that later traces of the
    same shape with tune=None use them. With ``cache_path`` the choice is also kept in a JSON file
    and a matching entry there is reused without measuring. One job without ``graph`` tunes
    :func:`trace`; otherwise :func:`trace_batch`. Returns (TuneParams, ms per call or None)."""
    import json
    import os
    flags = _mode(precision) | (CCSP_TRACE_GRAPH if graph else 0) | \
        (CCSP_TRACE_INPUT_ORDER if input_order else 0)
    shape = dict(n_items=len(jobs), rays=int(sum(j[3].shape[0] for j in jobs)),
                 triangles=int(sum(j[0].n_triangles for j in jobs)), precision=flags)
    entries = []
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            entries = json.load(f)
        for e in entries:
            B.tune_cache_set(e["n_items"], e["rays"], e["triangles"], e["precision"],
                             TuneParams(*e["params"]))
        hit = B.tune_cache_get(shape["n_items"], shape["rays"], shape["triangles"], flags)
        if hit is not None:
            return hit, None
    items, _ = _items(jobs)
    best, ms = B.autotune(items, flags, reps, _stream(stream))
    if cache_path:
        entries.append(dict(shape, params=list(best.as_tuple()), ms=ms))
        with open(cache_path, "w") as f:
            json.dump(entries, f, indent=1)
    return best, ms


def trace_bounces(scene: Scene, o, d, start, max_bounces, precision="fp32", stream=None,
                  tune: TuneParams | None = None, input_order=False, count=False):
    """Rays continued by specular reflection at hits, up to max_bounces times (see
    ``trace_bounces`` in the C header). Returns (Result of the last segment with steps over all
    segments, reflections made, last hit face 4*triangle+edge or -1). Asynchronous."""
    import torch
    n = _check_rays(o, d, start)
    res = _outputs(n, o.device, None)
    hits = torch.empty(n, dtype=torch.int32, device=o.device)
    face = torch.empty(n, dtype=torch.int32, device=o.device)
    mode = (_mode(precision) | (CCSP_TRACE_INPUT_ORDER if input_order else 0)
            | (CCSP_TRACE_COUNT if count else 0))
    B.trace_bounces(scene.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n, max_bounces,
                    mode, res.hit_prim.data_ptr(), res.hit_t.data_ptr(), res.steps.data_ptr(),
                    hits.data_ptr(), face.data_ptr(), tune, _stream(stream))
    return res, hits, face


def locate(scene: Scene, q, stream=None):
    """The triangle (caller's id) containing each point of q ((n,2) float64 CUDA tensor) and a
    status per point: 0 strictly inside, 1 on an edge or vertex, -1 outside, -2 not finite.
    Asynchronous."""
    import torch
    n = q.shape[0]
    if not q.is_cuda or q.dtype != torch.float64 or tuple(q.shape) != (n, 2) or not q.is_contiguous():
        raise ValueError("q must be a contiguous float64 CUDA tensor of shape (n, 2)")
    tri = torch.empty(n, dtype=torch.int32, device=q.device)
    status = torch.empty(n, dtype=torch.int32, device=q.device)
    B.locate_points(scene.handle, q.data_ptr(), n, tri.data_ptr(), status.data_ptr(),
                    _stream(stream))
    return tri, status


def contract(tri_v, kind, line, prim_v, xy, eps):
    """Contract the edges shorter than eps (see ``mesh_contract`` in ccsp_objective.h; host code).
    Arguments as for MovableMesh plus positions xy (V,2) float64 (numpy). Returns a dict of numpy
    arrays: tri_v, kind, line, xy of the contracted mesh, old_to_new (V,) and the number of
    contractions."""
    tri_v = np.ascontiguousarray(tri_v, dtype=np.int32)
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    line = np.ascontiguousarray(line, dtype=np.int32)
    prim_v = np.ascontiguousarray(prim_v, dtype=np.int32).reshape(-1, 2)
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    V, T = kind.shape[0], tri_v.shape[0]
    if tri_v.ndim != 2 or tri_v.shape[1] != 3 or line.shape != (V,) or xy.shape != (V, 2):
        raise ValueError("tri_v (T,3); kind, line (V,); xy (V,2)")
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    d = B.MeshDesc(V, p(kind), p(line), T, p(tri_v), prim_v.shape[0], p(prim_v))
    t_out = np.empty((T, 3), dtype=np.int32)
    k_out = np.empty(V, dtype=np.int32)
    l_out = np.empty(V, dtype=np.int32)
    xy_out = np.empty((V, 2), dtype=np.float64)
    m = np.empty(V, dtype=np.int32)
    counts = np.zeros(3, dtype=np.int64)  # triangles, vertices, contractions
    B.mesh_contract(d, p(xy), float(eps), p(t_out), p(counts[0:]), p(k_out), p(l_out), p(xy_out),
                    p(counts[1:]), p(m), p(counts[2:]))
    nt, nv = int(counts[0]), int(counts[1])
    return {"tri_v": t_out[:nt], "kind": k_out[:nv], "line": l_out[:nv], "xy": xy_out[:nv],
            "old_to_new": m, "contracted": int(counts[2])}


def subdivide(tri_v, kind, line, prim_v, xy):
    """The subdivision of Sec. 3.5.2 (see ``mesh_subdivide`` in ccsp_objective.h; host code):
    every triangle split into four at its edge midpoints. Arguments as for MovableMesh plus
    positions xy (V,2) float64. Returns (tri_v, kind, line, prim_v, xy) of the result (numpy)."""
    tri_v = np.ascontiguousarray(tri_v, dtype=np.int32)
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    line = np.ascontiguousarray(line, dtype=np.int32)
    prim_v = np.ascontiguousarray(prim_v, dtype=np.int32).reshape(-1, 2)
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    V, T = kind.shape[0], tri_v.shape[0]
    if tri_v.ndim != 2 or tri_v.shape[1] != 3 or line.shape != (V,) or xy.shape != (V, 2):
        raise ValueError("tri_v (T,3); kind, line (V,); xy (V,2)")
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    d = B.MeshDesc(V, p(kind), p(line), T, p(tri_v), prim_v.shape[0], p(prim_v))
    sizes = np.zeros(2, dtype=np.int64)
    B.mesh_subdivide(d, p(xy), p(sizes))
    nv, nt = int(sizes[0]), int(sizes[1])
    xo = np.empty((nv, 2), dtype=np.float64)
    to = np.empty((nt, 3), dtype=np.int32)
    ko = np.empty(nv, dtype=np.int32)
    lo = np.empty(nv, dtype=np.int32)
    B.mesh_subdivide(d, p(xy), p(sizes), p(xo), p(to), p(ko), p(lo))
    return to, ko, lo, prim_v, xo


class MovableMesh:
    """A triangulation with movable Steiner vertices for the low-weight objective (see
    ``mesh_load`` in ccsp_objective.h). Built from host arrays: tri_v (T,3) counter-clockwise,
    kind (V,) 0 original / 1 constrained / 2 free, line (V,) original edge of constrained
    vertices, prim_v (P,2) ends of each original edge. Positions are passed per call."""

    def __init__(self, tri_v, kind, line, prim_v):
        tri_v = np.ascontiguousarray(tri_v, dtype=np.int32)
        kind = np.ascontiguousarray(kind, dtype=np.int32)
        line = np.ascontiguousarray(line, dtype=np.int32)
        prim_v = np.ascontiguousarray(prim_v, dtype=np.int32).reshape(-1, 2)
        if tri_v.ndim != 2 or tri_v.shape[1] != 3 or kind.shape != line.shape or kind.ndim != 1:
            raise ValueError("tri_v must be (T,3); kind and line (V,)")
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
        d = B.MeshDesc(kind.shape[0], p(kind), p(line), tri_v.shape[0], p(tri_v), prim_v.shape[0],
                       p(prim_v))
        self.handle = None
        self.handle = B.mesh_load(d)
        self.n_vertices = int(kind.shape[0])
        self.n_triangles = int(tri_v.shape[0])
        self.movable = np.nonzero(kind != 0)[0].astype(np.int32)  # caller ids, increasing
        self.n_edges = B.mesh_info(self.handle)

    @classmethod
    def from_mesh(cls, mesh):
        return cls(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)

    def edges(self):
        out = np.empty((self.n_edges, 2), dtype=np.int32)
        B.mesh_info(self.handle, out.ctypes.data_as(ctypes.c_void_p).value)
        return out

    def _xy(self, xy):
        import torch
        if (not xy.is_cuda or xy.dtype != torch.float64 or tuple(xy.shape) != (self.n_vertices, 2)
                or not xy.is_contiguous()):
            raise ValueError("xy must be a contiguous float64 CUDA tensor of shape (V, 2)")
        return xy.data_ptr()

    def eval(self, xy, params, per_edge=False, stream=None):
        """f, w_contr, P_angle, P_len (a float64 CUDA tensor of 4) and, with per_edge, the
        contractible flags and weights of the edges. Asynchronous."""
        import torch
        out = torch.empty(4, dtype=torch.float64, device=xy.device)
        con = w = None
        if per_edge:
            con = torch.empty(self.n_edges, dtype=torch.uint8, device=xy.device)
            w = torch.empty(self.n_edges, dtype=torch.float64, device=xy.device)
        B.objective_eval(self.handle, self._xy(xy), params, out.data_ptr(),
                         con.data_ptr() if per_edge else 0, w.data_ptr() if per_edge else 0,
                         _stream(stream))
        return (out, con, w) if per_edge else out

    def delta(self, xy, params, vid, q, stream=None):
        """Change of f and status of each proposed move of vertex vid[i] to q[i] (int32 and
        (k,2) float64 CUDA tensors), each against xy. Asynchronous."""
        import torch
        k = vid.shape[0]
        if (not vid.is_cuda or vid.dtype != torch.int32 or not vid.is_contiguous() or not q.is_cuda
                or q.dtype != torch.float64 or tuple(q.shape) != (k, 2) or not q.is_contiguous()):
            raise ValueError("vid must be int32 (k,) and q float64 (k,2), contiguous CUDA tensors")
        d = torch.empty(k, dtype=torch.float64, device=xy.device)
        st = torch.empty(k, dtype=torch.int32, device=xy.device)
        B.objective_delta(self.handle, self._xy(xy), params, vid.data_ptr(), q.data_ptr(), k,
                          d.data_ptr(), st.data_ptr(), _stream(stream))
        return d, st

    def classes(self):
        """Classes of movable vertices (caller ids) whose moves do not interact."""
        n = B.mesh_classes(self.handle)
        off = np.empty(n + 1, dtype=np.int64)
        B.mesh_classes(self.handle, off.ctypes.data_as(ctypes.c_void_p).value)
        v = np.empty(int(off[-1]), dtype=np.int32)
        B.mesh_classes(self.handle, off.ctypes.data_as(ctypes.c_void_p).value,
                       v.ctypes.data_as(ctypes.c_void_p).value)
        return [v[off[i]:off[i + 1]] for i in range(n)]

    def anneal(self, xy, params, temperature, vid, disp, u, stream=None):
        """One Metropolis step for each move (see ``anneal_moves``); accepted positions are written
        into xy in place. Returns (delta, status). Asynchronous."""
        import torch
        k = vid.shape[0]
        if (not vid.is_cuda or vid.dtype != torch.int32 or not vid.is_contiguous()
                or tuple(disp.shape) != (k, 2) or disp.dtype != torch.float64
                or not disp.is_contiguous() or tuple(u.shape) != (k,) or u.dtype != torch.float64
                or not u.is_contiguous()):
            raise ValueError("vid int32 (k,), disp float64 (k,2), u float64 (k,): contiguous CUDA")
        d = torch.empty(k, dtype=torch.float64, device=xy.device)
        st = torch.empty(k, dtype=torch.int32, device=xy.device)
        B.anneal_moves(self.handle, self._xy(xy), params, float(temperature), vid.data_ptr(),
                       disp.data_ptr(), u.data_ptr(), k, d.data_ptr(), st.data_ptr(),
                       _stream(stream))
        return d, st

    def joint(self, xy, params, temperature, lam, vid, xi, u, stream=None):
        """One Metropolis step for one move of the distinct movable vertices vid (caller ids,
        int32 CUDA tensor) together, by lam * eta_i * xi[i] (xi (k,2) float64 CUDA unit draws; see
        ``anneal_joint``), u a float in [0, 1). xy is updated in place when the move is accepted.
        Returns (delta, status) as Python numbers. Synchronous."""
        import torch
        k = vid.shape[0]
        if (not vid.is_cuda or vid.dtype != torch.int32 or not vid.is_contiguous()
                or tuple(xi.shape) != (k, 2) or xi.dtype != torch.float64
                or not xi.is_contiguous() or not xi.is_cuda):
            raise ValueError("vid int32 (k,), xi float64 (k,2): contiguous CUDA tensors")
        return B.anneal_joint(self.handle, self._xy(xy), params, float(temperature), float(lam),
                              vid.data_ptr(), k, xi.data_ptr(), float(u), _stream(stream))

    def joint_groups(self, xy, params, temperature, lam, centres, draws, u, stream=None):
        """One Metropolis step for the group moves of the centres (caller ids, int32 CUDA tensor)
        made together (see ``anneal_joint_groups``): draws (n,4) float64 CUDA (xi.x, xi.y, r,
        unused), u a float in [0, 1). xy is updated in place when the move is accepted. Returns
        (delta, status) as Python numbers. Synchronous."""
        import torch
        n = centres.shape[0]
        if (not centres.is_cuda or centres.dtype != torch.int32 or not centres.is_contiguous()
                or tuple(draws.shape) != (n, 4) or draws.dtype != torch.float64
                or not draws.is_contiguous() or not draws.is_cuda):
            raise ValueError("centres int32 (n,), draws float64 (n,4): contiguous CUDA tensors")
        return B.anneal_joint_groups(self.handle, self._xy(xy), params, float(temperature),
                                     float(lam), centres.data_ptr(), n, draws.data_ptr(),
                                     float(u), _stream(stream))

    def sweep(self, xy, params, temperature, disp, u, stream=None):
        """One Metropolis step for every movable vertex, class by class (see ``anneal_sweep``):
        disp (M,2) and u (M,) float64 CUDA tensors in the order of ``classes()``. xy is updated in
        place. Returns (delta, status) in that order. Asynchronous."""
        import torch
        m = self.n_movable()
        if (tuple(disp.shape) != (m, 2) or disp.dtype != torch.float64 or not disp.is_contiguous()
                or not disp.is_cuda or tuple(u.shape) != (m,) or u.dtype != torch.float64
                or not u.is_contiguous() or not u.is_cuda):
            raise ValueError(f"disp float64 ({m},2) and u float64 ({m},), contiguous CUDA tensors")
        d = torch.empty(m, dtype=torch.float64, device=xy.device)
        st = torch.empty(m, dtype=torch.int32, device=xy.device)
        B.anneal_sweep(self.handle, self._xy(xy), params, float(temperature), disp.data_ptr(),
                       u.data_ptr(), d.data_ptr(), st.data_ptr(), _stream(stream))
        return d, st

    def propose(self, xy, params, temperature, kind, draws, u, stream=None):
        """One sweep with the proposals of Secs. 3.2.4-3.2.6 (see ``anneal_propose``): kind is
        "resample", "swap" or "contract"; draws (M,4) and u (M,) float64 CUDA tensors in the order
        of ``classes()``. xy is updated in place. Returns (delta, status). Asynchronous."""
        import torch
        kinds = {"resample": B.CCSP_PROPOSE_RESAMPLE, "swap": B.CCSP_PROPOSE_SWAP,
                 "contract": B.CCSP_PROPOSE_CONTRACT}
        if kind not in kinds:
            raise ValueError(f"kind must be one of {sorted(kinds)}")
        m = self.n_movable()
        if (tuple(draws.shape) != (m, 4) or draws.dtype != torch.float64
                or not draws.is_contiguous() or not draws.is_cuda or tuple(u.shape) != (m,)
                or u.dtype != torch.float64 or not u.is_contiguous() or not u.is_cuda):
            raise ValueError(f"draws float64 ({m},4) and u float64 ({m},), contiguous CUDA tensors")
        d = torch.empty(m, dtype=torch.float64, device=xy.device)
        st = torch.empty(m, dtype=torch.int32, device=xy.device)
        B.anneal_propose(self.handle, self._xy(xy), params, float(temperature), kinds[kind],
                         draws.data_ptr(), u.data_ptr(), d.data_ptr(), st.data_ptr(),
                         _stream(stream))
        return d, st

    def group_sweep(self, xy, params, temperature, lam, draws, u, centres=None, stream=None):
        """Group moves (see ``anneal_group``) for the centres (caller ids; default every movable
        vertex once, in increasing id): draws (M,4) (xi.x, xi.y, r, unused) and u (M,) float64
        CUDA tensors, one row per centre. xy is updated in place. Returns (delta, status, members,
        round) per centre; the result is that of the sequential chain over the centres in the
        order of increasing (round, index). Synchronous (one synchronisation per round)."""
        import torch
        if centres is None:
            centres = self.movable
        cen = torch.as_tensor(np.ascontiguousarray(centres, dtype=np.int32)).to(xy.device) \
            if not isinstance(centres, torch.Tensor) else centres.to(torch.int32).contiguous()
        m = cen.shape[0]
        if (tuple(draws.shape) != (m, 4) or draws.dtype != torch.float64
                or not draws.is_contiguous() or not draws.is_cuda or tuple(u.shape) != (m,)
                or u.dtype != torch.float64 or not u.is_contiguous() or not u.is_cuda):
            raise ValueError(f"draws float64 ({m},4) and u float64 ({m},), contiguous CUDA tensors")
        d = torch.empty(m, dtype=torch.float64, device=xy.device)
        st = torch.empty(m, dtype=torch.int32, device=xy.device)
        mem = torch.empty(m, dtype=torch.int32, device=xy.device)
        rnd = torch.empty(m, dtype=torch.int32, device=xy.device)
        B.anneal_group(self.handle, self._xy(xy), params, float(temperature), float(lam),
                       cen.data_ptr(), m, draws.data_ptr(), u.data_ptr(), d.data_ptr(),
                       st.data_ptr(), mem.data_ptr(), rnd.data_ptr(), _stream(stream))
        return d, st, mem, rnd

    def schedule(self, xy, params, temperatures, eps, lambda0, xi, u, target=0.23, stream=None):
        """Simulated annealing with a temperature and contraction-length schedule and an adaptive
        step scale (see ``anneal_schedule``): temperatures and eps are sequences of one value per
        sweep; xi (S, M, 2) and u (S, M) float64 CUDA tensors hold the unit draws of the movable
        vertices in the order of ``classes()``. xy is updated in place. Returns the step scale of
        every sweep and its accepted moves (numpy arrays). Synchronous."""
        import torch
        temps = np.ascontiguousarray(temperatures, dtype=np.float64)
        epss = np.ascontiguousarray(eps, dtype=np.float64)
        s, m = temps.shape[0], self.n_movable()
        if (epss.shape != (s,) or tuple(xi.shape) != (s, m, 2) or tuple(u.shape) != (s, m)
                or xi.dtype != torch.float64 or u.dtype != torch.float64 or not xi.is_cuda
                or not u.is_cuda or not xi.is_contiguous() or not u.is_contiguous()):
            raise ValueError(f"{s} eps values, xi float64 ({s},{m},2) and u ({s},{m}) CUDA tensors")
        lam = np.zeros(s, dtype=np.float64)
        acc = np.zeros(s, dtype=np.int64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
        B.anneal_schedule(self.handle, self._xy(xy), params, s, p(temps), p(epss), float(lambda0),
                          float(target), xi.data_ptr(), u.data_ptr(), p(lam), p(acc),
                          _stream(stream))
        return lam, acc

    def n_movable(self):
        n = B.mesh_classes(self.handle)
        off = np.empty(n + 1, dtype=np.int64)
        B.mesh_classes(self.handle, off.ctypes.data_as(ctypes.c_void_p).value)
        return int(off[-1])

    def close(self):
        if self.handle:
            B.mesh_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flip_anneal(xy, tri_v, tri_nbr, tri_prim, temperatures, seed, vertex_line=None, prim_v=None,
                stream=None):
    """Annealing by edge flips with the weight as energy (see ``flip_anneal`` in
    ccsp_objective.h): xy (V,2) float64 and tri_v, tri_nbr, tri_prim (T,3) int32 CUDA tensors, the
    latter three updated in place; one round per temperature. With Steiner vertices on original
    edges, vertex_line (V,) int32 (original edge of each such vertex, -1 otherwise) and prim_v
    (P,2) int32 CUDA tensors keep flips from making triangles flat on an original edge. Returns
    the flips of each round (numpy). Synchronous."""
    import torch
    for a, dt in ((tri_v, torch.int32), (tri_nbr, torch.int32), (tri_prim, torch.int32)):
        if not a.is_cuda or a.dtype != dt or a.dim() != 2 or a.shape[1] != 3 or not a.is_contiguous():
            raise ValueError("tri_v, tri_nbr, tri_prim must be contiguous int32 CUDA tensors (T,3)")
    if not xy.is_cuda or xy.dtype != torch.float64 or xy.dim() != 2 or xy.shape[1] != 2 \
            or not xy.is_contiguous():
        raise ValueError("xy must be a contiguous float64 CUDA tensor (V,2)")
    if tri_nbr.shape != tri_v.shape or tri_prim.shape != tri_v.shape:
        raise ValueError("tri_v, tri_nbr and tri_prim must have the same shape")
    lp, np_, pp = 0, 0, 0
    if vertex_line is not None:
        if (not vertex_line.is_cuda or vertex_line.dtype != torch.int32
                or tuple(vertex_line.shape) != (xy.shape[0],) or not vertex_line.is_contiguous()
                or prim_v is None or not prim_v.is_cuda or prim_v.dtype != torch.int32
                or prim_v.dim() != 2 or prim_v.shape[1] != 2 or not prim_v.is_contiguous()):
            raise ValueError("vertex_line (V,) and prim_v (P,2): contiguous int32 CUDA tensors")
        lp, np_, pp = vertex_line.data_ptr(), prim_v.shape[0], prim_v.data_ptr()
    temps = np.ascontiguousarray(temperatures, dtype=np.float64)
    counts = np.zeros(temps.shape[0], dtype=np.int64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    B.flip_anneal(xy.shape[0], xy.data_ptr(), tri_v.shape[0], tri_v.data_ptr(), tri_nbr.data_ptr(),
                  tri_prim.data_ptr(), lp, np_, pp, temps.shape[0], p(temps), int(seed), p(counts),
                  _stream(stream))
    return counts


def objective_params(eps, delta=None, eps0=1e-10, mu_angle=1.0, mu_len=10.0, polish=False):
    """Parameters of the objective (defaults: delta = cos(179 deg) + 1, the paper's eps0 and
    weights for a scene normalised to the unit square)."""
    import math
    if delta is None:
        delta = math.cos(math.radians(179.0)) + 1.0
    return B.ObjectiveParams(eps, delta, eps0, mu_angle, mu_len, int(bool(polish)), 0)


def read_counters(reset=False):
    """(steps, binary32 deferrals, binary64 deferrals, rays) since the last reset."""
    return B.read_counters(reset)


class Server:
    """Continuous-batching request server over resident scenes (see ``server_create`` in the C
    header). Requests bring host tensors (pinned memory lets their copies overlap); results are
    written into host tensors, which must stay alive until the request is reported done."""

    def __init__(self, precision="fp32", slots=4, max_items=256, max_rays=1 << 22,
                 memory_bytes=1 << 30):
        cfg = B.ServerConfig(slots, max_items, max_rays, memory_bytes, _mode(precision), 0)
        self.handle = None
        self.handle = B.server_create(cfg)
        self._live = {}

    def submit(self, scene: Scene, o, d, start, out: Result) -> int:
        """o, d: (n,2) float64, start: (n,) int32 CPU tensors; out: CPU Result of n rays."""
        n = start.shape[0]
        for name, x in (("o", o), ("d", d), ("start", start), ("hit_prim", out.hit_prim),
                        ("hit_t", out.hit_t), ("steps", out.steps)):
            if x.is_cuda or not x.is_contiguous() or x.shape[0] != n:
                raise ValueError(f"{name} must be a contiguous CPU tensor of {n} rows")
        rid = B.server_submit(self.handle, scene.handle, o.data_ptr(), d.data_ptr(),
                              start.data_ptr(), n, out.hit_prim.data_ptr(), out.hit_t.data_ptr(),
                              out.steps.data_ptr())
        self._live[rid] = (o, d, start, out)  # keep the host buffers alive while in flight
        return rid

    def poll(self, max_n=4096, timeout_s=0.0):
        """[(id, status, t_submit, t_done)] of completed requests (CLOCK_MONOTONIC seconds, the
        clock of time.monotonic())."""
        done = B.server_poll(self.handle, max_n, timeout_s)
        for rid, *_ in done:
            self._live.pop(rid, None)
        return done

    def stats(self) -> dict:
        keys = ("launches", "requests", "rays", "max_items_per_launch", "peak_pool_bytes",
                "admissions_stopped_by_memory", "max_slots_busy", "pending")
        return dict(zip(keys, B.server_stats(self.handle)))

    def close(self):
        if self.handle:
            B.server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
