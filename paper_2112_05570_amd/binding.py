"""ctypes binding of libccsp_walk.so (include/ccsp_walk.h), same names as the C ABI.

Argument marshalling only: every step of the walk runs in the library's HIP kernels. Device
buffers are passed as raw pointers (torch tensors on the GPU via ``data_ptr()``), streams as
``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``). The module raises at import
if the library is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccsp_walk.so")

# The library must bind to the HIP runtime that owns the caller's device memory and streams.
# PyTorch ships its own libamdhip64; loading it first makes the dynamic linker resolve the
# library's libamdhip64.so.7 dependency to that already-loaded runtime instead of a second copy.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(the walk has no non-HIP implementation)")

_lib = ctypes.CDLL(LIB_PATH)

CCSP_OK = 0
CCSP_E_ARG = -1
CCSP_E_BAD_TRIANGULATION = -2
CCSP_E_OOM = -3
CCSP_E_HIP = -4
CCSP_E_BAD_RAY = -5
CCSP_RAY_MISS = -1
CCSP_RAY_GUARD = -2
CCSP_RAY_BAD = -3
CCSP_TRACE_FP64 = 0
CCSP_TRACE_FP32_FILTERED = 1
CCSP_TRACE_VALIDATE = 1 << 8
CCSP_TRACE_COUNT = 1 << 9
CCSP_TRACE_INPUT_ORDER = 1 << 10
CCSP_TRACE_TIMED = 1 << 11
CCSP_TRACE_GRAPH = 1 << 12
CCSP_MOVE_SKIPPED = 3
CCSP_MOVE_FIXED, CCSP_MOVE_BAD = -1, -2
CCSP_PROPOSE_DISPLACE, CCSP_PROPOSE_RESAMPLE, CCSP_PROPOSE_SWAP, CCSP_PROPOSE_CONTRACT = 0, 1, 2, 3

EXPORTS = ("load_triangulation", "trace_rays", "trace_rays_tuned", "trace_batch",
           "free_triangulation", "last_error", "read_counters", "triangulation_info",
           "reserve_workspace", "gather_roofline", "read_stage_times", "autotune",
           "tune_cache_set", "tune_cache_get", "server_create", "server_submit", "server_poll",
           "server_stats", "server_destroy", "locate_points", "trace_bounces", "mesh_load",
           "mesh_info", "objective_eval", "objective_delta", "mesh_free", "mesh_classes",
           "anneal_moves", "anneal_joint", "anneal_joint_groups", "anneal_sweep", "anneal_propose", "anneal_schedule",
           "flip_anneal", "mesh_contract", "anneal_group",
           "trace_rays_static", "mesh_subdivide",
           "load_tetmesh", "free_tetmesh", "tetmesh_info", "trace_rays3d",
           "trace3d_stage_times")


class TriangulationDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("xy", ctypes.c_void_p),
                ("n_triangles", ctypes.c_int64), ("tri_v", ctypes.c_void_p),
                ("tri_nbr", ctypes.c_void_p), ("tri_prim", ctypes.c_void_p),
                ("n_prims", ctypes.c_int64), ("prim_seg", ctypes.c_void_p)]


class TuneParams(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("tile_rays", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("refill_min", ctypes.c_int32),
                ("tiles_per_claim", ctypes.c_int32), ("xcd_chunks", ctypes.c_int32),
                ("bin", ctypes.c_int32), ("step_limit", ctypes.c_int32)]

    def as_tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_[:-1])


class TraceItem(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("o_xy", ctypes.c_void_p), ("d_xy", ctypes.c_void_p),
                ("start_tri", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("hit_prim", ctypes.c_void_p), ("hit_t", ctypes.c_void_p),
                ("steps", ctypes.c_void_p)]


_P, _I, _I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
_lib.load_triangulation.argtypes = [ctypes.POINTER(TriangulationDesc), _P, ctypes.POINTER(_P)]
_lib.load_triangulation.restype = _I
_lib.trace_rays.argtypes = [_P, _P, _P, _P, _I64, _I, _P, _P, _P, _P]
_lib.trace_rays.restype = _I
_lib.trace_rays_tuned.argtypes = [_P, _P, _P, _P, _I64, _I, _P, _P, _P,
                                  ctypes.POINTER(TuneParams), _P]
_lib.trace_rays_tuned.restype = _I
_lib.trace_rays_static.argtypes = [_P, _P, _P, _P, _I64, _I, _P, _P, _P,
                                   ctypes.POINTER(TuneParams), _P]
_lib.trace_rays_static.restype = _I
_lib.trace_batch.argtypes = [ctypes.POINTER(TraceItem), ctypes.c_int32, _I,
                             ctypes.POINTER(TuneParams), _P]
_lib.trace_batch.restype = _I
_lib.free_triangulation.argtypes = [_P]
_lib.free_triangulation.restype = None
_lib.last_error.argtypes = []
_lib.last_error.restype = ctypes.c_char_p
_lib.read_counters.argtypes = [ctypes.POINTER(ctypes.c_uint64 * 4), _I]
_lib.read_counters.restype = _I
_lib.triangulation_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64 * 4)]
_lib.triangulation_info.restype = _I
_lib.reserve_workspace.argtypes = [_I64]
_lib.reserve_workspace.restype = _I
_lib.gather_roofline.argtypes = [_I64, ctypes.c_int32, _I64, ctypes.POINTER(ctypes.c_double), _P]
_lib.gather_roofline.restype = _I
_lib.read_stage_times.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(ctypes.c_int32)]
_lib.read_stage_times.restype = _I
_lib.autotune.argtypes = [ctypes.POINTER(TraceItem), ctypes.c_int32, _I, ctypes.c_int32,
                          ctypes.POINTER(TuneParams), ctypes.POINTER(ctypes.c_float), _P]
_lib.autotune.restype = _I
_lib.tune_cache_set.argtypes = [ctypes.c_int32, _I64, _I64, _I, ctypes.POINTER(TuneParams)]
_lib.tune_cache_set.restype = _I
_lib.tune_cache_get.argtypes = [ctypes.c_int32, _I64, _I64, _I, ctypes.POINTER(TuneParams)]
_lib.tune_cache_get.restype = _I
_lib.locate_points.argtypes = [_P, _P, _I64, _P, _P, _P]
_lib.locate_points.restype = _I
_lib.trace_bounces.argtypes = [_P, _P, _P, _P, _I64, ctypes.c_int32, _I, _P, _P, _P, _P, _P,
                               ctypes.POINTER(TuneParams), _P]
_lib.trace_bounces.restype = _I


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_items", ctypes.c_int32),
                ("max_rays", ctypes.c_int64), ("memory_bytes", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib.server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]
_lib.server_create.restype = _I
_lib.server_submit.argtypes = [_P, _P, _P, _P, _P, _I64, _P, _P, _P, ctypes.POINTER(ctypes.c_uint64)]
_lib.server_submit.restype = _I
_lib.server_poll.argtypes = [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                             ctypes.c_double]
_lib.server_poll.restype = _I
_lib.server_stats.argtypes = [_P, ctypes.POINTER(ctypes.c_int64 * 8)]
_lib.server_stats.restype = _I
_lib.server_destroy.argtypes = [_P]
_lib.server_destroy.restype = None


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("kind", ctypes.c_void_p),
                ("line", ctypes.c_void_p), ("n_triangles", ctypes.c_int64),
                ("tri_v", ctypes.c_void_p), ("n_prims", ctypes.c_int64),
                ("prim_v", ctypes.c_void_p)]


class ObjectiveParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("delta", ctypes.c_double), ("eps0", ctypes.c_double),
                ("mu_angle", ctypes.c_double), ("mu_len", ctypes.c_double),
                ("polish", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib.mesh_subdivide.argtypes = [ctypes.POINTER(MeshDesc), _P, _P, _P, _P, _P, _P, _P]
_lib.mesh_subdivide.restype = _I
_lib.mesh_load.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(_P)]
_lib.mesh_load.restype = _I
_lib.mesh_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), _P]
_lib.mesh_info.restype = _I
_lib.objective_eval.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), _P, _P, _P, _P]
_lib.objective_eval.restype = _I
_lib.objective_delta.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), _P, _P, _I64, _P, _P, _P]
_lib.objective_delta.restype = _I
_lib.mesh_free.argtypes = [_P]
_lib.mesh_free.restype = None
_lib.mesh_classes.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), _P, _P]
_lib.mesh_classes.restype = _I
_lib.anneal_moves.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double, _P, _P, _P,
                              _I64, _P, _P, _P]
_lib.anneal_moves.restype = _I
_lib.anneal_joint.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double,
                              ctypes.c_double, _P, _I64, _P, ctypes.c_double, _P, _P, _P]
_lib.anneal_joint.restype = _I
_lib.anneal_joint_groups.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double,
                                     ctypes.c_double, _P, _I64, _P, ctypes.c_double, _P, _P, _P]
_lib.anneal_joint_groups.restype = _I
_lib.anneal_sweep.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double, _P, _P, _P,
                              _P, _P]
_lib.anneal_sweep.restype = _I
_lib.anneal_propose.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double,
                                ctypes.c_int32, _P, _P, _P, _P, _P]
_lib.anneal_propose.restype = _I
_lib.anneal_schedule.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_int32, _P, _P,
                                 ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P]
_lib.anneal_schedule.restype = _I
_lib.flip_anneal.argtypes = [_I64, _P, _I64, _P, _P, _P, _P, _I64, _P, ctypes.c_int32, _P,
                             ctypes.c_uint64, _P, _P]
_lib.flip_anneal.restype = _I
_lib.mesh_contract.argtypes = [ctypes.POINTER(MeshDesc), _P, ctypes.c_double, _P, _P, _P, _P, _P,
                               _P, _P, _P]
_lib.mesh_contract.restype = _I
_lib.anneal_group.argtypes = [_P, _P, ctypes.POINTER(ObjectiveParams), ctypes.c_double,
                              ctypes.c_double, _P, _I64, _P, _P, _P, _P, _P, _P, _P]
_lib.anneal_group.restype = _I


# ---- include/ccsp_tet.h

class TetMeshDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("n_tets", ctypes.c_int64), ("tet_v", ctypes.c_void_p),
                ("tet_nbr", ctypes.c_void_p), ("tet_prim", ctypes.c_void_p),
                ("n_prims", ctypes.c_int64), ("prims", ctypes.c_void_p)]


class Tune3d(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("rays_per_claim", ctypes.c_int32), ("refill_min", ctypes.c_int32),
                ("bin_key", ctypes.c_int32)]


_lib.load_tetmesh.argtypes = [ctypes.POINTER(TetMeshDesc), ctypes.POINTER(_P)]
_lib.load_tetmesh.restype = _I
_lib.free_tetmesh.argtypes = [_P]
_lib.free_tetmesh.restype = _I
_lib.tetmesh_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.tetmesh_info.restype = _I
_lib.trace_rays3d.argtypes = [_P, _P, _P, _P, _I64, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(Tune3d), _P, _P, _P, _P]
_lib.trace_rays3d.restype = _I
_lib.trace3d_stage_times.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
_lib.trace3d_stage_times.restype = _I


class CcspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccsp error {code}: {msg}")
        self.code = code


def last_error() -> str:
    return _lib.last_error().decode()


def _check(rc):
    if rc != CCSP_OK:
        raise CcspError(rc, last_error())
    return rc


def load_triangulation(desc: TriangulationDesc, stream: int = 0) -> int:
    h = _P()
    _check(_lib.load_triangulation(ctypes.byref(desc), _P(stream), ctypes.byref(h)))
    return h.value


def trace_rays(tri: int, o_xy: int, d_xy: int, start_tri: int, n: int, precision: int,
               hit_prim: int, hit_t: int, steps: int, stream: int = 0) -> None:
    _check(_lib.trace_rays(_P(tri), _P(o_xy), _P(d_xy), _P(start_tri), n, precision, _P(hit_prim),
                           _P(hit_t), _P(steps), _P(stream)))


def trace_rays_tuned(tri: int, o_xy: int, d_xy: int, start_tri: int, n: int, precision: int,
                     hit_prim: int, hit_t: int, steps: int, tune: TuneParams | None,
                     stream: int = 0) -> None:
    _check(_lib.trace_rays_tuned(_P(tri), _P(o_xy), _P(d_xy), _P(start_tri), n, precision,
                                 _P(hit_prim), _P(hit_t), _P(steps),
                                 ctypes.byref(tune) if tune is not None else None, _P(stream)))


def mesh_subdivide(desc, xy: int, sizes: int, xy_out: int = 0, tri_out: int = 0,
                   kind_out: int = 0, line_out: int = 0) -> None:
    """sizes: address of two int64 (vertices, triangles)."""
    _check(_lib.mesh_subdivide(ctypes.byref(desc), _P(xy), _P(sizes), _P(sizes + 8), _P(xy_out),
                               _P(tri_out), _P(kind_out), _P(line_out)))


def trace_rays_static(tri: int, o_xy: int, d_xy: int, start_tri: int, n: int, precision: int,
                      hit_prim: int, hit_t: int, steps: int, tune: TuneParams | None,
                      stream: int = 0) -> None:
    _check(_lib.trace_rays_static(_P(tri), _P(o_xy), _P(d_xy), _P(start_tri), n, precision,
                                  _P(hit_prim), _P(hit_t), _P(steps),
                                  ctypes.byref(tune) if tune is not None else None, _P(stream)))


CCSP_STATIC_MAX_RAYS = 1 << 20


def trace_batch(items, precision: int, tune: TuneParams | None = None, stream: int = 0) -> None:
    arr = (TraceItem * len(items))(*items)
    _check(_lib.trace_batch(arr, len(items), precision,
                            ctypes.byref(tune) if tune is not None else None, _P(stream)))


def free_triangulation(tri: int) -> None:
    _lib.free_triangulation(_P(tri))


def read_counters(reset: bool = False) -> list:
    out = (ctypes.c_uint64 * 4)()
    _check(_lib.read_counters(ctypes.byref(out), int(reset)))
    return list(out)


def read_stage_times(max_records: int = 256) -> tuple:
    """(bin_ms, walk_ms, finish_ms) lists of the most recent CCSP_TRACE_TIMED traces, oldest
    first."""
    b = (ctypes.c_float * max(1, max_records))()
    w = (ctypes.c_float * max(1, max_records))()
    f = (ctypes.c_float * max(1, max_records))()
    n = ctypes.c_int32()
    _check(_lib.read_stage_times(max_records, b, w, f, ctypes.byref(n)))
    return list(b[:n.value]), list(w[:n.value]), list(f[:n.value])


def autotune(items, precision: int, reps: int = 3, stream: int = 0) -> tuple:
    """(TuneParams, mean ms per call) chosen by measurement; see the header."""
    arr = (TraceItem * len(items))(*items)
    best = TuneParams()
    ms = ctypes.c_float()
    _check(_lib.autotune(arr, len(items), precision, reps, ctypes.byref(best), ctypes.byref(ms),
                         _P(stream)))
    return best, ms.value


def tune_cache_set(n_items: int, total_rays: int, total_triangles: int, precision: int,
                   tune: TuneParams) -> None:
    _check(_lib.tune_cache_set(n_items, total_rays, total_triangles, precision, ctypes.byref(tune)))


def tune_cache_get(n_items: int, total_rays: int, total_triangles: int, precision: int):
    """The cached TuneParams for this workload shape, or None."""
    out = TuneParams()
    rc = _lib.tune_cache_get(n_items, total_rays, total_triangles, precision, ctypes.byref(out))
    if rc < 0:
        _check(rc)
    return out if rc == 1 else None


def trace_bounces(tri: int, o_xy: int, d_xy: int, start_tri: int, n: int, max_bounces: int,
                  precision: int, hit_prim: int, hit_t: int, steps: int, bounces: int,
                  hit_face: int, tune: TuneParams | None = None, stream: int = 0) -> None:
    _check(_lib.trace_bounces(_P(tri), _P(o_xy), _P(d_xy), _P(start_tri), n, max_bounces,
                              precision, _P(hit_prim), _P(hit_t), _P(steps), _P(bounces),
                              _P(hit_face), ctypes.byref(tune) if tune is not None else None,
                              _P(stream)))


def locate_points(tri: int, q_xy: int, n: int, tri_out: int, status: int, stream: int = 0) -> None:
    _check(_lib.locate_points(_P(tri), _P(q_xy), n, _P(tri_out), _P(status), _P(stream)))


def mesh_load(desc: MeshDesc) -> int:
    h = _P()
    _check(_lib.mesh_load(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def mesh_info(mesh: int, edge_v: int = 0) -> int:
    n = ctypes.c_int64()
    _check(_lib.mesh_info(_P(mesh), ctypes.byref(n), _P(edge_v)))
    return n.value


def objective_eval(mesh: int, xy: int, params: ObjectiveParams, out: int, contractible: int = 0,
                   weight: int = 0, stream: int = 0) -> None:
    _check(_lib.objective_eval(_P(mesh), _P(xy), ctypes.byref(params), _P(out), _P(contractible),
                               _P(weight), _P(stream)))


def objective_delta(mesh: int, xy: int, params: ObjectiveParams, vid: int, q_xy: int, k: int,
                    delta: int, status: int, stream: int = 0) -> None:
    _check(_lib.objective_delta(_P(mesh), _P(xy), ctypes.byref(params), _P(vid), _P(q_xy), k,
                                _P(delta), _P(status), _P(stream)))


def mesh_classes(mesh: int, class_off: int = 0, class_v: int = 0) -> int:
    n = ctypes.c_int32()
    _check(_lib.mesh_classes(_P(mesh), ctypes.byref(n), _P(class_off), _P(class_v)))
    return n.value


def anneal_moves(mesh: int, xy: int, params: ObjectiveParams, temperature: float, vid: int,
                 disp: int, u: int, k: int, delta: int, status: int, stream: int = 0) -> None:
    _check(_lib.anneal_moves(_P(mesh), _P(xy), ctypes.byref(params), temperature, _P(vid), _P(disp),
                             _P(u), k, _P(delta), _P(status), _P(stream)))


def anneal_joint(mesh: int, xy: int, params: ObjectiveParams, temperature: float, lam: float,
                 vid: int, k: int, xi: int, u: float, stream: int = 0) -> tuple:
    """Returns (delta, status) of the joint move (host values)."""
    delta = ctypes.c_double()
    status = ctypes.c_int32()
    _check(_lib.anneal_joint(_P(mesh), _P(xy), ctypes.byref(params), temperature, lam, _P(vid), k,
                             _P(xi), u, ctypes.byref(delta), ctypes.byref(status), _P(stream)))
    return delta.value, status.value


def anneal_joint_groups(mesh: int, xy: int, params: ObjectiveParams, temperature: float,
                        lam: float, centres: int, n: int, draws: int, u: float,
                        stream: int = 0) -> tuple:
    """Returns (delta, status) of the joint group move (host values)."""
    delta = ctypes.c_double()
    status = ctypes.c_int32()
    _check(_lib.anneal_joint_groups(_P(mesh), _P(xy), ctypes.byref(params), temperature, lam,
                                    _P(centres), n, _P(draws), u, ctypes.byref(delta),
                                    ctypes.byref(status), _P(stream)))
    return delta.value, status.value


def anneal_sweep(mesh: int, xy: int, params: ObjectiveParams, temperature: float, disp: int,
                 u: int, delta: int, status: int, stream: int = 0) -> None:
    _check(_lib.anneal_sweep(_P(mesh), _P(xy), ctypes.byref(params), temperature, _P(disp), _P(u),
                             _P(delta), _P(status), _P(stream)))


def anneal_propose(mesh: int, xy: int, params: ObjectiveParams, temperature: float, kind: int,
                   draws: int, u: int, delta: int, status: int, stream: int = 0) -> None:
    _check(_lib.anneal_propose(_P(mesh), _P(xy), ctypes.byref(params), temperature, kind,
                               _P(draws), _P(u), _P(delta), _P(status), _P(stream)))


def anneal_schedule(mesh: int, xy: int, params: ObjectiveParams, n_sweeps: int, temperature: int,
                    eps: int, lambda0: float, target: float, xi: int, u: int, lambda_out: int,
                    accepted_out: int, stream: int = 0) -> None:
    _check(_lib.anneal_schedule(_P(mesh), _P(xy), ctypes.byref(params), n_sweeps, _P(temperature),
                                _P(eps), lambda0, target, _P(xi), _P(u), _P(lambda_out),
                                _P(accepted_out), _P(stream)))


def flip_anneal(n_vertices: int, xy: int, n_triangles: int, tri_v: int, tri_nbr: int,
                tri_prim: int, vertex_line: int, n_prims: int, prim_v: int, n_rounds: int,
                temperature: int, seed: int, flips_out: int, stream: int = 0) -> None:
    _check(_lib.flip_anneal(n_vertices, _P(xy), n_triangles, _P(tri_v), _P(tri_nbr), _P(tri_prim),
                            _P(vertex_line), n_prims, _P(prim_v), n_rounds, _P(temperature),
                            seed & ((1 << 64) - 1), _P(flips_out), _P(stream)))


def mesh_contract(desc: MeshDesc, xy: int, eps: float, tri_out: int, n_triangles_out: int,
                  kind_out: int, line_out: int, xy_out: int, n_vertices_out: int,
                  old_to_new: int, n_contracted: int) -> None:
    _check(_lib.mesh_contract(ctypes.byref(desc), _P(xy), eps, _P(tri_out), _P(n_triangles_out),
                              _P(kind_out), _P(line_out), _P(xy_out), _P(n_vertices_out),
                              _P(old_to_new), _P(n_contracted)))


def anneal_group(mesh: int, xy: int, params: ObjectiveParams, temperature: float, lam: float,
                 centres: int, n: int, draws: int, u: int, delta: int, status: int, members: int,
                 rounds: int, stream: int = 0) -> None:
    _check(_lib.anneal_group(_P(mesh), _P(xy), ctypes.byref(params), temperature, lam,
                             _P(centres), n, _P(draws), _P(u), _P(delta), _P(status), _P(members),
                             _P(rounds), _P(stream)))


def mesh_free(mesh: int) -> None:
    _lib.mesh_free(_P(mesh))


def server_create(cfg: ServerConfig | None) -> int:
    h = _P()
    _check(_lib.server_create(ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(h)))
    return h.value


def server_submit(server: int, scene: int, o_xy: int, d_xy: int, start_tri: int, n: int,
                  hit_prim: int, hit_t: int, steps: int) -> int:
    rid = ctypes.c_uint64()
    _check(_lib.server_submit(_P(server), _P(scene), _P(o_xy), _P(d_xy), _P(start_tri), n,
                              _P(hit_prim), _P(hit_t), _P(steps), ctypes.byref(rid)))
    return rid.value


def server_poll(server: int, max_n: int = 1024, timeout_s: float = 0.0) -> list:
    """[(id, status, t_submit, t_done)] of completed requests."""
    ids = (ctypes.c_uint64 * max(1, max_n))()
    st = (ctypes.c_int32 * max(1, max_n))()
    ts = (ctypes.c_double * max(1, max_n))()
    td = (ctypes.c_double * max(1, max_n))()
    n = ctypes.c_int32()
    _check(_lib.server_poll(_P(server), max_n, ids, st, ts, td, ctypes.byref(n), timeout_s))
    return [(ids[k], st[k], ts[k], td[k]) for k in range(n.value)]


def server_stats(server: int) -> list:
    out = (ctypes.c_int64 * 8)()
    _check(_lib.server_stats(_P(server), ctypes.byref(out)))
    return list(out)


def server_destroy(server: int) -> None:
    _lib.server_destroy(_P(server))


def triangulation_info(tri: int) -> list:
    out = (ctypes.c_int64 * 4)()
    _check(_lib.triangulation_info(_P(tri), ctypes.byref(out)))
    return list(out)


def reserve_workspace(max_rays: int) -> None:
    _check(_lib.reserve_workspace(max_rays))


def gather_roofline(working_set_bytes: int, waves_per_cu: int = 16, steps_per_lane: int = 4096,
                    stream: int = 0) -> float:
    out = ctypes.c_double()
    _check(_lib.gather_roofline(working_set_bytes, waves_per_cu, steps_per_lane, ctypes.byref(out),
                                _P(stream)))
    return out.value


def raw_call(name: str, *args):
    """Direct access to an exported symbol (for tests of argument handling)."""
    return getattr(_lib, name)(*args)


def load_tetmesh(desc: TetMeshDesc) -> int:
    h = _P()
    _check(_lib.load_tetmesh(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def free_tetmesh(mesh: int) -> None:
    _check(_lib.free_tetmesh(_P(mesh)))


def tetmesh_info(mesh: int) -> tuple:
    nt, nb = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.tetmesh_info(_P(mesh), ctypes.byref(nt), ctypes.byref(nb)))
    return nt.value, nb.value


def trace_rays3d(mesh: int, o: int, d: int, start: int, n: int, flags: int, step_limit: int,
                 tune: Tune3d | None, hit_prim: int, hit_t: int, steps: int,
                 stream: int = 0) -> None:
    _check(_lib.trace_rays3d(_P(mesh), _P(o), _P(d), _P(start), n, flags, step_limit,
                             ctypes.byref(tune) if tune is not None else None, _P(hit_prim),
                             _P(hit_t), _P(steps), _P(stream)))


def trace3d_stage_times() -> tuple:
    b, w = ctypes.c_float(), ctypes.c_float()
    _check(_lib.trace3d_stage_times(ctypes.byref(b), ctypes.byref(w)))
    return b.value, w.value
