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
                      CCSP_TRACE_FP32_FILTERED, CCSP_TRACE_FP64, CCSP_TRACE_INPUT_ORDER,
                      CCSP_TRACE_TIMED, CCSP_TRACE_VALIDATE, CcspError, TuneParams,
                      read_stage_times, reserve_workspace)

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


def trace_batch(jobs, precision="fp32", tune: TuneParams | None = None, stream=None,
                graph=False, count=False, timed=False):
    """jobs: list of (Scene, o, d, start[, Result]). Returns the list of Results."""
    items, results = [], []
    for job in jobs:
        scene, o, d, start = job[:4]
        n = _check_rays(o, d, start)
        res = _outputs(n, o.device, job[4] if len(job) > 4 else None)
        results.append(res)
        items.append(B.TraceItem(scene.handle, o.data_ptr(), d.data_ptr(), start.data_ptr(), n,
                                 res.hit_prim.data_ptr(), res.hit_t.data_ptr(),
                                 res.steps.data_ptr()))
    if graph:
        tune = tune or TuneParams()
        tune = TuneParams(tune.wg_size, tune.tile_rays, tune.waves_per_cu, tune.refill_min,
                          (ctypes.c_int32 * 4)(1, 0, 0, 0))
    B.trace_batch(items, _mode(precision) | (CCSP_TRACE_COUNT if count else 0)
                  | (CCSP_TRACE_TIMED if timed else 0), tune, _stream(stream))
    return results


def read_counters(reset=False):
    """(steps, binary32 deferrals, binary64 deferrals, rays) since the last reset."""
    return B.read_counters(reset)
