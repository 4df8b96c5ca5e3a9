"""The C ABI library on the CPU: it loads, exports every declared symbol, and rejects bad
arguments and malformed triangulations in host code before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2112_05570_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    declared = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        hdr = open(os.path.join(ROOT, "include", h)).read()
        declared |= set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(\w+)\(", hdr, re.M))
    assert declared == set(B.EXPORTS), declared ^ set(B.EXPORTS)
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(sc, **over):
    arrs = dict(xy=np.ascontiguousarray(sc.xy), tri_v=sc.tri_v.copy(), tri_nbr=sc.tri_nbr.copy(),
                tri_prim=sc.tri_prim.copy(), prims=np.ascontiguousarray(sc.prims))
    arrs.update(over)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    d = B.TriangulationDesc(arrs["xy"].shape[0], p(arrs["xy"]), arrs["tri_v"].shape[0],
                            p(arrs["tri_v"]), p(arrs["tri_nbr"]), p(arrs["tri_prim"]),
                            arrs["prims"].shape[0], p(arrs["prims"]))
    return d, arrs


def _load_code(desc):
    h = ctypes.c_void_p()
    return B.raw_call("load_triangulation", ctypes.byref(desc), None, ctypes.byref(h))


@pytest.mark.parametrize("what,needle", [
    ("cw", "counter-clockwise"),
    ("nbr_range", "neighbour out of range"),
    ("asym", "symmetric|does not match"),
    ("prim_mismatch", "primitive differs"),
    ("prim_range", "primitive id out of range"),
    ("not_collinear", "collinear"),
    ("nan", "not finite"),
    ("euler", "Euler"),
    ("vid", "vertex id"),
])
def test_load_rejects_malformed(tiny_scene, what, needle):
    sc = tiny_scene
    tv, tn, tp, xy = sc.tri_v.copy(), sc.tri_nbr.copy(), sc.tri_prim.copy(), sc.xy.copy()
    t = int(np.nonzero((tn >= 0).all(1) & (tp < 0).all(1))[0][0])
    if what == "cw":
        tv[t, [1, 2]] = tv[t, [2, 1]]
    elif what == "nbr_range":
        tn[t, 0] = 10**6
    elif what == "asym":
        tn[t, 0] = tn[t, 1]
    elif what == "prim_mismatch":
        # drop the constraint on one side of an interior constrained edge
        tc, ic = map(int, np.argwhere((tp >= 0) & (tn >= 0))[0])
        tp[tc, ic] = -1
    elif what == "prim_range":
        tp[t, 0] = 10**6
    elif what == "not_collinear":
        # mark an interior edge as constrained on both sides, but with a primitive it is not on
        n = tn[t, 0]
        back = int(np.nonzero(tn[n] == t)[0][0])
        tp[t, 0] = 0
        tp[n, back] = 0
    elif what == "nan":
        xy[7, 0] = np.nan
    elif what == "euler":
        n = tn[t, 0]
        back = int(np.nonzero(tn[n] == t)[0][0])
        tn[t, 0] = -1
        tn[n, back] = -1
    elif what == "vid":
        tv[t, 0] = -5
    desc, keep = _desc(sc, tri_v=tv, tri_nbr=tn, tri_prim=tp, xy=xy)
    rc = _load_code(desc)
    assert rc in (B.CCSP_E_BAD_TRIANGULATION, B.CCSP_E_ARG), rc
    assert re.search(needle, B.last_error()), B.last_error()


def test_load_rejects_sizes():
    d = B.TriangulationDesc(2, None, 1, None, None, None, 0, None)
    assert _load_code(d) == B.CCSP_E_ARG
    d = B.TriangulationDesc(10, None, 1 << 29, None, None, None, 0, None)
    assert _load_code(d) == B.CCSP_E_ARG
    assert B.raw_call("load_triangulation", None, None, None) == B.CCSP_E_ARG


def test_trace_argument_errors():
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: argument checks come first
    z = ctypes.c_void_p(0)
    al = ctypes.c_void_p(0x10000)
    # null scene
    assert B.raw_call("trace_rays", z, al, al, al, ctypes.c_int64(5), 1, al, al, al, z) == B.CCSP_E_ARG
    # unknown mode and flags
    assert B.raw_call("trace_rays", fake, al, al, al, ctypes.c_int64(5), 7, al, al, al, z) == B.CCSP_E_ARG
    assert B.raw_call("trace_rays", fake, al, al, al, ctypes.c_int64(5), 1 | (1 << 12), al, al, al, z) == B.CCSP_E_ARG
    # negative count, null and misaligned buffers
    assert B.raw_call("trace_rays", fake, al, al, al, ctypes.c_int64(-1), 1, al, al, al, z) == B.CCSP_E_ARG
    assert B.raw_call("trace_rays", fake, z, al, al, ctypes.c_int64(5), 1, al, al, al, z) == B.CCSP_E_ARG
    mis = ctypes.c_void_p(0x10008)
    assert B.raw_call("trace_rays", fake, mis, al, al, ctypes.c_int64(5), 1, al, al, al, z) == B.CCSP_E_ARG
    assert "aligned" in B.last_error()
    # an empty trace is a no-op
    assert B.raw_call("trace_rays", fake, z, z, z, ctypes.c_int64(0), 1, z, z, z, z) == B.CCSP_OK


def test_trace_batch_argument_errors():
    assert B.raw_call("trace_batch", None, 3, 1, None, None) == B.CCSP_E_ARG
    assert B.raw_call("trace_batch", None, -1, 1, None, None) == B.CCSP_E_ARG
    item = B.TraceItem(None, 0x10000, 0x10000, 0x10000, 4, 0x10000, 0x10000, 0x10000)
    arr = (B.TraceItem * 1)(item)
    assert B.raw_call("trace_batch", arr, 1, 1, None, None) in (B.CCSP_E_ARG, B.CCSP_E_HIP)
    assert B.raw_call("trace_batch", arr, 1, 1 | B.CCSP_TRACE_VALIDATE, None, None) == B.CCSP_E_ARG


def test_read_stage_times_argument_errors():
    n = ctypes.c_int32(7)
    assert B.raw_call("read_stage_times", 4, None, None, None, None) == B.CCSP_E_ARG
    assert B.raw_call("read_stage_times", -1, None, None, None, ctypes.byref(n)) == B.CCSP_E_ARG
    assert n.value == 0
    assert B.raw_call("read_stage_times", 4, None, None, None, ctypes.byref(n)) == B.CCSP_E_ARG
    assert "null" in B.last_error()


def test_server_argument_errors():
    out = ctypes.c_void_p()
    bad = [B.ServerConfig(17, 0, 0, 0, 1, 0), B.ServerConfig(0, 5000, 0, 0, 1, 0),
           B.ServerConfig(0, 0, 0, 1000, 1, 0), B.ServerConfig(0, 0, 0, 0, 7, 0),
           B.ServerConfig(0, 0, 0, 0, 1 | (1 << 9), 0), B.ServerConfig(0, 0, -1, 0, 1, 0)]
    for cfg in bad:  # rejected before any device call
        assert B.raw_call("server_create", ctypes.byref(cfg), ctypes.byref(out)) == B.CCSP_E_ARG
    assert B.raw_call("server_create", None, None) == B.CCSP_E_ARG
    rid = ctypes.c_uint64()
    z = ctypes.c_void_p(0)
    assert B.raw_call("server_submit", z, z, z, z, z, ctypes.c_int64(1), z, z, z,
                      ctypes.byref(rid)) == B.CCSP_E_ARG
    n = ctypes.c_int32()
    assert B.raw_call("server_poll", z, 0, None, None, None, None, ctypes.byref(n),
                      ctypes.c_double(0)) == B.CCSP_E_ARG
    B.raw_call("server_destroy", z)  # no-op


def test_trace_bounces_argument_errors():
    fake = ctypes.c_void_p(0x1000)
    al = ctypes.c_void_p(0x10000)
    z = ctypes.c_void_p(0)
    n = ctypes.c_int64(5)
    assert B.raw_call("trace_bounces", fake, al, al, al, n, -1, 1, al, al, al, al, z, None, z) == B.CCSP_E_ARG
    assert B.raw_call("trace_bounces", fake, al, al, al, n, 2, 1 | B.CCSP_TRACE_VALIDATE, al, al, al, al, z, None, z) == B.CCSP_E_ARG
    assert B.raw_call("trace_bounces", fake, al, al, al, n, 2, 1, al, al, al, z, z, None, z) == B.CCSP_E_ARG
    assert B.raw_call("trace_bounces", z, al, al, al, n, 2, 1, al, al, al, al, z, None, z) == B.CCSP_E_ARG


def _mesh_desc(tri_v, kind, line, prim_v):
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (tri_v, kind, line, prim_v)]
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    d = B.MeshDesc(arrs[1].shape[0], p(arrs[1]), p(arrs[2]), arrs[0].shape[0], p(arrs[0]),
                   arrs[3].shape[0], p(arrs[3]))
    return d, arrs


@pytest.mark.parametrize("case,msg", [
    ("kind", "unknown vertex kind"),
    ("line", "names no original edge"),
    ("repeat", "repeats a vertex"),
    ("range", "out of range"),
    ("three", "more than two triangles"),
    ("orient", "the same way"),
    ("prim", "original edge end out of range"),
])
def test_mesh_load_rejects(case, msg):
    """Malformed movable meshes are rejected before any device work."""
    tri = [[0, 1, 2], [0, 2, 3]]
    kind, line, prim = [0, 2, 2, 1], [-1, -1, -1, 0], [[0, 1]]
    if case == "kind":
        kind = [0, 2, 5, 1]
    elif case == "line":
        line = [-1, -1, -1, 3]
    elif case == "repeat":
        tri = [[0, 1, 1], [0, 2, 3]]
    elif case == "range":
        tri = [[0, 1, 2], [0, 2, 4]]
    elif case == "three":
        tri = [[0, 1, 2], [0, 2, 3], [0, 4, 2]]
        kind, line = kind + [2], line + [-1]
    elif case == "orient":
        tri = [[0, 1, 2], [0, 3, 2]]
    elif case == "prim":
        prim = [[0, 7]]
    d, keep = _mesh_desc(tri, kind, line, prim)
    with pytest.raises(B.CcspError, match=msg):
        B.mesh_load(d)


def test_objective_calls_reject_null_arguments():
    p = B.ObjectiveParams(0.1, 1e-4, 1e-10, 1.0, 10.0, 0, 0)
    with pytest.raises(B.CcspError, match="null argument"):
        B.objective_eval(0, 0, p, 0)
    with pytest.raises(B.CcspError, match="null argument"):
        B.objective_delta(0, 0, p, 0, 0, 1, 0, 0)
    with pytest.raises(B.CcspError, match="null argument"):
        B.mesh_info(0)


def test_flip_anneal_rejects_before_any_device_call():
    """Argument errors are found on the host; zero rounds return at once (no device call)."""
    xy = np.zeros((4, 2), np.float64)
    tri = np.zeros((2, 3), np.int32)
    temps = np.array([1.0, -0.5])
    cnt = np.zeros(2, np.int64)
    p = lambda a: a.ctypes.data
    with pytest.raises(B.CcspError, match="null argument"):
        B.flip_anneal(4, 0, 2, p(tri), p(tri), p(tri), 0, 0, 0, 2, p(temps), 0, p(cnt))
    with pytest.raises(B.CcspError, match="null argument"):
        B.flip_anneal(4, p(xy), 2, p(tri), p(tri), p(tri), 0, 0, 0, 2, 0, 0, p(cnt))
    with pytest.raises(B.CcspError, match="temperatures"):
        B.flip_anneal(4, p(xy), 2, p(tri), p(tri), p(tri), 0, 0, 0, 2, p(temps), 0, p(cnt))
    with pytest.raises(B.CcspError, match="misaligned"):
        B.flip_anneal(4, p(xy) + 8, 2, p(tri), p(tri), p(tri), 0, 0, 0, 1, p(temps), 0, p(cnt))
    with pytest.raises(B.CcspError, match="too large"):
        B.flip_anneal(4, p(xy), 1 << 29, p(tri), p(tri), p(tri), 0, 0, 0, 1, p(temps), 0, p(cnt))
    with pytest.raises(B.CcspError, match="original edges' ends"):
        B.flip_anneal(4, p(xy), 2, p(tri), p(tri), p(tri), p(tri), 0, 0, 1, p(temps), 0, p(cnt))
    B.flip_anneal(4, p(xy), 2, p(tri), p(tri), p(tri), 0, 0, 0, 0, 0, 0, 0)
