"""The 3D walk's C ABI on the CPU: load_tetmesh rejects malformed tetrahedralisations in host
code before any device call, and trace_rays3d rejects bad arguments."""
import ctypes

import numpy as np
import pytest

import scenegen as sg
from paper_2112_05570_amd import binding as B


@pytest.fixture(scope="module")
def tets():
    return sg.make_tet_scene(600, seed=2)


def _code(xyz, tv, tn, tp, pr):
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (xyz, tv, tn, tp, pr)]
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    desc = B.TetMeshDesc(arrs[0].shape[0], p(arrs[0]), arrs[1].shape[0], p(arrs[1]), p(arrs[2]),
                         p(arrs[3]), arrs[4].shape[0], p(arrs[4]))
    h = ctypes.c_void_p()
    rc = B.raw_call("load_tetmesh", ctypes.byref(desc), ctypes.byref(h))
    return rc, B.last_error()


@pytest.mark.parametrize("what,needle", [
    ("negative", "not positively oriented"),
    ("grid", "off the grid"),
    ("vid", "vertex id out of range"),
    ("nbr_range", "out of range"),
    ("nbr_back", "does not share it back"),
    ("prim_range", "primitive id"),
    ("prim_side", "different primitives"),
    ("prim_verts", "primitive"),
])
def test_load_rejects_malformed(tets, what, needle):
    sc = tets
    xyz, tv, tn, tp, pr = (a.copy() for a in (sc.xyz, sc.tet_v, sc.tet_nbr, sc.tet_prim, sc.prims))
    t = int(np.nonzero((tn >= 0).all(1))[0][0])
    if what == "negative":
        tv[t, [0, 1]] = tv[t, [1, 0]]
    elif what == "grid":
        xyz[5, 2] = 1 << 19
    elif what == "vid":
        tv[t, 2] = xyz.shape[0]
    elif what == "nbr_range":
        tn[t, 1] = tv.shape[0] + 7
    elif what == "nbr_back":
        tn[t, 1] = tn[t, 2]
    elif what == "prim_range":
        tp[t, 0] = pr.shape[0]
    elif what == "prim_side":
        tt, i = np.argwhere((tp >= 0) & (tn >= 0))[0]
        tp[tt, i] = -1
    elif what == "prim_verts":
        k = int(tp[tp >= 0][0])
        pr[k, 0] = (pr[k, 0] + 1) % xyz.shape[0]
    rc, msg = _code(xyz, tv, tn, tp, pr)
    assert rc == B.CCSP_E_BAD_TRIANGULATION, (rc, msg)
    assert needle in msg, msg


def test_load_rejects_sizes(tets):
    sc = tets
    rc, msg = _code(sc.xyz[:3], sc.tet_v, sc.tet_nbr, sc.tet_prim, sc.prims)
    assert rc == B.CCSP_E_ARG and "n_vertices" in msg
    h = ctypes.c_void_p()
    assert B.raw_call("load_tetmesh", None, ctypes.byref(h)) == B.CCSP_E_ARG


def test_trace3d_argument_errors():
    lib_call = B.raw_call
    out = np.zeros(4, np.int64)
    p = out.ctypes.data
    assert lib_call("trace_rays3d", None, p, p, p, 1, 0, 0, None, p, p, p, None) == B.CCSP_E_ARG
    assert "null mesh" in B.last_error()
    assert lib_call("tetmesh_info", None, None, None) == B.CCSP_E_ARG
    assert lib_call("free_tetmesh", None) == B.CCSP_OK
