"""Checker for the triangulation ray walk: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. The walk library never does and shares no code with it.

``liboracle.so`` (``oracle.c``) holds a plain C implementation of what the walk computes (paper
Sec. 5.1 for the walk, Sec. 5.4 for the step count), every sign decided with exact integer
arithmetic. This module is ctypes marshalling only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (C11, no floating-point contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "oracle.c"),
           os.path.join(_HERE, "oracle3d.c"), "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Tri(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("xy", ctypes.c_void_p), ("nt", ctypes.c_int64),
                ("tri_v", ctypes.c_void_p), ("tri_nbr", ctypes.c_void_p),
                ("tri_prim", ctypes.c_void_p), ("np", ctypes.c_int64), ("prim", ctypes.c_void_p)]


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        for name in ("oracle_side_sign", "oracle_orient"):
            getattr(lib, name).argtypes = [P, P, P]
            getattr(lib, name).restype = I
        lib.oracle_incircle.argtypes = [P, P, P, P]
        lib.oracle_incircle.restype = I
        lib.oracle_t.argtypes = [P, P, P]
        lib.oracle_t.restype = ctypes.c_double
        lib.oracle_walk.argtypes = [P, I64, P, P, P, I64, P, P, P, I]
        lib.oracle_brute_edges.argtypes = [P, I64, P, P, P, P, P, I]
        lib.oracle_brute_prims.argtypes = [I64, P, I64, P, P, P, P, I]
        lib.oracle_validate.argtypes = [P, I, ctypes.c_char_p, I]
        lib.oracle_locate.argtypes = [P, I64, P, P, P, I]
        lib.oracle_bounce.argtypes = [P, I64, P, P, P, ctypes.c_int32, I64, P, P, P, P, P, I]
        lib.oracle_num_threads.restype = I
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Triangulation:
    """Keeps contiguous copies of the arrays alive for the C structure."""

    def __init__(self, xy, tri_v, tri_nbr, tri_prim, prims):
        self.xy = _c(xy, np.float64).reshape(-1, 2)
        self.tri_v = _c(tri_v, np.int32).reshape(-1, 3)
        self.tri_nbr = _c(tri_nbr, np.int32).reshape(-1, 3)
        self.tri_prim = _c(tri_prim, np.int32).reshape(-1, 3)
        self.prims = _c(prims, np.float64).reshape(-1, 4)
        self.c = _Tri(self.xy.shape[0], _p(self.xy), self.tri_v.shape[0], _p(self.tri_v),
                      _p(self.tri_nbr), _p(self.tri_prim), self.prims.shape[0], _p(self.prims))

    @classmethod
    def of(cls, scene):
        return cls(scene.xy, scene.tri_v, scene.tri_nbr, scene.tri_prim, scene.prims)


def side_sign(o, d, v) -> int:
    o, d, v = (_c(x, np.float64) for x in (o, d, v))
    return _L().oracle_side_sign(_p(o), _p(d), _p(v))


def orient(a, b, c) -> int:
    a, b, c = (_c(x, np.float64) for x in (a, b, c))
    return _L().oracle_orient(_p(a), _p(b), _p(c))


def incircle(a, b, c, d) -> int:
    a, b, c, d = (_c(x, np.float64) for x in (a, b, c, d))
    return _L().oracle_incircle(_p(a), _p(b), _p(c), _p(d))


def t_formula(o, d, seg) -> float:
    o, d, seg = (_c(x, np.float64) for x in (o, d, seg))
    return _L().oracle_t(_p(o), _p(d), _p(seg))


def _outs(n):
    return np.empty(n, np.int32), np.empty(n, np.float64), np.empty(n, np.int32)


def walk(tri: Triangulation, o, d, start, threads: int = 0, max_steps: int = 0):
    """The walk of Sec. 5.1 ray by ray. Returns (prim, t, steps). A ray whose walk would enter
    more than max_steps triangles ends with -2 and steps = max_steps (0: the triangle count)."""
    o, d, start = _c(o, np.float64), _c(d, np.float64), _c(start, np.int32)
    n = start.shape[0]
    prim, t, steps = _outs(n)
    _L().oracle_walk(ctypes.byref(tri.c), n, _p(o), _p(d), _p(start), int(max_steps), _p(prim),
                     _p(t), _p(steps), int(threads))
    return prim, t, steps


def brute_edges(tri: Triangulation, o, d, threads: int = 0):
    """First terminating edge and crossing count by brute force. Returns (prim, t, steps, status);
    status bit 0: an origin lies on an edge, bit 1: some ray found no terminating edge."""
    o, d = _c(o, np.float64), _c(d, np.float64)
    n = o.reshape(-1, 2).shape[0]
    prim, t, steps = _outs(n)
    st = _L().oracle_brute_edges(ctypes.byref(tri.c), n, _p(o), _p(d), _p(prim), _p(t), _p(steps),
                                 int(threads))
    return prim, t, steps, st


def brute_prims(prims, o, d, threads: int = 0):
    """First primitive crossed, by brute force over all primitives. Returns (prim, t, status)."""
    prims, o, d = _c(prims, np.float64), _c(o, np.float64), _c(d, np.float64)
    n = o.reshape(-1, 2).shape[0]
    prim, t, _ = _outs(n)
    st = _L().oracle_brute_prims(prims.reshape(-1, 4).shape[0], _p(prims), n, _p(o), _p(d),
                                 _p(prim), _p(t), int(threads))
    return prim, t, st


def bounce(tri: Triangulation, o, d, start, max_bounces: int, threads: int = 0,
           max_steps: int = 0):
    """The walk continued by specular reflections (Sec. 5.2's secondary rays). Returns
    (prim, t, steps, hits, face) per ray; see oracle.c. max_steps limits each segment as in
    walk()."""
    o, d, start = _c(o, np.float64), _c(d, np.float64), _c(start, np.int32)
    n = start.shape[0]
    prim, t, steps = _outs(n)
    hits = np.empty(n, np.int32)
    face = np.empty(n, np.int32)
    _L().oracle_bounce(ctypes.byref(tri.c), n, _p(o), _p(d), _p(start), int(max_bounces),
                       int(max_steps), _p(prim), _p(t), _p(steps), _p(hits), _p(face),
                       int(threads))
    return prim, t, steps, hits, face


def locate(tri: Triangulation, q, threads: int = 0):
    """Brute-force point location (Sec. 5.2). Returns (triangle, status) per point: status 0
    strictly inside, 1 on an edge or vertex (the first such triangle), -1 outside, -2 not
    finite."""
    q = _c(q, np.float64).reshape(-1, 2)
    n = q.shape[0]
    tr = np.empty(n, np.int32)
    st = np.empty(n, np.int32)
    _L().oracle_locate(ctypes.byref(tri.c), n, _p(q), _p(tr), _p(st), int(threads))
    return tr, st


def validate(tri: Triangulation, delaunay: bool = False) -> str:
    """'' if the triangulation passes every check, else the first failure."""
    buf = ctypes.create_string_buffer(256)
    r = _L().oracle_validate(ctypes.byref(tri.c), int(delaunay), buf, 256)
    return "" if r == 0 else buf.value.decode()


def num_threads() -> int:
    return int(_L().oracle_num_threads())


# ---------------------------------------------------------------- the 3D walk (oracle3d.c)

class _Tet(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("nt", ctypes.c_int64),
                ("tet_v", ctypes.c_void_p), ("tet_nbr", ctypes.c_void_p),
                ("tet_prim", ctypes.c_void_p), ("np", ctypes.c_int64), ("prims", ctypes.c_void_p)]


def _L3():
    lib = _L()
    if not getattr(lib, "_tet_ready", False):
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle3_orient.argtypes = [P, P, P, P]
        lib.oracle3_orient.restype = I64
        lib.oracle3_plucker.argtypes = [P, P, P, P]
        lib.oracle3_plucker.restype = I64
        lib.oracle3_pi.argtypes = [P, P, P, P, P]
        lib.oracle3_pi.restype = I
        lib.oracle3_walk.argtypes = [P, I64, P, P, P, I64, P, P, P, P, I]
        lib.oracle3_brute.argtypes = [P, I64, P, P, P, P, P, P, I]
        lib.oracle3_validate.argtypes = [P, ctypes.c_char_p, I]
        lib.oracle3_locate.argtypes = [P, I64, P, P, P, I]
        lib._tet_ready = True
    return lib


class TetMesh:
    """A tetrahedralisation for the 3D checker (contiguous copies kept alive for C)."""

    def __init__(self, xyz, tet_v, tet_nbr, tet_prim, prims):
        self.xyz = _c(xyz, np.int32).reshape(-1, 3)
        self.tet_v = _c(tet_v, np.int32).reshape(-1, 4)
        self.tet_nbr = _c(tet_nbr, np.int32).reshape(-1, 4)
        self.tet_prim = _c(tet_prim, np.int32).reshape(-1, 4)
        self.prims = _c(prims, np.int32).reshape(-1, 3)
        self.c = _Tet(self.xyz.shape[0], _p(self.xyz), self.tet_v.shape[0], _p(self.tet_v),
                      _p(self.tet_nbr), _p(self.tet_prim), self.prims.shape[0], _p(self.prims))

    @classmethod
    def of(cls, scene):
        return cls(scene.xyz, scene.tet_v, scene.tet_nbr, scene.tet_prim, scene.prims)


def orient3(a, b, c, d) -> int:
    """det[b - a; c - a; d - a] for integer grid points, exact."""
    a, b, c, d = (_c(x, np.int32) for x in (a, b, c, d))
    return int(_L3().oracle3_orient(_p(a), _p(b), _p(c), _p(d)))


def plucker3(o, d, p, q) -> int:
    """d . ((p - o) x (q - o)), exact."""
    o, d, p, q = (_c(x, np.int32) for x in (o, d, p, q))
    return int(_L3().oracle3_plucker(_p(o), _p(d), _p(p), _p(q)))


def pi3(o, d, p, q):
    """The walk's sign for the directed edge (p, q) after the symbolic move of the line; returns
    (sign, degenerate)."""
    o, d, p, q = (_c(x, np.int32) for x in (o, d, p, q))
    dg = ctypes.c_int(0)
    s = _L3().oracle3_pi(_p(o), _p(d), _p(p), _p(q), ctypes.byref(dg))
    return int(s), bool(dg.value)


def _outs3(n):
    return np.empty(n, np.int32), np.empty(n, np.float64), np.empty(n, np.int32), np.empty(n, np.int32)


def walk3(mesh: TetMesh, o, d, start, threads: int = 0, max_steps: int = 0):
    """The 3D walk ray by ray. Returns (prim, t, steps, degenerate): prim >= 0 the primitive hit,
    -1 out through a hull face that is not a primitive, -2 stopped at max_steps tetrahedra
    (0: the tetrahedron count), -3 invalid ray (zero direction, start out of range or the origin
    not strictly inside it)."""
    o, d, start = _c(o, np.int32).reshape(-1, 3), _c(d, np.int32).reshape(-1, 3), _c(start, np.int32)
    n = start.shape[0]
    prim, t, steps, dg = _outs3(n)
    _L3().oracle3_walk(ctypes.byref(mesh.c), n, _p(o), _p(d), _p(start), int(max_steps), _p(prim),
                       _p(t), _p(steps), _p(dg), int(threads))
    return prim, t, steps, dg


def brute3(mesh: TetMesh, o, d, threads: int = 0):
    """First primitive and crossing count by brute force over every face. Returns
    (prim, t, steps, ambiguous): bit 0 of ambiguous marks a hit, bit 1 a count, that depends on how
    ties are broken."""
    o, d = _c(o, np.int32).reshape(-1, 3), _c(d, np.int32).reshape(-1, 3)
    n = o.shape[0]
    prim, t, steps, dg = _outs3(n)
    st = _L3().oracle3_brute(ctypes.byref(mesh.c), n, _p(o), _p(d), _p(prim), _p(t), _p(steps),
                             _p(dg), int(threads))
    if st != 0:
        raise MemoryError("oracle3_brute")
    return prim, t, steps, dg


def locate3(mesh: TetMesh, q, threads: int = 0):
    """Brute-force point location. Returns (tet, status): 0 strictly inside, 1 on the boundary of
    the first tetrahedron holding the point, -1 in none."""
    q = _c(q, np.int32).reshape(-1, 3)
    n = q.shape[0]
    tt = np.empty(n, np.int32)
    st = np.empty(n, np.int32)
    _L3().oracle3_locate(ctypes.byref(mesh.c), n, _p(q), _p(tt), _p(st), int(threads))
    return tt, st


def validate3(mesh: TetMesh) -> str:
    """'' if the tetrahedralisation passes every check, else the first failure."""
    buf = ctypes.create_string_buffer(256)
    r = _L3().oracle3_validate(ctypes.byref(mesh.c), buf, 256)
    return "" if r == 0 else buf.value.decode()
