"""The subdivision of Sec. 3.5.2 (CPU): the checker's (oracle/subdivide.py) pinned by the paper's
figure and by counts and lengths that the split fixes, and the library's host mesh_subdivide
equal to it bit for bit, once and on an already subdivided mesh (the second round of the
pipeline, Sec. 3.5.3)."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle.subdivide import CONSTRAINED, FREE, ORIGINAL, subdivide


def _weight(tri_v, xy):
    """Total length of the distinct edges."""
    edges = {tuple(sorted((int(t[i]), int(t[(i + 1) % 3])))) for t in tri_v for i in range(3)}
    return sum(math.dist(xy[a], xy[b]) for a, b in edges)


def test_one_triangle_as_in_the_figure():
    """One triangle becomes four: three at the corners with the midpoints of the two edges
    there, and the middle one of the three midpoints; with dyadic coordinates every area is a
    quarter of the parent's exactly. No original edge: every midpoint is FREE."""
    xy = np.array([[0.0, 0.0], [4.0, 0.0], [1.0, 2.0]])
    s = subdivide(xy, [[0, 1, 2]], [ORIGINAL] * 3, [-1] * 3, np.zeros((0, 2), dtype=np.int32))
    assert s.n_vertices == 6 and s.n_triangles == 4
    # edges in (lower, higher) order: (0,1) (0,2) (1,2) -> vertices 3, 4, 5
    assert np.array_equal(s.xy[3:], [[2.0, 0.0], [0.5, 1.0], [2.5, 1.0]])
    # m0 (opposite v0 = 0) is the midpoint of (1,2) = 5, m1 of (0,2) = 4, m2 of (0,1) = 3
    assert s.tri_v.tolist() == [[0, 3, 4], [1, 5, 3], [2, 4, 5], [5, 4, 3]]
    area = lambda t: 0.5 * ((s.xy[t[1], 0] - s.xy[t[0], 0]) * (s.xy[t[2], 1] - s.xy[t[0], 1])
                            - (s.xy[t[1], 1] - s.xy[t[0], 1]) * (s.xy[t[2], 0] - s.xy[t[0], 0]))
    assert [area(t) for t in s.tri_v] == [1.0] * 4  # the parent's area is 4
    assert (s.kind[3:] == FREE).all() and (s.line[3:] == -1).all()


def test_counts_kinds_and_lengths_on_a_scene():
    """The tiny scene's CDT (a disk: E = V + T - 1): V + E vertices, 4T triangles; the midpoint of
    every original edge (segments and box sides) and only those are CONSTRAINED, to their own
    edge; every old edge is split into two halves of half its length (to rounding) and the new
    edges are half the opposite sides, so the weight grows by half the sum of the perimeters."""
    sc = sg.make_scene("tiny")
    xy, tv, kd, ln, pv = sg.movable_input(sc)
    s = subdivide(xy, tv, kd, ln, pv)
    V, T = xy.shape[0], tv.shape[0]
    E = V + T - 1
    assert s.n_vertices == V + E and s.n_triangles == 4 * T
    cons = np.nonzero(s.kind == CONSTRAINED)[0]
    assert cons.size == pv.shape[0]
    for v in cons:
        a, b = pv[s.line[v]]
        assert np.array_equal(s.xy[v], (xy[a] + xy[b]) * 0.5)
    assert (s.kind[:V] == ORIGINAL).all()
    per = sum(sum(math.dist(xy[t[i]], xy[t[(i + 1) % 3]]) for i in range(3)) for t in tv)
    w0, w1 = _weight(tv, xy), _weight(s.tri_v, s.xy)
    assert abs(w1 - (w0 + 0.5 * per)) <= 1e-12 * w1


def test_second_round_keeps_constraints():
    """Subdividing the subdivided mesh: each original edge, in two pieces after the first round,
    is in four after the second, so three CONSTRAINED vertices lie on it."""
    sc = sg.make_scene("tiny")
    s1 = subdivide(*sg.movable_input(sc))
    s2 = subdivide(s1.xy, s1.tri_v, s1.kind, s1.line, s1.prim_v)
    counts = np.bincount(s2.line[s2.kind == CONSTRAINED], minlength=s1.prim_v.shape[0])
    assert (counts == 3).all()
    assert s2.n_triangles == 16 * sc.n_triangles


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("large", dict(n_seg=2000)), ("grid", {})])
def test_library_equals_checker(name, kw):
    ccsp = pytest.importorskip("paper_2112_05570_amd")
    sc = sg.make_scene(name, **kw)
    xy, tv, kd, ln, pv = sg.movable_input(sc)
    ref = subdivide(xy, tv, kd, ln, pv)
    tv2, kd2, ln2, pv2, xy2 = ccsp.subdivide(tv, kd, ln, pv, xy)
    assert np.array_equal(tv2, ref.tri_v) and np.array_equal(kd2, ref.kind)
    assert np.array_equal(ln2, ref.line) and np.array_equal(xy2, ref.xy)
    if name == "tiny":  # the second round, from a mesh with Steiner vertices
        ref2 = subdivide(ref.xy, ref.tri_v, ref.kind, ref.line, ref.prim_v)
        out = ccsp.subdivide(ref.tri_v, ref.kind, ref.line, ref.prim_v, ref.xy)
        assert all(np.array_equal(a, b) for a, b in
                   zip(out, (ref2.tri_v, ref2.kind, ref2.line, ref2.prim_v, ref2.xy)))


def test_library_rejects_bad_input():
    ccsp = pytest.importorskip("paper_2112_05570_amd")
    xy = np.array([[0.0, 0.0], [4.0, 0.0], [1.0, 2.0]])
    with pytest.raises(ccsp.CcspError):
        ccsp.subdivide([[0, 1, 3]], [0, 0, 0], [-1] * 3, np.zeros((0, 2)), xy)
    with pytest.raises(ccsp.CcspError):  # clockwise: its sub-triangles are too
        ccsp.subdivide([[0, 2, 1]], [0, 0, 0], [-1] * 3, np.zeros((0, 2)), xy)
    with pytest.raises(ccsp.CcspError):  # a CONSTRAINED vertex needs an original edge
        ccsp.subdivide([[0, 1, 2]], [0, 1, 0], [-1] * 3, np.zeros((0, 2)), xy)
