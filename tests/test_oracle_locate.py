"""Pins for the checker's point location (paper Sec. 5.2), against things other than itself:
hand-derived cases on the unit square split by its diagonal, and ray origins whose containing
triangle is known by construction (the generator draws each origin inside its start triangle and
checks strict inclusion exactly)."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _square():
    with open(os.path.join(HERE, "golden", "unit_square_diagonal.json")) as f:
        g = json.load(f)
    return oracle.Triangulation(np.array(g["xy"], float), np.array(g["tri_v"], np.int32),
                                np.array(g["tri_nbr"], np.int32), np.array(g["tri_prim"], np.int32),
                                np.array(g["prims"], float))


def test_locate_hand_cases():
    tri = _square()
    q = np.array([[0.75, 0.25], [0.25, 0.75], [0.5, 0.5], [0.0, 0.0], [1.0, 0.5], [2.0, 2.0],
                  [-1e-300, 0.5], [np.nan, 0.5], [0.5, np.inf]])
    t, s = oracle.locate(tri, q)
    # triangle 0 = (0,0),(1,0),(1,1) below the diagonal; triangle 1 above it
    assert list(s) == [0, 0, 1, 1, 1, -1, -1, -2, -2]
    assert t[0] == 0 and t[1] == 1
    assert t[2] in (0, 1) and t[3] in (0, 1) and t[4] == 0  # (1, 0.5) is on triangle 0's side
    assert t[5] == -1 and t[6] == -1


def test_locate_ray_origins(tiny_scene, tiny_rays):
    tri = oracle.Triangulation.of(tiny_scene)
    t, s = oracle.locate(tri, tiny_rays.o)
    assert (s == 0).all() and np.array_equal(t, tiny_rays.start)


def test_locate_vertices_are_on_the_boundary(tiny_scene):
    tri = oracle.Triangulation.of(tiny_scene)
    t, s = oracle.locate(tri, tiny_scene.xy)
    assert (s == 1).all()
    for v in range(tiny_scene.n_vertices):
        assert v in tiny_scene.tri_v[t[v]]
