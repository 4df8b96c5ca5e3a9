"""Pins for the checker's continued walk (reflections at hits; Sec. 5.2's secondary rays)."""
import json
import os

import numpy as np

import oracle
import scenegen as sg

HERE = os.path.dirname(os.path.abspath(__file__))


def _square():
    with open(os.path.join(HERE, "golden", "unit_square_diagonal.json")) as f:
        g = json.load(f)
    return oracle.Triangulation(np.array(g["xy"], float), np.array(g["tri_v"], np.int32),
                                np.array(g["tri_nbr"], np.int32), np.array(g["tri_prim"], np.int32),
                                np.array(g["prims"], float))


def test_hand_derived_billiards():
    tri = _square()
    with open(os.path.join(HERE, "golden", "unit_square_bounces.json")) as f:
        cases = json.load(f)["rays"]
    for c in cases:
        p, t, s, h, face = oracle.bounce(tri, np.array([c["o"]]), np.array([c["d"]]),
                                         np.array([c["start"]], np.int32), c["bounces"])
        assert (p[0], t[0], s[0], h[0], face[0]) == (c["prim"], c["t"], c["steps"], c["hits"],
                                                      c["face"]), c


def test_zero_bounces_is_the_walk(tiny_scene, tiny_rays):
    tri = oracle.Triangulation.of(tiny_scene)
    r = tiny_rays
    p, t, s = oracle.walk(tri, r.o, r.d, r.start)
    bp, bt, bs, bh, face = oracle.bounce(tri, r.o, r.d, r.start, 0)
    assert np.array_equal(p, bp) and np.array_equal(t, bt) and np.array_equal(s, bs)
    assert (bh == 0).all()
    hit = bp >= 0
    assert np.array_equal(tiny_scene.tri_prim.reshape(-1)[(face[hit] >> 2) * 3 + (face[hit] & 3)], bp[hit])


def _reflect(o, d, seg, t):
    ex, ey = seg[2] - seg[0], seg[3] - seg[1]
    nx, ny = -ey, ex
    k = (2.0 * (d[0] * nx + d[1] * ny)) / (nx * nx + ny * ny)
    return np.array([o[0] + t * d[0], o[1] + t * d[1]]), np.array([d[0] - k * nx, d[1] - k * ny])


def test_segments_equal_brute_force_and_reflect(tiny_scene, tiny_rays):
    """Every continued segment hits what brute force over all primitives (but the one just hit)
    finds from the reflected ray; the reflection keeps |d| and flips the normal component."""
    tri = oracle.Triangulation.of(tiny_scene)
    r = tiny_rays.slice(0, 3000)
    prev = oracle.bounce(tri, r.o, r.d, r.start, 0)
    o, d = r.o.copy(), r.d.copy()
    checked = 0
    for b in range(1, 4):
        p, t, s, h, face = oracle.bounce(tri, r.o, r.d, r.start, b)
        for k in np.nonzero((prev[0] >= 0) & (h == b))[0]:
            seg = tiny_scene.prims[prev[0][k]]
            o2, d2 = _reflect(o[k], d[k], seg, prev[1][k])
            n = np.array([-(seg[3] - seg[1]), seg[2] - seg[0]])
            assert abs(np.hypot(*d2) - np.hypot(*d[k])) <= 1e-12 * np.hypot(*d[k])
            assert abs(d2 @ n + d[k] @ n) <= 1e-12 * np.hypot(*d[k]) * np.hypot(*n)
            prims = tiny_scene.prims.copy()
            prims[prev[0][k]] = [1e6, 1e6, 1e6 + 1, 1e6]  # the segment it leaves
            bp, bt, st = oracle.brute_prims(prims, o2[None], d2[None])
            assert st == 0 and bp[0] == p[k] and bt[0] == t[k], (k, b)
            o[k], d[k] = o2, d2
            checked += 1
        prev = (p, t)
    assert checked > 6000


def test_bounces_do_not_depend_on_the_triangulation(tiny_scene, tiny_rays):
    an, _ = sg.anneal_flips(tiny_scene, seed=1)
    start_an = sg.locate(an, tiny_rays.o)
    a = oracle.bounce(oracle.Triangulation.of(tiny_scene), tiny_rays.o, tiny_rays.d, tiny_rays.start, 5)
    b = oracle.bounce(oracle.Triangulation.of(an), tiny_rays.o, tiny_rays.d, start_an, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
    assert not np.array_equal(a[2], b[2])
