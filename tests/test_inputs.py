"""Input builders checked by the independent validator, and the validator checked by planted
mistakes (all on the CPU)."""
import numpy as np
import pytest

import oracle
import scenegen as sg


def _counts(sc):
    S = sc.seg_v.shape[0]
    V = 2 * S + 4
    T = 2 * V - 4 - 2  # Euler with a 4-vertex hull and no Steiner points
    return V, T


def test_tiny_shape_and_validity(tiny_scene):
    V, T = _counts(tiny_scene)
    assert tiny_scene.n_vertices == V == 132 and tiny_scene.n_triangles == T == 258
    assert tiny_scene.n_prims == 68
    assert oracle.validate(oracle.Triangulation.of(tiny_scene), delaunay=True) == ""


def test_segments_strictly_inside_and_disjoint(tiny_scene):
    seg = tiny_scene.prims[:-4]
    assert ((seg > 0) & (seg < 1)).all()
    L = np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1])
    assert (L >= 0.02 - 1e-12).all() and (L <= 0.1 + 1e-12).all()
    # pairwise: no two segments touch (exact signs from the checker)
    for i in range(seg.shape[0]):
        for j in range(i + 1, seg.shape[0]):
            a, b, c, d = seg[i, :2], seg[i, 2:], seg[j, :2], seg[j, 2:]
            o1, o2 = oracle.orient(a, b, c), oracle.orient(a, b, d)
            o3, o4 = oracle.orient(c, d, a), oracle.orient(c, d, b)
            assert o1 * o2 > 0 or o3 * o4 > 0


def test_rays_strictly_inside_start(tiny_scene, tiny_rays):
    r = tiny_rays
    assert r.n == 65536
    tv = tiny_scene.tri_v[r.start]
    for k in range(0, r.n, 97):
        for i in range(3):
            a = tiny_scene.xy[tv[k, (i + 1) % 3]]
            b = tiny_scene.xy[tv[k, (i + 2) % 3]]
            assert oracle.orient(a, b, r.o[k]) > 0
    np.testing.assert_allclose(np.hypot(r.d[:, 0], r.d[:, 1]), 1.0, atol=4e-16)


def test_rays_are_area_weighted(tiny_scene, tiny_rays):
    xy = tiny_scene.xy[tiny_scene.tri_v]
    area = 0.5 * ((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1])
                  - (xy[:, 1, 1] - xy[:, 0, 1]) * (xy[:, 2, 0] - xy[:, 0, 0]))
    cnt = np.bincount(tiny_rays.start, minlength=tiny_scene.n_triangles)
    exp = area / area.sum() * tiny_rays.n
    big = exp > 200
    z = (cnt[big] - exp[big]) / np.sqrt(exp[big])
    assert np.abs(z).max() < 5.5
    # origins uniform over the square: quadrant counts
    q = (tiny_rays.o[:, 0] > 0.5) * 2 + (tiny_rays.o[:, 1] > 0.5)
    assert np.abs(np.bincount(q) / tiny_rays.n - 0.25).max() < 0.01


def test_deterministic(tiny_scene):
    sc2 = sg.make_scene("tiny", seed=0)
    assert np.array_equal(sc2.xy, tiny_scene.xy) and np.array_equal(sc2.tri_v, tiny_scene.tri_v)
    r1 = sg.sample_rays(tiny_scene, 1000, seed=0, threads=1)
    r2 = sg.sample_rays(tiny_scene, 1000, seed=0, threads=4)
    assert np.array_equal(r1.o, r2.o) and np.array_equal(r1.start, r2.start)
    assert not np.array_equal(sg.sample_rays(tiny_scene, 1000, seed=1).o, r1.o)


@pytest.fixture(scope="module")
def grid_pair():
    sc = sg.make_scene("grid")
    an, stats = sg.anneal_flips(sc, seed=0)
    return sc, an, stats


def test_grid_cdt_and_annealed(grid_pair):
    sc, an, stats = grid_pair
    V, T = _counts(sc)
    assert sc.n_prims == 130560 + 4 and sc.n_triangles == T == 522242
    assert oracle.validate(oracle.Triangulation.of(sc), delaunay=True) == ""
    assert oracle.validate(oracle.Triangulation.of(an)) == ""
    assert an.n_triangles == sc.n_triangles
    assert stats["w_end"] < stats["w_start"]
    assert abs(sg.weight(an) - stats["w_end"]) < 1e-6 * stats["w_end"]


def _broken(sc, what):
    tv, tn, tp = sc.tri_v.copy(), sc.tri_nbr.copy(), sc.tri_prim.copy()
    t = int(np.nonzero((tn >= 0).all(1) & (tp < 0).all(1))[0][0])
    if what == "cw":
        tv[t, [1, 2]] = tv[t, [2, 1]]
    elif what == "adjacency":
        tn[t, 0] = tn[t, 1]
    elif what == "prim":
        tp[t, 0] = 3
    elif what == "euler":
        tn[t, 0] = -1
    elif what == "delaunay":
        # flip an unconstrained edge of a CDT: the result is valid but not Delaunay
        return None
    return oracle.Triangulation(sc.xy, tv, tn, tp, sc.prims)


@pytest.mark.parametrize("what", ["cw", "adjacency", "prim", "euler"])
def test_validator_catches_planted_mistakes(tiny_scene, what):
    assert oracle.validate(_broken(tiny_scene, what)) != ""


def test_validator_catches_non_delaunay(tiny_scene):
    an, _ = sg.anneal_flips(tiny_scene, seed=3, moves_per_edge=2.0, t1_rel=1e-2)
    tri = oracle.Triangulation.of(an)
    assert oracle.validate(tri) == ""
    # greedy flips shorten edges; the result differs from the CDT, so some edge is not Delaunay
    if not np.array_equal(an.tri_v, tiny_scene.tri_v):
        assert "Delaunay" in oracle.validate(tri, delaunay=True)


def test_validator_catches_uncovered_primitive(tiny_scene):
    tp = tiny_scene.tri_prim.copy()
    tp[tp == 5] = -1
    assert "covered" in oracle.validate(oracle.Triangulation(tiny_scene.xy, tiny_scene.tri_v,
                                                            tiny_scene.tri_nbr, tp, tiny_scene.prims))


def test_multi_scene_sizes():
    segs, rays = sg.multi_sizes("batch", seed=0)
    assert segs.shape == (256,) and segs.min() >= 100 and segs.max() <= 100_000
    assert rays.min() >= 1024 and rays.max() <= 1 << 20
    segs, rays = sg.multi_sizes("serve", seed=0)
    assert segs.shape == (64,) and segs.min() >= 1000 and segs.max() <= 500_000
