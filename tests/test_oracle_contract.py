"""Pins of the contraction checker (oracle/contract.py); CPU only.

A hand-built square with a short interior edge fixes the whole result by hand: the free pair
merges at the midpoint, an original vertex survives where it is, two original vertices are never
merged, and a pinched edge (a third common neighbour) is left alone. On meshes with many short
edges the result is a valid triangulation (exact orientation, Euler, edges shared by at most two
triangles) that keeps every original vertex, keeps each original edge covered by a chain of edges,
and is unchanged by a second contraction.
"""
import math

import numpy as np

import oracle
import helpers
import scenegen as sg
from oracle import contract as ct
from oracle import objective as ob

O, C, F = ob.ORIGINAL, ob.CONSTRAINED, ob.FREE


def _square(k4=F, k5=F):
    """Unit square (original corners 0..3) with vertices 4 = (0.5, 0.5) and 5 = (0.52, 0.5)."""
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5], [0.52, 0.5]], dtype=np.float64)
    tv = np.array([[0, 1, 5], [0, 5, 4], [1, 2, 5], [2, 4, 5], [2, 3, 4], [3, 0, 4]])
    kind = np.array([O, O, O, O, k4, k5])
    return tv, kind, np.zeros(6, dtype=np.int64), np.zeros((0, 2), dtype=np.int64), xy


def test_square_free_pair_merges_at_the_midpoint():
    tv, kind, line, prim_v, xy = _square()
    t2, k2, l2, xy2, m, n = ct.contract(tv, kind, line, prim_v, xy, 0.05)
    assert n == 1
    assert t2.tolist() == [[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]]
    assert xy2.tolist() == [[0, 0], [1, 0], [1, 1], [0, 1], [0.51, 0.5]]
    assert m.tolist() == [0, 1, 2, 3, 4, 4] and k2.tolist() == [O, O, O, O, F]


def test_square_original_survives_in_place_and_two_originals_do_not_merge():
    tv, kind, line, prim_v, xy = _square(k4=O)
    t2, _, _, xy2, _, n = ct.contract(tv, kind, line, prim_v, xy, 0.05)
    assert n == 1 and xy2[4].tolist() == [0.5, 0.5] and t2.shape == (4, 3)
    tv, kind, line, prim_v, xy = _square(k4=O, k5=O)
    t2, _, _, xy2, _, n = ct.contract(tv, kind, line, prim_v, xy, 0.05)
    assert n == 0 and np.array_equal(t2, tv) and np.array_equal(xy2, xy)


def test_pinched_edge_is_left_alone():
    """The cycle 4-5-6 encloses vertex 7, so 4 and 5 have a common neighbour (6) that is not
    opposite their edge: contracting (4, 5) would fold the cycle onto one edge (the link
    condition), and it is the only edge shorter than eps, so nothing changes."""
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.45, 0.3], [0.55, 0.3], [0.5, 0.7],
                   [0.5, 0.5]])
    tv = np.array([[0, 1, 5], [0, 5, 4], [1, 2, 5], [2, 6, 5], [2, 3, 6], [3, 4, 6], [3, 0, 4],
                   [4, 5, 7], [5, 6, 7], [6, 4, 7]])
    for tri in tv:
        assert oracle.orient(*xy[tri]) > 0
    assert len(_edges(tv)) == 17  # Euler: 8 - 17 + 10 = 1
    kind = np.array([O, O, O, O, F, F, O, O])
    e = 0.15
    short = [k for k in _edges(tv) if ct._len(xy, *k) < e]
    assert short == [(4, 5)]
    t2, _, _, xy2, _, n = ct.contract(tv, kind, np.zeros(8, dtype=np.int64),
                                      np.zeros((0, 2), dtype=np.int64), xy, e)
    assert n == 0 and np.array_equal(t2, tv) and np.array_equal(xy2, xy)
    # with vertex 7 gone (6 now opposite the edge) the same edge contracts
    tv7 = np.array([[0, 1, 5], [0, 5, 4], [1, 2, 5], [2, 6, 5], [2, 3, 6], [3, 4, 6], [3, 0, 4],
                    [4, 5, 6]])
    t3, _, _, xy3, _, n = ct.contract(tv7, kind[:7], np.zeros(7, dtype=np.int64),
                                      np.zeros((0, 2), dtype=np.int64), xy[:7], e)
    assert n == 1 and t3.shape == (6, 3) and xy3[4].tolist() == [0.5, 0.3]


def _edges(tv):
    e = {}
    for t in tv:
        for i in range(3):
            a, b = int(t[(i + 1) % 3]), int(t[(i + 2) % 3])
            e[(min(a, b), max(a, b))] = e.get((min(a, b), max(a, b)), 0) + 1
    return e


def _clustered_mesh(seed, eps):
    """The subdivided tiny scene with many vertices pulled next to a neighbour."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    om = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    rng = np.random.default_rng(seed)
    xy = mesh.xy.copy()
    for v in rng.choice(np.nonzero(mesh.kind != O)[0], 2500):
        nb = om.nbr[om.nbr_off[v]:om.nbr_off[v + 1]]
        w = nb[rng.integers(0, nb.shape[0])]
        r = 0.4 * eps * math.sqrt(rng.random())
        th = 2 * math.pi * rng.random()
        q = xy[w] + r * np.array([math.cos(th), math.sin(th)])
        if mesh.kind[v] == C:
            a, b = mesh.prim_v[mesh.line[v]]
            e = xy[b] - xy[a]
            q = xy[v] + ((q - xy[v]) @ e) / (e @ e) * e
        if ob.move_status(om, xy, int(v), q) == ob.MOVED:
            xy[v] = q
    return mesh, xy


def test_contracted_mesh_is_a_valid_triangulation():
    eps = 0.02
    mesh, xy = _clustered_mesh(1, eps)
    t2, k2, l2, xy2, m, n = ct.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    assert n > 50
    V, T = xy2.shape[0], t2.shape[0]
    assert V == mesh.kind.shape[0] - n
    e = _edges(t2)
    assert max(e.values()) <= 2 and V - len(e) + T == 1
    for t in t2:
        assert oracle.orient(*xy2[t]) > 0
    # original vertices all survive, where they were
    orig = np.nonzero(mesh.kind == O)[0]
    assert np.array_equal(xy2[m[orig]], xy[orig]) and (k2[m[orig]] == O).all()
    assert (k2 == O).sum() == orig.shape[0]
    # each original edge is still a chain of edges through the vertices on it
    for k, (a, b) in enumerate(mesh.prim_v):
        on = [int(m[a]), int(m[b])] + [v for v in range(V) if k2[v] == C and l2[v] == k]
        d = xy2[int(m[b])] - xy2[int(m[a])]
        on.sort(key=lambda v: (xy2[v] - xy2[int(m[a])]) @ d)
        for p, q in zip(on, on[1:]):
            assert (min(p, q), max(p, q)) in e
    # nothing left to contract
    assert ct.contract(t2, k2, l2, mesh.prim_v, xy2, eps)[5] == 0
    # the contraction shortened the weight
    w0 = sum(ct._len(xy, a, b) for a, b in _edges(mesh.tri_v))
    w1 = sum(ct._len(xy2, a, b) for a, b in e)
    assert w1 < w0


def test_no_triangle_flat_on_an_original_edge():
    """Segment A-B (original edge 0) with C constrained to it, 2^-60 below the line as rounding
    may leave it. Contracting the short edge A-G would turn (C, B, G) into (C, B, A): three
    vertices on the original edge, a triangle of zero area in intent that exact orientation alone
    accepts. It is refused."""
    va, vb, vc, vg, vf, vy = 0, 1, 2, 3, 4, 5
    xy = np.array([[0, 0], [3, 0], [1, -2.0 ** -60], [0.01, 0.005], [1.5, 1], [1.5, -1]])
    tv = np.array([[va, vc, vg], [vc, vb, vg], [va, vg, vf], [vg, vb, vf], [va, vy, vc],
                   [vc, vy, vb]])
    for tri in tv:
        assert oracle.orient(*xy[tri]) > 0
    assert oracle.orient(xy[vc], xy[vb], xy[va]) > 0  # the sliver would pass the orientation test
    kind = np.array([O, O, C, F, O, O])
    line = np.array([0, 0, 0, 0, 0, 0])
    prim_v = np.array([[va, vb]])
    short = [k for k in _edges(tv) if ct._len(xy, *k) < 0.05]
    assert short == [(va, vg)]
    t2, _, _, xy2, _, n = ct.contract(tv, kind, line, prim_v, xy, 0.05)
    assert n == 0 and np.array_equal(t2, tv)
