"""Pins of the edge-flip annealing checker (oracle/flips.py); CPU only."""
import numpy as np

import oracle
import scenegen as sg
from oracle import flips as fl


def test_splitmix64_reference_outputs():
    """The first outputs of SplitMix64 from state 0, as published with the generator."""
    out = [fl.splitmix64(k * fl.GOLDEN) for k in (1, 2, 3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    p, u = fl.draws(0, 0, 0)
    assert p == 0xE220A8397B1DCDAF and u == (0x6E789E6AA1B965F4 >> 11) * 2.0 ** -53


def _quad(dy):
    """Triangles (a, b, c) and (d, c, b) of the quad a=(0,0), b=(1,-dy), d=(2,0), c=(1,dy)."""
    xy = np.array([[0.0, 0.0], [1.0, -dy], [1.0, dy], [2.0, 0.0]])
    tv = np.array([[0, 1, 2], [3, 2, 1]])
    nbr = np.array([[1, -1, -1], [0, -1, -1]])
    prim = -np.ones((2, 3), dtype=np.int64)
    return xy, tv, nbr, prim


def test_single_quad():
    """A flat rhombus flips to its shorter diagonal at T = 0; a tall one keeps its diagonal; a
    non-convex quad never flips, whatever the temperature."""
    xy, tv, nbr, prim = _quad(0.2)  # diagonal b-c of length 0.4 against a-d of length 2
    ok, ch = fl.try_flip(xy, tv.copy(), nbr.copy(), prim.copy(), 0, 0.0, 0.5)
    assert not ok and abs(ch - 1.6) < 1e-15
    xy, tv, nbr, prim = _quad(3.0)  # b-c of length 6 against 2
    ok, ch = fl.try_flip(xy, tv, nbr, prim, 0, 0.0, 0.5)
    assert ok and abs(ch + 4.0) < 1e-15
    assert tv.tolist() == [[0, 1, 3], [0, 3, 2]] and nbr.tolist() == [[-1, 1, -1], [-1, -1, 0]]
    assert oracle.orient(*xy[tv[0]]) > 0 and oracle.orient(*xy[tv[1]]) > 0
    xy, tv, nbr, prim = _quad(3.0)
    xy[3] = [1.2, 6.0]  # (d, c, b) stays counter-clockwise, the quad is reflex at c
    assert oracle.orient(xy[3], xy[2], xy[1]) > 0 and oracle.orient(xy[0], xy[3], xy[2]) < 0
    assert fl.try_flip(xy, tv, nbr, prim, 0, 1e300, 0.0) == (False, 0.0)


def _scene():
    sc = sg.make_scene("tiny")
    return sc, sc.tri_v.astype(np.int64), sc.tri_nbr.astype(np.int64), sc.tri_prim.astype(np.int64)


def test_rounds_are_independent_and_order_free():
    """Chosen flips touch disjoint triangles, and applying them in reverse order gives the same
    triangulation."""
    sc, tv, nbr, prim = _scene()
    for r in range(3):
        ch = fl.chosen(tv, nbr, prim, 7, r)
        assert len(ch) > 5
        seen = set()
        for s in ch:
            t = fl.touched(nbr, s)
            assert not (t & seen)
            seen |= t
        a = [x.copy() for x in (tv, nbr, prim)]
        b = [x.copy() for x in (tv, nbr, prim)]
        for s in ch:
            fl.try_flip(sc.xy, *a, s, 1e-3, fl.draws(7, r, s)[1])
        for s in reversed(ch):
            fl.try_flip(sc.xy, *b, s, 1e-3, fl.draws(7, r, s)[1])
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        tv, nbr, prim = a


def test_annealing_keeps_a_valid_triangulation_and_converges():
    """Rounds at falling temperature then at 0: the triangulation stays valid (orientation,
    adjacency, Euler, constraints covered), the weight falls by the accepted changes, and at the
    end no unconstrained interior edge has a strictly convex quad with a shorter other diagonal."""
    sc, tv, nbr, prim = _scene()
    w0 = fl.weight(sc.xy, tv, nbr)
    temps = list(np.geomspace(2e-2, 1e-4, 12)) + [0.0] * 30
    tv2, nbr2, prim2, counts = fl.anneal(sc.xy, tv, nbr, prim, temps, 3)
    assert counts[-1] == 0 and sum(counts) > 10
    an = sc.copy_with(tv2.astype(np.int32), nbr2.astype(np.int32), prim2.astype(np.int32))
    assert oracle.validate(oracle.Triangulation.of(an)) == ""
    assert fl.weight(sc.xy, tv2, nbr2) < w0
    for s in fl.candidates(tv2, nbr2, prim2):
        t, i = divmod(s, 3)
        u = nbr2[t, i]
        j = [k for k in range(3) if nbr2[u, k] == t][0]
        a, b, c, d = tv2[t, i], tv2[t, (i + 1) % 3], tv2[t, (i + 2) % 3], tv2[u, j]
        convex = oracle.orient(sc.xy[a], sc.xy[b], sc.xy[d]) > 0 and \
            oracle.orient(sc.xy[a], sc.xy[d], sc.xy[c]) > 0
        assert not convex or fl._len(sc.xy, a, d) >= fl._len(sc.xy, b, c)


def test_no_flip_makes_a_triangle_flat_on_an_original_edge():
    """Segment A-B (original edge 0) through constrained C, 2^-60 below the line. The quad
    A, C, B, X is strictly convex by exact orientation only through that rounding; flipping X-C to
    A-B would make the triangle (A, C, B) of zero area in intent. At a temperature that accepts any
    valid flip, it happens without the vertices' original edges and is refused with them."""
    A, B, Cv, X, Y = 0, 1, 2, 3, 4
    xy = np.array([[0, 0], [3, 0], [1.5, -2.0 ** -60], [1.5, 0.05], [1.5, -1]])
    tv = np.array([[X, A, Cv], [X, Cv, B], [Cv, A, Y], [Cv, Y, B]])
    nbr = np.array([[2, 1, -1], [3, -1, 0], [-1, 3, 0], [-1, 1, 2]])
    prim = np.array([[0, -1, -1], [0, -1, -1], [-1, -1, 0], [-1, 0, -1]])
    for ti in range(4):
        assert oracle.orient(*xy[tv[ti]]) > 0
        for i in range(3):
            u = nbr[ti, i]
            if u >= 0:  # edge i is (v[i+1], v[i+2]); the neighbour holds it reversed
                k = [k for k in range(3) if nbr[u, k] == ti][0]
                assert (tv[u, (k + 1) % 3], tv[u, (k + 2) % 3]) == \
                    (tv[ti, (i + 2) % 3], tv[ti, (i + 1) % 3])
                assert prim[u, k] == prim[ti, i]
    s = 1  # edge (C, X) in triangle 0, the lower id of its two triangles
    assert oracle.orient(xy[A], xy[Cv], xy[B]) > 0  # the new triangle passes the exact test
    assert fl.test_flip(xy, tv, nbr, s, 1e9, 0.5)[0]
    line = np.array([-1, -1, 0, -1, -1])
    pv = np.array([[A, B]])
    assert fl.test_flip(xy, tv, nbr, s, 1e9, 0.5, line, [tuple(p) for p in pv]) == (False, 0.0)
    tv2, nbr2, prim2, counts = fl.anneal(xy, tv, nbr, prim, [1e9, 1e9], 5, line, pv)
    assert counts == [0, 0] and np.array_equal(tv2, tv)
    assert fl.anneal(xy, tv, nbr, prim, [1e9], 5)[3] == [1]
