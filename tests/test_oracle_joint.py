"""Pins of the checker's joint move (the second variant of Sec. 3.2.2, oracle/objective.py
joint_move); CPU only.

The joint move's change of f is a sum of term differences over the whole mesh. It is pinned
against the single-vertex change of f (delta_f, itself pinned against full evaluations): a joint
move of one vertex is that move, and a joint move of vertices more than four edges apart changes f
by the sum of their single moves, each taken from the positions before the joint move. The
decision, the projection of constrained vertices, validity and the rejected inputs follow the
paper's rules.
"""
import math

import numpy as np
import pytest

import helpers
import scenegen as sg
from oracle import objective as ob


@pytest.fixture(scope="module")
def tiny():
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    return mesh, ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)


def _far_apart(om, rng, n, hops=4):
    """n movable vertices pairwise more than `hops` edges apart (greedy over a random order)."""
    chosen, blocked = [], set()
    for v in rng.permutation(om.nv):
        v = int(v)
        if om.kind[v] == ob.ORIGINAL or v in blocked:
            continue
        chosen.append(v)
        seen, front = {v}, [v]
        for _ in range(hops):
            nxt = []
            for a in front:
                for w in om.nbr[om.nbr_off[a]:om.nbr_off[a + 1]].tolist():
                    if w not in seen:
                        seen.add(w)
                        nxt.append(w)
            front = nxt
        blocked |= seen
        if len(chosen) == n:
            break
    return chosen


def _single(om, xy, p, v, lam, x):
    """The single move of v by (lam * sqrt(star area)) * x: (status, delta, bound, q)."""
    k = lam * math.sqrt(ob.star_area(om, xy, v))
    q = xy[v] + ob.project(om, xy, v, np.array([k * x[0], k * x[1]]))
    s, d, bound = ob.delta_f(om, xy, p, v, q)
    return s, d, bound, q


def test_one_vertex_is_the_single_move(tiny):
    mesh, om = tiny
    p = ob.Params(0.03)
    rng = np.random.default_rng(3)
    movable = np.nonzero(mesh.kind != sg.ORIGINAL)[0]
    done = 0
    for v in rng.choice(movable, 40, replace=False):
        x = rng.standard_normal(2)
        s1, d1, b1, q = _single(om, mesh.xy, p, int(v), 0.05, x)
        st, d, b, new, _ = ob.joint_move(om, mesh.xy, p, 1e-3, 0.05, [int(v)], [x], 0.5)
        if s1 != ob.MOVED:
            assert st == ob.FOLDED
            continue
        assert st in (ob.ACCEPTED, ob.REJECTED)
        assert abs(d - d1) <= b + b1 + 1e-300
        if st == ob.ACCEPTED:
            assert np.array_equal(new[int(v)], q)
        done += 1
    assert done > 20


def test_far_apart_vertices_add_up(tiny):
    mesh, om = tiny
    p = ob.Params(0.03)
    rng = np.random.default_rng(4)
    added = 0
    for trial in range(5):
        vids = _far_apart(om, rng, 6)
        assert len(vids) == 6
        xi = 0.3 * rng.standard_normal((6, 2))
        singles = [_single(om, mesh.xy, p, v, 0.05, xi[i]) for i, v in enumerate(vids)]
        st, d, b, new, _ = ob.joint_move(om, mesh.xy, p, 0.0, 0.05, vids, xi, 0.5)
        if any(s[0] != ob.MOVED for s in singles):
            assert st == ob.FOLDED
            continue
        total = sum(s[1] for s in singles)
        assert abs(d - total) <= b + sum(s[2] for s in singles) + 1e-300, trial
        # at T = 0 the move is taken exactly when f does not rise
        assert (st == ob.ACCEPTED) == (d <= 0.0)
        if st == ob.ACCEPTED:
            for i, v in enumerate(vids):
                assert np.array_equal(new[v], singles[i][3])
        added += 1
    assert added >= 3


def test_constrained_vertices_stay_on_their_edge(tiny):
    mesh, om = tiny
    p = ob.Params(0.03)
    rng = np.random.default_rng(5)
    cons = np.nonzero(mesh.kind == sg.CONSTRAINED)[0]
    vids = [int(v) for v in rng.choice(cons, 5, replace=False)]
    xi = 0.2 * rng.standard_normal((5, 2))
    st, d, b, new, _ = ob.joint_move(om, mesh.xy, p, 1e9, 0.05, vids, xi, 0.0)
    assert st == ob.ACCEPTED  # T huge, u = 0: any valid move is taken
    for v in vids:
        a, c = mesh.prim_v[mesh.line[v]]
        e, w = mesh.xy[c] - mesh.xy[a], new[v] - mesh.xy[a]
        assert abs(e[0] * w[1] - e[1] * w[0]) <= 1e-12 * np.dot(e, e)


def test_invalid_inputs_and_folds(tiny):
    mesh, om = tiny
    p = ob.Params(0.03)
    free = [int(v) for v in np.nonzero(mesh.kind == sg.FREE)[0][:3]]
    orig = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
    x = np.full((3, 2), 0.1)
    for vids, xs in (([free[0], free[1], free[0]], x), ([free[0], orig, free[1]], x),
                     ([free[0], free[1], mesh.n_vertices], x),
                     (free, np.array([[0.1, 0.1], [np.nan, 0.0], [0.1, 0.1]]))):
        st, d, _, new, _ = ob.joint_move(om, mesh.xy, p, 1e-3, 0.05, vids, xs, 0.5)
        assert st == ob.BAD and d == math.inf and np.array_equal(new, mesh.xy)
    st, d, _, new, _ = ob.joint_move(om, mesh.xy, p, 1e-3, 50.0, free, x, 0.5)
    assert st == ob.FOLDED and d == math.inf and np.array_equal(new, mesh.xy)


def test_one_group_is_the_group_move(tiny):
    """Joint groups with one centre are that centre's group move (group_chain's single step):
    same status, positions and change of f."""
    mesh, om = tiny
    p = ob.Params(0.05)
    rng = np.random.default_rng(8)
    movable = np.nonzero(mesh.kind != sg.ORIGINAL)[0]
    seen = set()
    for c in rng.choice(movable, 25, replace=False):
        xi = 0.3 * rng.standard_normal((1, 2))
        rd = rng.random(1)
        u = rng.random(1)
        xy_c, st_c, df_c, _, size = ob.group_chain(om, mesh.xy, p, 1e-3, 0.05, [int(c)], xi, rd, u)
        st, d, b, new, _ = ob.joint_groups(om, mesh.xy, p, 1e-3, 0.05, [int(c)], xi, rd, u[0])
        assert st == st_c[0]
        assert np.array_equal(new, xy_c)
        if st in (ob.ACCEPTED, ob.REJECTED):
            assert d == df_c[0]
        seen.add(int(st))
        seen.add(-int(size[0] > 1))
    assert {ob.ACCEPTED, ob.REJECTED, -1} <= seen


def test_far_apart_groups_add_up_and_overlaps_take_the_first(tiny):
    """Groups far apart change f by the sum of their single moves; a vertex in two groups moves
    with the first group's displacement."""
    mesh, om = tiny
    p = ob.Params(0.02)
    rng = np.random.default_rng(9)
    added = 0
    for trial in range(6):
        cs = _far_apart(om, rng, 3, hops=12)
        xi = 0.2 * rng.standard_normal((3, 2))
        rd = np.zeros(3)  # d = eps / 2: small groups
        singles = [ob.group_chain(om, mesh.xy, p, 0.0, 0.05, [c], xi[i:i + 1], rd[i:i + 1],
                                  [0.5]) for i, c in enumerate(cs)]
        st, d, b, new, _ = ob.joint_groups(om, mesh.xy, p, 0.0, 0.05, cs, xi, rd, 0.5)
        if any(sg_[1][0] == ob.FOLDED for sg_ in singles):
            assert st == ob.FOLDED
            continue
        total = sum(sg_[2][0] for sg_ in singles)
        assert abs(d - total) <= b + 1e-9 * sum(abs(sg_[2][0]) for sg_ in singles) + 1e-300
        added += 1
    assert added >= 3
    # overlapping groups: a centre and its neighbour, both with a large d
    free = [int(v) for v in np.nonzero(mesh.kind == sg.FREE)[0]]
    c0 = free[0]
    c1 = int(next(w for w in om.nbr[om.nbr_off[c0]:om.nbr_off[c0 + 1]] if mesh.kind[w] == sg.FREE))
    xi = np.array([[1e-3, 0.0], [0.0, 1e-3]])
    rd = np.ones(2)
    st, d, b, new, _ = ob.joint_groups(om, mesh.xy, p, 1e9, 0.05, [c0, c1], xi, rd, 0.0)
    m0 = ob.group_members(om, mesh.xy, c0, 5.0 * p.eps)
    k0 = 0.05 * math.sqrt(ob.group_area(om, mesh.xy, m0))
    assert st == ob.ACCEPTED and c1 in m0
    want = mesh.xy[c1] + ob.project(om, mesh.xy, c1, np.array([k0 * 1e-3, 0.0]))
    assert np.array_equal(new[c1], want)


def test_joint_groups_bad_inputs(tiny):
    mesh, om = tiny
    p = ob.Params(0.05)
    free = [int(v) for v in np.nonzero(mesh.kind == sg.FREE)[0][:2]]
    orig = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
    xi = np.full((2, 2), 0.1)
    for cs, x, rd in (([free[0], orig], xi, np.zeros(2)), ([free[0], mesh.n_vertices], xi, np.zeros(2)),
                      (free, np.array([[0.1, np.inf], [0.1, 0.1]]), np.zeros(2))):
        st, d, _, new, _ = ob.joint_groups(om, mesh.xy, p, 1e-3, 0.05, cs, x, rd, 0.5)
        assert st == ob.BAD and d == math.inf and np.array_equal(new, mesh.xy)
