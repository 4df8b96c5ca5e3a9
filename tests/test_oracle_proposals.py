"""Pins of the checker's vertex proposals of Secs. 3.2.4-3.2.6 (oracle/objective.py); CPU only.

Each pin checks the proposal against what the paper states it samples, not against its own code:
uniform density by area over the vertex's triangles, validity inside a convex star, positions
within the drawn radius of the chosen neighbour, the contraction-change rule, the constrained
projection, and a zero-temperature chain that never raises f.
"""
import math

import numpy as np
import pytest

import oracle
import helpers
import scenegen as sg
from oracle import objective as ob

scipy_stats = pytest.importorskip("scipy.stats")


def _star(radii, centre=(0.0, 0.0)):
    """A free vertex 0 at `centre` inside a ring of original vertices 1..n at angles 2 pi k / n."""
    n = len(radii)
    ring = [[r * math.cos(2 * math.pi * k / n), r * math.sin(2 * math.pi * k / n)]
            for k, r in enumerate(radii)]
    xy = np.array([list(centre)] + ring)
    tv = np.array([[0, 1 + k, 1 + (k + 1) % n] for k in range(n)])
    kind = np.array([ob.FREE] + [ob.ORIGINAL] * n)
    m = ob.Mesh(tv, kind, np.zeros(n + 1, dtype=np.int64), np.zeros((0, 2), dtype=np.int64))
    return m, xy


def _containing(xy, tv, q):
    """Ids of the triangles holding q (closed), by exact orientation."""
    return [t for t in range(tv.shape[0])
            if all(oracle.orient(xy[tv[t, i]], xy[tv[t, (i + 1) % 3]], q) >= 0 for i in range(3))]


def test_resample_is_uniform_by_area():
    """Counts per triangle follow the areas (chi-square), each point lies in the triangle it was
    drawn in, and the points of the largest triangle average to its centroid."""
    radii = [1.0, 2.0, 1.0, 3.0, 1.5, 1.0]
    m, xy = _star(radii)
    areas = np.array([ob._tri_area(xy, m.tri_v[t]) for t in range(6)])
    rng = np.random.default_rng(1)
    n = 30000
    r = rng.random((n, 3))
    pts = np.array([ob.resample_in_star(m, xy, 0, *r[i]) for i in range(n)])
    # the triangle drawn: the running-sum rule, written out independently
    cum = np.cumsum(areas)
    drawn = np.searchsorted(cum, r[:, 0] * cum[-1], side="right").clip(max=5)
    for i in range(0, n, 97):
        assert drawn[i] in _containing(xy, m.tri_v, pts[i])
    counts = np.bincount(drawn, minlength=6)
    chi2 = ((counts - n * areas / areas.sum()) ** 2 / (n * areas / areas.sum())).sum()
    assert chi2 < scipy_stats.chi2.ppf(1 - 1e-6, 5), (counts, areas)
    big = int(np.argmax(areas))
    sel = pts[drawn == big]
    centroid = xy[m.tri_v[big]].mean(axis=0)
    se = sel.std(axis=0) / math.sqrt(sel.shape[0])
    assert (np.abs(sel.mean(axis=0) - centroid) < 5 * se).all()


def test_resample_in_convex_star_is_always_valid():
    """Inside a convex star every resampled position keeps the triangulation valid (Sec. 3.2.4)."""
    radii = [1.0, 1.2, 1.0, 1.1, 1.0, 1.3]
    m, xy = _star(radii, centre=(0.2, -0.1))
    ring = xy[1:]
    assert all(oracle.orient(ring[k], ring[(k + 1) % 6], ring[(k + 2) % 6]) > 0 for k in range(6))
    rng = np.random.default_rng(2)
    for r in rng.random((2000, 3)):
        q = ob.resample_in_star(m, xy, 0, *r)
        assert ob.move_status(m, xy, 0, q) == ob.MOVED


def _disk(rng, n):
    rad = np.sqrt(rng.random(n))
    th = 2 * math.pi * rng.random(n)
    return np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)


def test_swap_proposal():
    """A vertex with an edge shorter than the drawn l moves into the disk of radius l around the
    neighbour of rank floor(r1 deg); with none shorter, nothing is proposed; l covers
    [0.2 eps, 2 eps)."""
    m, xy = _star([1.0] * 6, centre=(0.95, 0.0))  # 0.05 from vertex 1
    p = ob.Params(0.1)
    rng = np.random.default_rng(3)
    n = 4000
    r = np.concatenate([rng.random((n, 2)), _disk(rng, n)], axis=1)
    nb = m.nbr[m.nbr_off[0]:m.nbr_off[1]]
    assert nb.tolist() == [1, 2, 3, 4, 5, 6]
    skipped, ranks = 0, np.zeros(6, dtype=np.int64)
    for i in range(n):
        ln = 0.02 + 0.18 * r[i, 0]
        q = ob.propose(m, xy, p, 0, ob.SWAP, r[i])
        if ln <= 0.05 - 1e-12:
            assert q is None
        if q is None:
            skipped += 1
            assert ln <= 0.05 + 1e-12
            continue
        k = int(r[i, 1] * 6)
        ranks[k] += 1
        assert np.hypot(*(q - xy[nb[k]])) <= ln * (1 + 1e-12)
    assert abs(skipped / n - 0.03 / 0.18) < 0.03
    assert ranks.min() > 0.8 * ranks.mean()


def test_contract_proposal_changes_the_contracted_state():
    """A contraction move is proposed exactly when the vertex's contracted state (an edge shorter
    than eps) differs between its old and new positions; an uncontracted vertex goes near a
    neighbour, a contracted one away from all."""
    p = ob.Params(0.3)
    rng = np.random.default_rng(4)
    for centre, was in (((0.1, 0.05), False), ((0.8, 0.05), True)):
        m, xy = _star([1.0] * 6, centre=centre)
        assert bool((ob.incident_lengths(m, xy, 0) < p.eps).any()) == was
        kept = 0
        for r in rng.random((3000, 4)):
            q = ob.propose(m, xy, p, 0, ob.CONTRACT, r)
            raw = ob.resample_in_star(m, xy, 0, r[0], r[1], r[2])
            base = xy[0] + (raw - xy[0])  # the move is formed as o + (q - o)
            now = bool((ob.incident_lengths(m, xy, 0, base) < p.eps).any())
            if now == was:
                assert q is None
            else:
                kept += 1
                assert np.array_equal(q, base)
        assert kept > 30


def test_constrained_proposals_stay_on_their_edge():
    """Proposals for a constrained vertex are projected on its original edge (Sec. 3.2.1)."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    xy = mesh.xy
    cons = np.nonzero(mesh.kind == ob.CONSTRAINED)[0][:10]
    rng = np.random.default_rng(5)
    p = ob.Params(0.05)
    for v in cons:
        a, b = xy[m.prim_v[m.line[v]]]
        e = b - a
        for r in rng.random((20, 3)):
            q = ob.propose(m, xy, p, int(v), ob.RESAMPLE, np.append(r, 0.0))
            w = q - a
            assert abs(e[0] * w[1] - e[1] * w[0]) <= 1e-12 * np.hypot(*e) * (1 + np.hypot(*w))


@pytest.mark.parametrize("kind", [ob.RESAMPLE, ob.SWAP, ob.CONTRACT])
def test_zero_temperature_chain_never_raises_f(kind):
    """At T = 0 only moves that do not raise f are taken: f falls by the sum of the accepted
    changes, and only accepted vertices move."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    p = ob.Params(0.05)
    rng = np.random.default_rng(6)
    vid = np.nonzero(mesh.kind != ob.ORIGINAL)[0]
    r = np.concatenate([rng.random((vid.shape[0], 2)), _disk(rng, vid.shape[0])], axis=1)
    if kind != ob.SWAP:
        r[:, 2] = rng.random(vid.shape[0])
    xy1, st, df, _ = ob.proposal_chain(m, mesh.xy, p, 0.0, kind, vid, r, rng.random(vid.shape[0]))
    f0 = ob.objective(m, mesh.xy, p)["f"]
    f1 = ob.objective(m, xy1, p)["f"]
    acc = st == ob.ACCEPTED
    assert acc.sum() > 0 and (df[acc] <= 0).all()
    assert abs((f1 - f0) - df[acc].sum()) < 1e-9 * (1 + abs(f0))
    moved = (xy1 != mesh.xy).any(axis=1)
    assert not moved[np.setdiff1d(np.arange(mesh.kind.shape[0]), vid[acc])].any()
    if kind == ob.SWAP:
        assert (st == ob.SKIPPED).sum() > 0


def test_group_members_and_area():
    """With d just above the two nearest neighbours' distance, no other vertex comes that close in
    a CDT-based mesh, so the members are the centre and those movable neighbours; the group area
    counts the triangles two members share once (star areas added, shared ones taken off)."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    xy = mesh.xy
    checked = 0
    for c in np.nonzero(mesh.kind == ob.FREE)[0][:200]:
        nb = m.nbr[m.nbr_off[c]:m.nbr_off[c + 1]]
        lens = np.hypot(*(xy[nb] - xy[c]).T)
        d = float(np.sort(lens)[1]) * (1 + 1e-9)  # the two nearest neighbours
        mem = ob.group_members(m, xy, int(c), d)
        want = [int(w) for w, l in zip(nb, lens) if l <= d and mesh.kind[w] != ob.ORIGINAL]
        if mem != [int(c)] + want:  # a vertex closer than a neighbour without an edge to c
            far = set(mem) - set(want) - {int(c)}
            assert far and all(not m.has_edge(int(c), w) for w in far)
            continue
        if len(mem) == 2:
            w = mem[1]
            shared = [t for t in range(m.tri_v.shape[0]) if c in m.tri_v[t] and w in m.tri_v[t]]
            expect = ob.star_area(m, xy, c) + ob.star_area(m, xy, w) - sum(
                ob._tri_area(xy, m.tri_v[t]) for t in shared)
            assert abs(ob.group_area(m, xy, mem) - expect) <= 1e-12 * expect
            checked += 1
    assert checked > 10


def test_lone_centre_is_the_single_vertex_move():
    """A group with no member but its centre makes the move of Sec. 3.2.2: the same position,
    status and acceptance as the single-vertex chain with displacement lam * sqrt(star area) * xi."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    p = ob.Params(1e-9)  # d < every edge: lone centres
    rng = np.random.default_rng(8)
    c = rng.choice(np.nonzero(mesh.kind != ob.ORIGINAL)[0], 40, replace=False)
    xi = rng.standard_normal((40, 2)) * 0.5
    rd, u = rng.random(40), rng.random(40)
    xy_g, st_g, df_g, _, size = ob.group_chain(m, mesh.xy, p, 1e-3, 0.05, c, xi, rd, u)
    assert (size == 1).all()
    xy_s = mesh.xy.copy()
    for i, v in enumerate(c):
        k = 0.05 * math.sqrt(ob.star_area(m, xy_s, int(v)))
        d = np.array([k * xi[i, 0], k * xi[i, 1]])
        xy_s, st, df, _ = ob.metropolis_chain(m, xy_s, p, 1e-3, [int(v)], [d], [u[i]])
        assert st[0] == st_g[i]
        if np.isfinite(df[0]):
            assert abs(df[0] - df_g[i]) <= 1e-9 * (1 + abs(df[0]))
    assert np.array_equal(xy_s, xy_g)


def test_group_moves_rigidly():
    """Free members share one displacement: the edges between them keep their lengths (to
    rounding) when the move is accepted."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    p = ob.Params(0.2)  # d up to 1: whole neighbourhoods
    rng = np.random.default_rng(9)
    seen = 0
    for c in np.nonzero(mesh.kind == ob.FREE)[0][:60]:
        mem, qs = ob.group_move(m, mesh.xy, p, int(c), 0.05, rng.standard_normal(2), 0.9)
        free = [j for j, v in enumerate(mem) if mesh.kind[v] == ob.FREE]
        for j in free:
            for k in free:
                if j < k and m.has_edge(mem[j], mem[k]):
                    before = np.hypot(*(mesh.xy[mem[j]] - mesh.xy[mem[k]]))
                    after = np.hypot(*(qs[j] - qs[k]))
                    assert abs(after - before) <= 1e-12 * (1 + before)
                    seen += 1
    assert seen > 20


def _fan_chain(k, step):
    """Free vertices 0..k-1 on the x axis at spacing `step` (a contracted chain) under an apex of
    original vertices: vertex i joins only its chain neighbours and the apexes above and below,
    so 0 and 2 share no edge. Apexes k (above) and k+1 (below) are ORIGINAL."""
    xy = np.array([[i * step, 0.0] for i in range(k)] + [[0.5 * (k - 1) * step, 5.0],
                                                          [0.5 * (k - 1) * step, -5.0]])
    up, down = k, k + 1
    tv = [[i, i + 1, up] for i in range(k - 1)] + [[i + 1, i, down] for i in range(k - 1)]
    kind = np.array([ob.FREE] * k + [ob.ORIGINAL] * 2)
    m = ob.Mesh(np.array(tv), kind, np.zeros(k + 2, dtype=np.int64),
                np.zeros((0, 2), dtype=np.int64))
    return m, xy


def test_group_of_a_chain_reaches_past_the_neighbours():
    """Sec. 3.2.3 moves every vertex within d of the centre: on a chain of spacing 0.4, the centre
    2 with d = 0.9 takes 0 and 4 (0.8 away, two edges away) besides its neighbours 1 and 3, and not
    5 (1.2 away); the ORIGINAL apexes never belong."""
    m, xy = _fan_chain(9, 0.4)
    assert not m.has_edge(2, 0) and not m.has_edge(2, 4)
    assert ob.group_members(m, xy, 2, 0.9) == [2, 0, 1, 3, 4]
    assert ob.group_members(m, xy, 2, 0.79) == [2, 1, 3]
    assert ob.group_members(m, xy, 8, 1.25) == [8, 5, 6, 7]
    # d just covering the apex distance still leaves the ORIGINAL apexes out
    assert 9 not in ob.group_members(m, xy, 4, 5.5) and len(ob.group_members(m, xy, 4, 5.5)) == 9


def test_group_has_no_size_limit():
    """A centre with twenty movable neighbours within d and ten more free vertices 1.5 away,
    reached by no edge from it: all thirty join, the centre first."""
    n = 20
    ring = [[math.cos(2 * math.pi * k / n), math.sin(2 * math.pi * k / n)] for k in range(n)]
    outer = [[1.5 * math.cos(2 * math.pi * (k + 0.5) / 10), 1.5 * math.sin(2 * math.pi * (k + 0.5) / 10)]
             for k in range(10)]
    xy = np.array([[0.0, 0.0]] + ring + outer)
    tv = [[0, 1 + k, 1 + (k + 1) % n] for k in range(n)]
    # the outer vertices hang off the ring: outer j between ring vertices 2j+1 and 2j+2
    for j in range(10):
        a, b = 1 + (2 * j + 1) % n, 1 + (2 * j + 2) % n
        tv.append([a, 21 + j, b])
    m = ob.Mesh(np.array(tv), np.array([ob.FREE] * 31), np.zeros(31, dtype=np.int64),
                np.zeros((0, 2), dtype=np.int64))
    assert all(not m.has_edge(0, 21 + j) for j in range(10))
    assert ob.group_members(m, xy, 0, 2.0) == list(range(31))
    assert ob.group_members(m, xy, 0, 1.2) == list(range(21))
    assert ob.group_members(m, xy, 25, 0.0) == [25]
