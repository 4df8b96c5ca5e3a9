"""Pins of the objective checker (oracle/objective.py) against the paper's worked examples,
closed forms and properties of f; CPU only."""
import math

import numpy as np
import pytest

import oracle
import helpers
import scenegen as sg
from oracle import objective as ob


def _ccw(xy, tris):
    out = []
    for t in tris:
        a, b, c = (xy[k] for k in t)
        s = oracle.orient(a, b, c)
        assert s != 0
        out.append(t if s > 0 else (t[0], t[2], t[1]))
    return np.array(out)


def _edge(m, a, b):
    return int(np.nonzero((m.edge_v[:, 0] == min(a, b)) & (m.edge_v[:, 1] == max(a, b)))[0][0])


SQUARE = np.array([[-1.0, 1.0], [1.0, 1.0], [-1.0, -1.0], [1.0, -1.0]])  # TL, TR, BL, BR
CENTRE = np.array([-0.05, 0.1])
TL, TR, BL, BR = range(4)
BOX = np.array([[TL, TR], [TR, BR], [BR, BL], [BL, TL]])


def _shrunk(pts, s):
    """The figure's inner vertices pulled towards its centre vertex by the factor s."""
    return CENTRE + s * (np.asarray(pts) - CENTRE)


def _figure_one_contracted(s):
    """The contraction figure of Sec. 2.2.1, panel with one contracted edge (U-D)."""
    U, D = 4, 5
    xy = np.concatenate([SQUARE, _shrunk([[0.05, 0.2], [-0.15, 0.0]], s)])
    tris = _ccw(xy, [(TL, TR, U), (TR, BR, U), (U, BR, D), (BR, BL, D), (BL, TL, D), (TL, U, D)])
    return ob.Mesh(tris, [0, 0, 0, 0, 2, 2], [-1] * 6, BOX), xy


def _figure_three_contracted(s):
    """Same figure, panel with three contracted edges (triangle U-D-X) and the red edge TL-X."""
    U, D, X = 4, 5, 6
    xy = np.concatenate([SQUARE, _shrunk([[0.15, 0.2], [-0.15, -0.1], [-0.15, 0.2]], s)])
    tris = _ccw(xy, [(TL, TR, U), (TR, BR, U), (U, BR, D), (BR, BL, D), (BL, TL, D),
                     (TL, D, X), (TL, X, U), (X, D, U)])
    return ob.Mesh(tris, [0, 0, 0, 0, 2, 2, 2], [-1] * 7, BOX), xy


def test_figure_single_contracted_edge_weights():
    """The merged edge pairs weigh 1/2, the rest 1; the fuzzy weight tends to the length of the
    contracted state (square plus four spokes to the merged vertex) as the cluster shrinks."""
    eps = 0.1
    contracted = 8.0 + np.linalg.norm(SQUARE - CENTRE, axis=1).sum()
    prev = None
    for s in (1e-3, 1e-5, 1e-7):
        m, xy = _figure_one_contracted(s)
        r = ob.objective(m, xy, ob.Params(eps))
        half = [_edge(m, TL, 4), _edge(m, TL, 5), _edge(m, BR, 4), _edge(m, BR, 5)]
        tol = 4 * s / eps
        assert np.allclose(r["w"][half], 0.5, atol=tol, rtol=0)
        rest = np.setdiff1d(np.arange(m.n_edges), half)
        assert np.allclose(r["w"][rest], 1.0, atol=tol, rtol=0)
        err = abs(r["wcontr"] - contracted)
        assert err < 10 * s
        if prev is not None:
            assert err < prev
        prev = err


def test_figure_three_contracted_edges_weights():
    """Merged pairs weigh 1/2, the doubly merged red edge 0, the contracted edges themselves 0,
    with the three inner edges contracted as the figure has them. On its own, U-D is
    incontractible under the 1-hop rule (TL is a nontrivial 1-hop vertex far from both of its
    opposite vertices): the figure shows a cluster, which the rule does not look at."""
    eps = 0.1
    s = 1e-6
    m, xy = _figure_three_contracted(s)
    U, D, X = 4, 5, 6
    inner = [_edge(m, U, D), _edge(m, D, X), _edge(m, X, U)]
    ln = ob.lengths(xy, m.edge_v[:, 0], m.edge_v[:, 1])
    contr = np.zeros(m.n_edges, dtype=bool)
    contr[inner] = True
    w = ob.edge_weight(m, ob.c_eps(ln, contr, eps))
    tol = 8 * s / eps
    for a, b in ((TL, U), (TL, D)):
        assert abs(w[_edge(m, a, b)] - 0.5) < tol
    assert w[_edge(m, TL, X)] < tol
    assert (w[inner] < tol).all()
    c = ob.contractible(m, xy, eps)
    assert not c[_edge(m, U, D)] and c[_edge(m, D, X)] and c[_edge(m, X, U)]


def test_figure_one_hop_rule():
    """The 1-hop figure of Sec. 2.2.2: V1V2 has the nontrivial 1-hop vertex H and is contractible
    exactly when ||V3 H|| < eps."""
    V1, V2, H, V3 = range(4)
    xy = np.array([[-0.8, 1.1], [-1.3, 0.0], [2.0, 0.0], [1.0, 0.27]])
    m = ob.Mesh(_ccw(xy, [(V1, V2, V3), (V1, V3, H), (V2, H, V3)]), [2] * 4, [-1] * 4,
                np.zeros((0, 2), int))
    d = math.sqrt(1.0 + 0.27 ** 2)
    e = _edge(m, V1, V2)
    assert not ob.contractible(m, xy, np.nextafter(d, 0))[e]
    assert not ob.contractible(m, xy, 1.0)[e]
    assert ob.contractible(m, xy, np.nextafter(d, 2))[e]
    assert ob.contractible(m, xy, 1.1)[e]
    # edges V3-x have no nontrivial 1-hop vertex: contractible at any eps
    for x in (V1, V2, H):
        assert ob.contractible(m, xy, 1e-9)[_edge(m, V3, x)]


def test_direct_restrictions():
    """Sec. 2.2.2, restrictions from the original geometry, one case per rule on a fan."""
    # original edges: 0 = (0,1), 1 = (2,3); vertex 4 on edge 0, 5 and 6 on edge 1, 7 free
    xy = np.array([[0.0, 0.0], [4.0, 0.0], [4.0, 4.0], [0.0, 4.0], [2.0, 0.0], [4.0, 2.0],
                   [1.0, 4.0], [2.0, 2.0]])
    kind = [0, 0, 0, 0, 1, 1, 1, 2]
    line = [-1, -1, -1, -1, 0, 1, 1, -1]
    prim_v = [[0, 1], [2, 3]]
    tris = _ccw(xy, [(0, 4, 7), (4, 1, 7), (1, 5, 7), (5, 2, 7), (2, 6, 7), (6, 3, 7), (3, 0, 7)])
    m = ob.Mesh(tris, kind, line, prim_v)
    ok = ob.direct_contractible(m)
    want = {(0, 4): True,    # original end of the constrained vertex's own edge
            (1, 4): True,
            (1, 5): False,   # original vertex not ending edge 1
            (2, 5): True,
            (2, 6): True,
            (3, 6): True,
            (0, 3): False,   # two original vertices
            (5, 7): True, (0, 7): True}  # free vertex: no restriction
    for (a, b), w in want.items():
        assert ok[_edge(m, a, b)] == w, (a, b)
    # two constrained vertices: same original edge yes, different edges no
    kind2 = [0, 0, 0, 0, 1, 1, 1, 1]
    line2 = [-1, -1, -1, -1, 0, 1, 1, 1]
    ok2 = ob.direct_contractible(ob.Mesh(tris, kind2, line2, prim_v))
    assert ok2[_edge(m, 5, 7)] and ok2[_edge(m, 6, 7)] and not ok2[_edge(m, 4, 7)]


def _one_triangle(xy):
    return ob.Mesh(_ccw(xy, [(0, 1, 2)]), [2, 2, 2], [-1] * 3, np.zeros((0, 2), int))


@pytest.mark.parametrize("deg", [179.2, 179.5, 179.9])
def test_angle_penalty_closed_form(deg):
    """A corner of deg degrees costs (cos(180 - deg) - cos 1)/(1 - cos 1) with delta = cos 179 + 1;
    in polishing, a corner of 180 - deg degrees costs the same."""
    th = math.radians(180.0 - deg)
    want = (math.cos(th) - math.cos(math.radians(1.0))) / (1.0 - math.cos(math.radians(1.0)))
    # obtuse corner at vertex 0: edges to 1 and 2 at angle deg
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [math.cos(math.radians(deg)), math.sin(math.radians(deg))]])
    a = ob.angle_terms(_one_triangle(xy), xy, ob.Params(0.1))
    assert abs(a.sum() - want) < 1e-8
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [math.cos(th), math.sin(th)]])
    a = ob.angle_terms(_one_triangle(xy), xy, ob.Params(0.1, polish=True))
    assert abs(a.sum() - want) < 1e-8
    # a right triangle costs nothing in either mode
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    for pol in (False, True):
        assert ob.angle_terms(_one_triangle(xy), xy, ob.Params(0.1, polish=pol)).sum() == 0.0


def test_length_penalty_and_total():
    """An edge of a quarter of eps0 costs 3/4; f adds the parts with their weights."""
    e0 = 1e-3
    xy = np.array([[0.0, 0.0], [e0 / 4, 0.0], [0.0, 1.0]])
    m = _one_triangle(xy)
    p = ob.Params(1e-300, eps0=e0, mu_angle=2.0, mu_len=10.0)
    r = ob.objective(m, xy, p)
    assert abs(r["plen"] - 0.75) < 1e-12
    assert r["f"] == r["wcontr"] + 2.0 * r["pangle"] + 10.0 * r["plen"]


def test_vanishing_eps_is_plain_weight():
    """As eps -> 0 every edge weighs 1: w_contr is the triangulation's weight."""
    sc = sg.make_scene("tiny")
    mesh = helpers.subdivided(sc)
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    r = ob.objective(m, mesh.xy, ob.Params(1e-300))
    assert (r["w"] == 1.0).all()
    ln = r["length"]
    assert abs(r["wcontr"] - ln.sum()) <= 1e-12 * ln.sum()
    # subdivision keeps the original edges' total length on its halves (each triangle's medial
    # triangle adds half the perimeter): weight(sub) = weight(cdt) + 1/2 sum of triangle perimeters
    per = sum(np.linalg.norm(sc.xy[sc.tri_v[:, (i + 1) % 3]] - sc.xy[sc.tri_v[:, (i + 2) % 3]],
                             axis=1).sum() for i in range(3))
    assert abs(r["wcontr"] - (sg.weight(sc) + 0.5 * per)) < 1e-9 * r["wcontr"]
    # polishing ignores eps
    rp = ob.objective(m, mesh.xy, ob.Params(1e3, polish=True))
    assert rp["wcontr"] == r["wcontr"]


def test_large_eps_halves_contractible_edges():
    """With eps beyond every length, contractible edges have c -> 1/2 as |e|/eps -> 0; an edge
    whose neighbours are all contractible weighs x M(x) for x = 1/16 (two triangles) = 0."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    r = ob.objective(m, mesh.xy, ob.Params(1e12))
    assert np.allclose(r["c"][r["contractible"]], 0.5, atol=1e-11)
    n = m.edge_nbr
    all_c = (n[:, 2] >= 0) & r["contractible"][n].all(axis=1)
    assert all_c.any() and (r["w"][all_c] == 0.0).all()


def _moves(mesh, n, seed, lam):
    v, q = sg.vertex_moves(mesh, n, seed, lam)
    return v, q


def test_delta_properties():
    """Null moves change nothing; moving back undoes a move; a chain of accepted moves adds up to
    the change of f; folding, fixed and malformed moves are flagged."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    p = ob.Params(0.02)
    xy = mesh.xy.copy()
    f0 = ob.objective(m, xy, p)["f"]
    v, q = _moves(mesh, 60, 1, 0.05)
    assert ob.delta_f(m, xy, p, v[0], xy[v[0]]) == (1, 0.0, 0.0)
    total, scale, n_ok = 0.0, 0.0, 0
    for k in range(v.shape[0]):
        st, df, b = ob.delta_f(m, xy, p, v[k], q[k])
        if st != 1:
            assert df == math.inf
            continue
        old = xy[v[k]].copy()
        xy[v[k]] = q[k]
        st2, back, b2 = ob.delta_f(m, xy, p, v[k], old)
        assert st2 == 1 and abs(back + df) <= 1e-12 * (b + b2)
        total += df
        scale += b
        n_ok += 1
    assert n_ok > 10
    f1 = ob.objective(m, xy, p)["f"]
    assert abs((f1 - f0) - total) <= 1e-12 * (scale + abs(f0) * len(m.edge_v))
    fixed = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
    assert ob.delta_f(m, xy, p, fixed, xy[fixed] + 1e-3)[0] == ob.FIXED
    free = int(np.nonzero(mesh.kind == sg.FREE)[0][0])
    assert ob.delta_f(m, xy, p, free, [np.nan, 0.0])[0] == ob.BAD
    assert ob.delta_f(m, xy, p, m.nv, [0.0, 0.0])[0] == ob.BAD
    # across a far vertex of its star: some triangle folds
    star = m.tri_v[(m.tri_v == free).any(axis=1)]
    far = max((w for w in star.ravel() if w != free),
              key=lambda w: np.linalg.norm(xy[w] - xy[free]))
    beyond = xy[free] + 2.0 * (xy[far] - xy[free])
    assert ob.delta_f(m, xy, p, free, beyond)[0] == ob.FOLDED


def test_metropolis_chain_properties():
    """T = 0 accepts exactly the moves that do not increase f, so f never rises and the accepted
    changes add up to the change of f; a huge T accepts every valid move; constrained vertices stay
    on their original edges."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    p = ob.Params(0.03)
    rng = np.random.default_rng(4)
    vid = rng.choice(np.nonzero(mesh.kind != sg.ORIGINAL)[0], 150)
    disp = sg.vertex_displacements(mesh, vid, 2, 0.05)
    u = rng.random(150)
    f0 = ob.objective(m, mesh.xy, p)["f"]
    xy, st, df, _ = ob.metropolis_chain(m, mesh.xy, p, 0.0, vid, disp, u)
    acc = st == ob.ACCEPTED
    assert acc.any() and (st == ob.REJECTED).any()
    assert (df[acc] <= 0).all() and (df[st == ob.REJECTED] > 0).all()
    f1 = ob.objective(m, xy, p)["f"]
    assert f1 <= f0 and abs((f1 - f0) - df[acc].sum()) <= 1e-12 * f0 * m.n_edges
    _, st_hot, _, _ = ob.metropolis_chain(m, mesh.xy, p, 1e300, vid, disp, u)
    assert ((st_hot == ob.ACCEPTED) | (st_hot == ob.FOLDED)).all()
    con = mesh.kind == sg.CONSTRAINED
    a, b = mesh.xy[mesh.prim_v[mesh.line[con]]].transpose(1, 0, 2)
    c = xy[con]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    assert (np.abs(cross) <= 1e-12 * (np.abs(b - a).sum(1) * (np.abs(c - a).sum(1) + 1))).all()


def test_edge_values_one_by_one_equal_whole_evaluation():
    """The per-edge evaluation used to sample large meshes equals the whole-mesh evaluation, on a
    clustered state where contractions, merges and the 1-hop rule all occur."""
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    m = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    rng = np.random.default_rng(9)
    xy = mesh.xy.copy()
    for v in rng.choice(np.nonzero(mesh.kind == sg.FREE)[0], 300):
        nb = m.nbr[m.nbr_off[v]:m.nbr_off[v + 1]]
        q = xy[nb[rng.integers(0, nb.shape[0])]] + 0.005 * (rng.random(2) - 0.5)
        if ob.move_status(m, xy, int(v), q) == ob.MOVED:
            xy[v] = q
    for p in (ob.Params(0.03), ob.Params(0.03, polish=True)):
        ref = ob.objective(m, xy, p)
        edges = np.arange(m.n_edges)
        k, c, w = ob.edge_values(m, xy, p, edges)
        assert np.array_equal(k, ref["contractible"]) and np.array_equal(c, ref["c"])
        assert np.array_equal(w, ref["w"])
    assert (ref["w"] == 1.0).all() and (~ref["contractible"]).any()


# ---- Sec. 2.2.2: the flat-triangle and conditioning restrictions, on hand-built meshes

def _fan_over_line(xs, f=(1.0, 3.0), end=10.0):
    """The paper's figure of the flat-triangle rule: an original edge from C0 = (0, 0) to
    CN = (end, 0), CONSTRAINED vertices at x = xs on it, and a FREE vertex F above fanned over all
    of them. Vertex ids: C0 0, CN 1, the constrained ones 2.., F last."""
    cs = [[x, 0.0] for x in xs]
    xy = np.array([[0.0, 0.0], [end, 0.0]] + cs + [list(f)])
    F = xy.shape[0] - 1
    line_v = [0] + list(range(2, 2 + len(xs))) + [1]
    tv = [[line_v[i], line_v[i + 1], F] for i in range(len(line_v) - 1)]
    kind = np.array([ob.ORIGINAL, ob.ORIGINAL] + [ob.CONSTRAINED] * len(xs) + [ob.FREE])
    line = np.zeros(xy.shape[0], dtype=np.int64)
    m = ob.Mesh(np.array(tv), kind, line, np.array([[0, 1]]))
    return m, xy, F


def _contractible_edge(m, xy, a, b, eps):
    e = int(np.nonzero((m.edge_v[:, 0] == min(a, b)) & (m.edge_v[:, 1] == max(a, b)))[0][0])
    return bool(ob.contractible(m, xy, eps)[e]), bool(ob.edge_values(m, xy, ob.Params(eps), [e])[0][0])


def test_flat_triangle_rule_as_in_the_figure():
    """Snapping F onto C0 flattens F's triangles over the original edge; the trapped vertices
    C1..C4 must already be contracted (edges shorter than eps along the edge) to C0 or to CN.
    With one gap longer than eps the edge F-C0 is contractible, as the figure states; with two
    gaps it is not (C3 reaches neither end); with every gap short it is."""
    eps = 0.5
    m, xy, F = _fan_over_line([0.3, 0.6, 9.4, 9.7])  # gaps 0.3 0.3 8.8 0.3 0.3
    assert _contractible_edge(m, xy, F, 0, eps) == (True, True)
    m, xy, F = _fan_over_line([0.3, 0.6, 8.0, 9.7])  # gaps 0.3 0.3 7.4 1.7 0.3: C3 is stuck
    assert _contractible_edge(m, xy, F, 0, eps) == (False, False)
    assert _contractible_edge(m, xy, F, 0, 2.0) == (True, True)  # 1.7 < eps: C3 reaches CN
    # the rule does not concern an edge between F and a vertex off the line's fan, nor two free
    # vertices: with F's contraction onto C1 the trapped C2..C4 must reach C1 or an end
    m, xy, F = _fan_over_line([0.3, 0.6, 9.4, 9.7])
    assert _contractible_edge(m, xy, F, 2, eps) == (True, True)
    m, xy, F = _fan_over_line([2.0, 4.0, 6.0, 8.0])  # every gap 2
    assert _contractible_edge(m, xy, F, 0, eps) == (False, False)
    assert _contractible_edge(m, xy, F, 0, 2.5) == (True, True)


def test_conditioning_rule():
    """Snapping a vertex onto a less free one must not force a badly conditioned triangle: three
    ORIGINAL vertices near-collinear (16 * area / perimeter^2 = 0.0005 < 0.01) forbid it, a
    well-shaped triple (0.23) does not; two ORIGINAL and a CONSTRAINED vertex forbid it only if
    the constrained vertex is near-collinear at both ends and the middle of its original edge."""
    # F = 3 free, O1 = 0, O2 = 1, O3 = 2 original; F's triangle (F, O2, O3) becomes (O1, O2, O3)
    for o3, bad in (((20.0, 0.01), True), ((20.0, 5.0), False)):
        xy = np.array([[0.0, 0.0], [10.0, 0.0], list(o3), [5.0, -3.0]])
        tv = np.array([[0, 1, 3], [3, 1, 2]]) if ob.orient(xy[3], xy[1], xy[2]) > 0 else \
            np.array([[0, 1, 3], [3, 2, 1]])
        if ob.orient(*xy[tv[0]]) < 0:
            tv[0] = tv[0][[0, 2, 1]]
        m = ob.Mesh(tv, np.array([ob.ORIGINAL] * 3 + [ob.FREE]), np.zeros(4, dtype=np.int64),
                    np.array([[0, 1], [1, 2]]))
        assert ob.near_collinear(xy[0], xy[1], xy[2]) == bad
        assert ob.conditioning_ok(m, xy, 3, 0) == (not bad)
    # two ORIGINAL (0, 1) and a CONSTRAINED S (4) on the original edge 2-3
    for b3, bad in (((30.0, 0.0), True), ((30.0, 20.0), False)):
        xy = np.array([[0.0, 0.0], [10.0, 0.0], [20.0, 0.0], list(b3), [25.0, b3[1] / 2], [5.0, -3.0]])
        tv = np.array([[0, 1, 5], [5, 1, 4]])
        for t in range(2):
            if ob.orient(*xy[tv[t]]) < 0:
                tv[t] = tv[t][[0, 2, 1]]
        kind = np.array([ob.ORIGINAL] * 4 + [ob.CONSTRAINED, ob.FREE])
        line = np.array([0, 0, 0, 0, 1, 0])
        m = ob.Mesh(tv, kind, line, np.array([[0, 1], [2, 3]]))
        assert ob.conditioning_ok(m, xy, 5, 0) == (not bad)
