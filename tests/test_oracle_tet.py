"""Pins of the 3D walk's checker (oracle3d.c) against the definition and the geometry.

* Hand cases in one tetrahedron: the exit face and t worked out by hand, a ray through a vertex.
* The symbolic move of the line on hand-computed Plücker cases (zero values resolved by the first
  nonzero term of the expansion, antisymmetric).
* The walk equals brute force over every face (first primitive crossed, t, tetrahedra visited)
  on random rays, and on rays through vertices, through edge midpoints, parallel to edges and
  along edge lines wherever brute force has a unique answer.
* The 3D Cauchy-Crofton relation: isotropic uniform random lines through the hull cross the
  interior faces 2 A_int / A(hull) times on average.
* The step guard, invalid rays, point location and the validator catching planted errors.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg


@pytest.fixture(scope="module")
def scene():
    sc = sg.make_tet_scene(2000, seed=0)
    return sc, oracle.TetMesh.of(sc)


def _one_tet():
    xyz = np.array([[0, 0, 0], [8, 0, 0], [0, 8, 0], [0, 0, 8]], np.int32)
    tv = np.array([[0, 1, 2, 3]], np.int32)
    nb = -np.ones((1, 4), np.int32)
    prims = np.array([[tv[0, f[0]], tv[0, f[1]], tv[0, f[2]]] for f in sg.TET_FACES], np.int32)
    return oracle.TetMesh(xyz, tv, nb, np.arange(4, dtype=np.int32)[None], prims)


def test_orient_and_plucker_closed_forms():
    e = np.eye(3, dtype=np.int32)
    assert oracle.orient3([0, 0, 0], 8 * e[0], 8 * e[1], 8 * e[2]) == 512
    assert oracle.orient3([0, 0, 0], 8 * e[1], 8 * e[0], 8 * e[2]) == -512
    # the z axis passes the edge x -> y of the unit triangle anticlockwise seen from +z
    assert oracle.plucker3([0, 0, 0], [0, 0, 1], e[0], e[1]) == 1
    assert oracle.plucker3([0, 0, 0], [0, 0, 1], e[1], e[0]) == -1
    # largest magnitudes on the grid stay exact: (2^19 - 1)^3 for the orientation
    g = (1 << 19) - 1
    assert oracle.orient3([0, 0, 0], [g, 0, 0], [0, g, 0], [0, 0, g]) == g ** 3


def test_symbolic_move_hand_cases():
    z = [0, 0, 0]
    assert oracle.pi3(z, [0, 0, 1], [1, 0, 0], [0, 1, 0]) == (1, False)
    # the ray passes the vertex p: d.W = 0, c = d x (q - p) = (0, 0, 1) -> c_z decides
    assert oracle.pi3(z, [1, 0, 0], [2, 0, 0], [2, 1, 0]) == (1, True)
    assert oracle.pi3(z, [1, 0, 0], [2, 1, 0], [2, 0, 0]) == (-1, True)
    # the ray crosses the edge (3,0,1)-(3,0,-1) at (3,0,0): c = (1,0,0) x (0,0,-2) = (0,2,0)
    assert oracle.pi3(z, [1, 0, 0], [3, 0, 1], [3, 0, -1]) == (1, True)
    # ... and the edge (3,1,0)-(3,-1,0): c = (1,0,0) x (0,-2,0) = (0,0,-2)
    assert oracle.pi3(z, [1, 0, 0], [3, 1, 0], [3, -1, 0]) == (-1, True)
    # parallel edges: c = 0, then W_x, -a_z, a_y, W_y, a_z, -a_x
    assert oracle.pi3(z, [0, 0, 1], [0, 1, 0], [0, 1, 5]) == (1, True)      # W = (5, 0, 0)
    assert oracle.pi3(z, [1, 0, 0], [0, 0, 1], [2, 0, 1]) == (1, True)      # W = (0, 2, 0)
    assert oracle.pi3(z, [1, 0, 0], [0, 1, 0], [3, 1, 0]) == (-1, True)     # W = (0, 0, -3): -a_x
    assert oracle.pi3(z, [1, 0, 0], [3, 1, 0], [0, 1, 0]) == (1, True)
    # the ray along the edge's own line: W = 0, a = (4, 0, 0): -a_x
    assert oracle.pi3(z, [1, 0, 0], [2, 0, 0], [6, 0, 0]) == (-1, True)


def test_one_tetrahedron_by_hand():
    m = _one_tet()
    assert oracle.validate3(m) == ""
    o = np.array([[1, 1, 1]] * 5, np.int32)
    d = np.array([[1, 0, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 1, 1]], np.int32)
    prim, t, steps, dg = oracle.walk3(m, o, d, np.zeros(5, np.int32))
    # +x meets x + y + z = 8 at (6, 1, 1): face 0 (opposite the origin vertex), s = 5; the
    # coordinate planes at s = 1; (1,1,1) + s (1,1,1) meets the slanted face at s = 5/3
    assert prim.tolist() == [0, 1, 2, 3, 0]
    assert t.tolist() == [5.0, 1.0, 1.0, 1.0, 5.0 / 3.0]
    assert steps.tolist() == [1] * 5
    # -z runs parallel to the edge (0,0,0)-(0,0,8), which the search meets on face 1: a zero value
    # resolved by the moved line; the other rays decide every sign they take without one
    assert dg.tolist() == [0, 0, 0, 1, 0]
    # through the vertex (8, 0, 0) at s = 1: any of the three faces holding it, at t = 1 exactly
    prim, t, steps, dg = oracle.walk3(m, [[1, 1, 1]], [[7, -1, -1]], [0])
    assert prim[0] in (0, 2, 3) and t[0] == 1.0 and dg[0] == 1


def test_walk_equals_brute_force(scene):
    sc, m = scene
    for seed in (1, 2):
        r = sg.sample_rays3(sc, 3000, seed)
        w = oracle.walk3(m, r.o, r.d, r.start)
        b = oracle.brute3(m, r.o, r.d)
        ok = b[3] == 0
        assert ok.mean() > 0.99
        for k, name in enumerate(("prim", "t", "steps")):
            bad = np.nonzero((w[k] != b[k]) & ok)[0]
            assert bad.size == 0, f"{name} differs at {bad[:5]}"
        assert (w[0] >= 0).all() and w[2].max() > 10


def _degenerate_rays(sc, rng, n):
    """Rays that meet vertices or edges exactly. Vertices are taken among those on no primitive,
    so that brute force's hit stays unique: a ray touching a primitive's vertex before its first
    proper crossing has a hit that depends on the tie rule."""
    P = sc.xyz.astype(np.int64)
    free = np.ones(sc.n_vertices, bool)
    free[sc.prims.ravel()] = False
    base = sg.sample_rays3(sc, 4 * n, 11)
    o = base.o.astype(np.int64)
    E = sc.tet_v[rng.integers(0, sc.n_tets, 16 * n)][:, :2].astype(np.int64)
    Ef = E[free[E[:, 0]] & free[E[:, 1]]][:4 * n]
    V = rng.choice(np.nonzero(free)[0], 4 * n)
    p, q = P[Ef[:, 0]], P[Ef[:, 1]]
    m = min(Ef.shape[0], 4 * n)
    kinds = {
        "vertex": (o, P[V] - o, base.start),
        "midpoint": (o[:m], (p + q - 2 * o[:m]), base.start[:m]),
        "parallel": (o, P[E[:4 * n, 1]] - P[E[:4 * n, 0]], base.start),
    }
    # along an edge's line: start at 2p - q where that point is inside a tetrahedron
    a = 2 * p - q
    inside = ((a >= 0) & (a < sg.GRID3)).all(axis=1)
    kinds["edge line"] = (a[inside], (q - p)[inside], None)
    out = {}
    for name, (oo, dd, st) in kinds.items():
        keep = (np.abs(dd) <= sg.GRID3).all(axis=1) & (dd != 0).any(axis=1)
        oo, dd = oo[keep][:n], dd[keep][:n]
        if st is None:
            tt, s = oracle.locate3(oracle.TetMesh.of(sc), oo)
            good = s == 0
            oo, dd, st = oo[good], dd[good], tt[good]
        else:
            st = st[keep][:n]
        out[name] = (oo.astype(np.int32), dd.astype(np.int32), st.astype(np.int32))
    return out


def test_degenerate_rays_follow_a_moved_line():
    """Rays through vertices, edge midpoints, parallel to edges and along edge lines: the walk
    never fails (no -2, -3), and where brute force's hit does not depend on ties the hit and t are
    the same (the count too where it does not either)."""
    sc = sg.make_tet_scene(2000, seed=0, frac_prims=0.02)
    m = oracle.TetMesh.of(sc)
    rng = np.random.default_rng(5)
    for name, (o, d, st) in _degenerate_rays(sc, rng, 600).items():
        assert o.shape[0] >= 50, name
        w = oracle.walk3(m, o, d, st)
        b = oracle.brute3(m, o, d)
        assert (w[0] >= 0).all(), f"{name}: codes {np.unique(w[0])}"
        ok = (b[3] & 1) == 0
        assert ok.mean() > 0.5, (name, ok.mean())
        for k, what in enumerate(("prim", "t")):
            bad = np.nonzero((w[k] != b[k]) & ok)[0]
            assert bad.size == 0, f"{name}: {what} differs at {bad[:5]}"
        # rays whose walk passes the vertex or edge (at s = 1, 1/2, 1) decided a zero by the rule
        s0 = {"vertex": 1.0, "midpoint": 0.5, "edge line": 1.0}.get(name)
        if s0 is not None:
            past = b[1] > s0
            assert past.sum() > 100 and w[3][past].all(), name
        ok2 = b[3] == 0
        assert np.array_equal(w[2][ok2], b[2][ok2]), name


def _areas(sc, interior):
    P = sc.xyz.astype(np.float64)
    t_idx, i_idx = np.nonzero((sc.tet_nbr > np.arange(sc.n_tets)[:, None]) if interior
                              else (sc.tet_nbr < 0))
    F = np.array(sg.TET_FACES)[i_idx]
    v = [P[sc.tet_v[t_idx, F[:, k]]] for k in range(3)]
    n = np.cross(v[1] - v[0], v[2] - v[0])
    return 0.5 * np.linalg.norm(n, axis=1), n, v[0]


def test_crofton_3d():
    """Isotropic uniform random lines meeting the hull K cross a surface S inside it
    2 A(S) / A(boundary of K) times on average (Cauchy-Crofton; S = boundary gives 2). With only
    hull faces as primitives, a line through an interior grid point crosses (steps(+d) - 1) +
    (steps(-d) - 1) interior faces."""
    sc = sg.make_tet_scene(1500, seed=3, frac_prims=0.0)
    m = oracle.TetMesh.of(sc)
    a_int = _areas(sc, True)[0].sum()
    a_hull, n_hull, p_hull = _areas(sc, False)
    rng = np.random.default_rng(17)
    P = sc.xyz.astype(np.float64)
    c = 0.5 * (P.min(0) + P.max(0))
    R = 0.5 * np.linalg.norm(P.max(0) - P.min(0)) * 1.01
    N = 24_000
    g = rng.standard_normal((N, 3))
    u = g / np.linalg.norm(g, axis=1, keepdims=True)
    h = np.where(np.abs(u[:, :1]) < 0.9, [[1.0, 0, 0]], [[0, 1.0, 0]])
    e1 = np.cross(u, h)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(u, e1)
    r = R * np.sqrt(rng.random(N))
    th = 2 * np.pi * rng.random(N)
    x = c + r[:, None] * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
    # the chord inside K: n.(x + s u - p) <= 0 for every outward hull face normal n
    nu = u @ n_hull.T
    rhs = ((p_hull[None] - x[:, None]) * n_hull[None]).sum(-1)
    s_hi = np.where(nu > 0, rhs / np.where(nu > 0, nu, 1), np.inf).min(1)
    s_lo = np.where(nu < 0, rhs / np.where(nu < 0, nu, 1), -np.inf).max(1)
    hit = s_hi > s_lo + 1e-6 * R
    o = np.rint(x + (0.5 * (s_lo + s_hi))[:, None] * u)[hit].astype(np.int32)
    d = np.rint(u * (sg.GRID3 - 1))[hit].astype(np.int32)
    st, status = oracle.locate3(m, o)
    good = status == 0
    o, d, st = o[good], d[good], st[good]
    assert o.shape[0] > 0.9 * hit.sum() and hit.mean() > 0.4
    fwd = oracle.walk3(m, o, d, st)
    bwd = oracle.walk3(m, o, -d, st)
    assert (fwd[0] >= 0).all() and (bwd[0] >= 0).all()
    k = (fwd[2] - 1) + (bwd[2] - 1)
    expect = 2.0 * a_int / a_hull.sum()
    se = k.std() / np.sqrt(k.size)
    assert abs(k.mean() - expect) < 4 * se, (k.mean(), expect, se)
    assert se < 0.01 * expect


def test_guard_and_invalid_rays(scene):
    sc, m = scene
    r = sg.sample_rays3(sc, 2000, 4)
    full = oracle.walk3(m, r.o, r.d, r.start)
    lim = oracle.walk3(m, r.o, r.d, r.start, max_steps=5)
    long_ = full[2] > 5
    assert long_.sum() > 100
    assert (lim[0][long_] == -2).all() and (lim[2][long_] == 5).all()
    assert np.isinf(lim[1][long_]).all()
    for k in range(3):
        assert np.array_equal(lim[k][~long_], full[k][~long_])
    # zero direction, start out of range, origin on a face or outside its start
    tv = sc.tet_v[r.start[0]]
    vtx = sc.xyz[tv[0]]
    o = np.array([r.o[0], r.o[0], vtx, r.o[1]], np.int32)
    d = np.array([[0, 0, 0], r.d[0], r.d[0], r.d[1]], np.int32)
    st = np.array([r.start[0], sc.n_tets, r.start[0], (r.start[1] + 1) % sc.n_tets], np.int32)
    p, t, s, _ = oracle.walk3(m, o, d, st)
    assert p.tolist() == [-3, -3, -3, -3] and s.tolist() == [0, 0, 0, 0]


def test_locate3(scene):
    sc, m = scene
    P = sc.xyz.astype(np.int64)
    # centroids (x4, then halved twice with rounding) sit strictly inside their tetrahedron for
    # all but the flattest ones; vertices lie on boundaries
    cen = np.rint(P[sc.tet_v[:500]].mean(1)).astype(np.int32)
    tt, st = oracle.locate3(m, cen)
    inside = st == 0
    assert inside.mean() > 0.9
    assert np.array_equal(tt[inside], np.arange(500)[inside])
    tt, st = oracle.locate3(m, sc.xyz[:50])
    assert (st == 1).all()
    tt, st = oracle.locate3(m, [[-1, 0, 0]])
    assert st[0] == -1


def test_validator_catches_planted_errors(scene):
    sc, _ = scene
    assert oracle.validate3(oracle.TetMesh.of(sg.make_tet_scene(800, seed=1, open_hull=True))) == ""
    def broken(edit):
        tv, nb, tp, pr = sc.tet_v.copy(), sc.tet_nbr.copy(), sc.tet_prim.copy(), sc.prims.copy()
        edit(tv, nb, tp, pr)
        return oracle.validate3(oracle.TetMesh(sc.xyz, tv, nb, tp, pr))
    def swap(tv, nb, tp, pr):
        tv[7, [0, 1]] = tv[7, [1, 0]]
    def nbr(tv, nb, tp, pr):
        i = int(np.nonzero(nb[9] >= 0)[0][0])
        nb[9, i] = (nb[9, i] + 1) % sc.n_tets
    def prim(tv, nb, tp, pr):
        t, i = np.argwhere((tp >= 0) & (nb >= 0))[0]
        tp[t, i] = -1
    def drop(tv, nb, tp, pr):
        t, i = np.argwhere(nb >= 0)[0]
        nb[t, i] = -1
    assert "oriented" in broken(swap)
    assert broken(nbr) != ""
    assert "primitive" in broken(prim)
    assert broken(drop) != ""
