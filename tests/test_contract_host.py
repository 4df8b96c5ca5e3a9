"""The library's contraction (mesh_contract, host code) against the checker (oracle/contract.py):
identical triangles, kinds, lines, positions, vertex maps and counts. CPU only: the entry point
makes no device call."""
import numpy as np
import pytest

import paper_2112_05570_amd as ccsp
import helpers
import scenegen as sg
from oracle import contract as ct
from oracle import objective as ob
from test_oracle_contract import _clustered_mesh, _square


def _same(r, o):
    return (np.array_equal(r["tri_v"], o[0]) and np.array_equal(r["kind"], o[1])
            and np.array_equal(r["line"], o[2]) and np.array_equal(r["xy"], o[3])
            and np.array_equal(r["old_to_new"], o[4]) and r["contracted"] == o[5])


def test_square_cases():
    for k4, k5 in ((ob.FREE, ob.FREE), (ob.ORIGINAL, ob.FREE), (ob.ORIGINAL, ob.ORIGINAL)):
        tv, kind, line, prim_v, xy = _square(k4, k5)
        assert _same(ccsp.contract(tv, kind, line, prim_v, xy, 0.05),
                     ct.contract(tv, kind, line, prim_v, xy, 0.05))


@pytest.mark.parametrize("seed,eps", [(1, 0.02), (2, 0.05), (3, 0.01), (4, 0.1)])
def test_clustered_tiny(seed, eps):
    mesh, xy = _clustered_mesh(seed, eps)
    r = ccsp.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    o = ct.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    assert o[5] > 50 and _same(r, o)


def test_subdivided_mid_scene():
    """An 8,002-triangle scene subdivided (32,008 triangles), vertices jittered by valid moves,
    contracted at a length that catches many of its edges."""
    mesh = helpers.subdivided(sg.make_scene("large", n_seg=2000))
    om = ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)
    rng = np.random.default_rng(7)
    xy = mesh.xy.copy()
    lens = ob.lengths(xy, om.edge_v[:, 0], om.edge_v[:, 1])
    eps = float(np.quantile(lens, 0.03))
    for v in rng.choice(np.nonzero(mesh.kind == ob.FREE)[0], 3000, replace=False):
        nb = om.nbr[om.nbr_off[v]:om.nbr_off[v + 1]]
        q = xy[v] + 0.7 * (xy[nb[rng.integers(0, nb.shape[0])]] - xy[v])
        if ob.move_status(om, xy, int(v), q) == ob.MOVED:
            xy[v] = q
    r = ccsp.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    o = ct.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    assert o[5] > 500 and _same(r, o)


def test_rejects_bad_input():
    tv, kind, line, prim_v, xy = _square()
    with pytest.raises(ccsp.CcspError, match="eps"):
        ccsp.contract(tv, kind, line, prim_v, xy, 0.0)
    with pytest.raises(ccsp.CcspError, match="counter-clockwise"):
        ccsp.contract(tv[:, ::-1], kind, line, prim_v, xy, 0.05)
    bad = kind.copy()
    bad[4] = ob.CONSTRAINED
    with pytest.raises(ccsp.CcspError, match="constrained vertex without edge"):
        ccsp.contract(tv, bad, line, prim_v, xy, 0.05)


def test_walk_arrays_of_a_subdivided_mesh():
    """Every constrained edge of the subdivided tiny scene becomes its own primitive, lying on its
    original one (to rounding of the midpoints); the arrays pass the checker's validator."""
    import oracle
    from paper_2112_05570_amd import pipeline as pl
    sc = sg.make_scene("tiny")
    mesh = helpers.subdivided(sc)
    nbr, prim, prims, s2o = pl.walk_arrays(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy)
    assert prims.shape == (2 * sc.n_prims, 4) and np.bincount(s2o).tolist() == [2] * sc.n_prims
    assert oracle.validate(oracle.Triangulation(mesh.xy, mesh.tri_v, nbr, prim, prims)) == ""
    for j in range(prims.shape[0]):
        a, b = sc.prims[s2o[j], :2], sc.prims[s2o[j], 2:]
        for p in (prims[j, :2], prims[j, 2:]):
            cross = (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
            assert abs(cross) <= 1e-12 * np.hypot(*(b - a)) * (1 + np.abs(p).max())


@pytest.mark.parametrize("seed,eps", [(1, 0.02), (4, 0.1)])
def test_walk_arrays_after_contraction(seed, eps):
    """A clustered mesh contracted by the library still gives valid walk arrays: every
    constrained edge of the result is its own primitive on its original one, and the checker's
    validator accepts the triangulation."""
    import oracle
    from paper_2112_05570_amd import pipeline as pl
    mesh, xy = _clustered_mesh(seed, eps)
    r = ccsp.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy, eps)
    nbr, prim, prims, s2o = pl.walk_arrays(r["tri_v"], r["kind"], r["line"], mesh.prim_v, r["xy"])
    tri = oracle.Triangulation(r["xy"], r["tri_v"], nbr, prim, prims)
    assert oracle.validate(tri) == ""
    # each original primitive is covered by its sub-primitives end to end
    sc = sg.make_scene("tiny")
    for k in range(sc.n_prims):
        sub = prims[s2o == k]
        ends = np.concatenate([sub[:, :2], sub[:, 2:]])
        u, c = np.unique(ends, axis=0, return_counts=True)
        assert (c == 1).sum() == 2  # a chain: only its two ends appear once
    assert pl.weight(r["tri_v"], r["xy"]) < pl.weight(mesh.tri_v, xy)


def test_flat_triangle_case_matches():
    """The hand-built case of a contraction that would leave a triangle flat on an original edge:
    the library refuses it too."""
    xy = np.array([[0, 0], [3, 0], [1, -2.0 ** -60], [0.01, 0.005], [1.5, 1], [1.5, -1]])
    tv = np.array([[0, 2, 3], [2, 1, 3], [0, 3, 4], [3, 1, 4], [0, 5, 2], [2, 5, 1]])
    kind = np.array([0, 0, 1, 2, 0, 0])
    line = np.zeros(6, dtype=np.int64)
    prim_v = np.array([[0, 1]])
    r = ccsp.contract(tv, kind, line, prim_v, xy, 0.05)
    o = ct.contract(tv, kind, line, prim_v, xy, 0.05)
    assert _same(r, o) and r["contracted"] == 0
