"""GPU edge-flip annealing (flip_anneal) against the checker in oracle/flips.py.

A run is fixed by its seed and temperatures, so the GPU's triangulation (tri_v, tri_nbr, tri_prim)
and its flips per round must equal the checker's exactly. Both sides decide acceptance in binary64
from the same correctly rounded lengths and quotient; only exp differs (neither side's is
correctly rounded), which could change a decision only if the uniform fell within an ulp or so of
exp(-change / T), about 1e-16 per decision, and these seeds do not.
At the grid workload's size (522k triangles) the result is checked by properties: a valid
triangulation with the same constraints, lower weight, no improving flip left after the cold
rounds, the same hits and distances for the walk with fewer steps, and identical repeated runs.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import flips as fl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


def _temps(sc, hot, cold, t0=2e-2, t1=1e-4):
    side = sc.box[1] - sc.box[0]
    return list(side * np.geomspace(t0, t1, hot)) + [0.0] * cold


def _gpu(ccsp, sc, temps, seed):
    xy = torch.from_numpy(np.ascontiguousarray(sc.xy)).to(DEV)
    arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)
            for a in (sc.tri_v, sc.tri_nbr, sc.tri_prim)]
    counts = ccsp.flip_anneal(xy, *arrs, temps, seed)
    return [a.cpu().numpy() for a in arrs], counts


@pytest.mark.parametrize("name,kw,hot,cold,seed", [
    ("tiny", {}, 12, 20, 3), ("tiny", {}, 12, 20, 11), ("tiny", {}, 0, 8, 0),
    ("large", dict(n_seg=2000), 6, 4, 5), ("large", dict(n_seg=2000, seed=2), 0, 6, 9)])
def test_matches_checker(ccsp, name, kw, hot, cold, seed):
    sc = sg.make_scene(name, **kw)
    temps = _temps(sc, hot, cold)
    (tv, nbr, prim), counts = _gpu(ccsp, sc, temps, seed)
    rv, rn, rp, rc = fl.anneal(sc.xy, sc.tri_v, sc.tri_nbr, sc.tri_prim, temps, seed)
    assert list(counts) == list(rc), f"{name} seed {seed}: flips per round"
    assert sum(rc) > 0
    assert np.array_equal(tv, rv) and np.array_equal(nbr, rn) and np.array_equal(prim, rp)


def test_no_rounds_and_converged_input(ccsp):
    """Zero rounds change nothing; cold rounds on a converged triangulation flip nothing."""
    sc = sg.make_scene("tiny")
    (tv, nbr, prim), counts = _gpu(ccsp, sc, [], 1)
    assert counts.shape == (0,) and np.array_equal(tv, sc.tri_v) and np.array_equal(nbr, sc.tri_nbr)
    (tv, nbr, prim), counts = _gpu(ccsp, sc, [0.0] * 30, 1)
    assert counts[-1] == 0
    conv = sc.copy_with(tv, nbr, prim)
    (tv2, nbr2, prim2), counts = _gpu(ccsp, conv, [0.0] * 3, 77)
    assert list(counts) == [0, 0, 0]
    assert np.array_equal(tv2, tv) and np.array_equal(nbr2, nbr) and np.array_equal(prim2, prim)


def test_bad_arguments(ccsp):
    sc = sg.make_scene("tiny")
    xy = torch.from_numpy(np.ascontiguousarray(sc.xy)).to(DEV)
    arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)
            for a in (sc.tri_v, sc.tri_nbr, sc.tri_prim)]
    with pytest.raises(RuntimeError, match="temperatures"):
        ccsp.flip_anneal(xy, *arrs, [1.0, -1.0], 0)
    with pytest.raises(RuntimeError, match="temperatures"):
        ccsp.flip_anneal(xy, *arrs, [float("nan")], 0)
    with pytest.raises(ValueError):
        ccsp.flip_anneal(xy, arrs[0].long(), arrs[1], arrs[2], [0.0], 0)
    assert np.array_equal(arrs[0].cpu().numpy(), sc.tri_v)


def _orient_signs(xy, a, b, c):
    """Exact orientation signs: a binary64 filter, the checker's exact predicate where it is
    inconclusive."""
    l = (xy[b, 0] - xy[a, 0]) * (xy[c, 1] - xy[a, 1])
    r = (xy[b, 1] - xy[a, 1]) * (xy[c, 0] - xy[a, 0])
    det, bound = l - r, 2.0 ** -50 * (np.abs(l) + np.abs(r))
    s = np.sign(det).astype(np.int64)
    for k in np.nonzero(np.abs(det) <= bound)[0]:
        s[k] = oracle.orient(xy[a[k]], xy[b[k]], xy[c[k]])
    return s


def _improving_flips(xy, tv, nbr, prim):
    """Number of unconstrained interior edges whose quad is strictly convex and whose other
    diagonal is strictly shorter."""
    t, i = np.nonzero((nbr > np.arange(tv.shape[0])[:, None]) & (prim < 0))
    u = nbr[t, i]
    j = np.argmax(nbr[u] == t[:, None], axis=1)
    a, b, c = tv[t, i], tv[t, (i + 1) % 3], tv[t, (i + 2) % 3]
    d = tv[u, j]
    convex = (_orient_signs(xy, a, b, d) > 0) & (_orient_signs(xy, a, d, c) > 0)
    ln = lambda p, q: np.sqrt((xy[q, 0] - xy[p, 0]) ** 2 + (xy[q, 1] - xy[p, 1]) ** 2)
    return int(np.count_nonzero(convex & (ln(a, d) < ln(b, c))))


@pytest.fixture(scope="module")
def grid_annealed(ccsp):
    sc = sg.make_scene("grid")
    temps = _temps(sc, 300, 100)
    (tv, nbr, prim), counts = _gpu(ccsp, sc, temps, 0)
    return sc, sc.copy_with(tv, nbr, prim), counts, temps


def test_grid_valid_converged_lighter(ccsp, grid_annealed):
    sc, an, counts, temps = grid_annealed
    assert oracle.validate(oracle.Triangulation.of(an)) == ""
    assert counts[-1] == 0 and counts[0] > 1000
    assert _improving_flips(sc.xy, an.tri_v, an.tri_nbr, an.tri_prim) == 0
    assert _improving_flips(sc.xy, sc.tri_v, sc.tri_nbr, sc.tri_prim) > 1000
    w0, w1 = sg.weight(sc), sg.weight(an)
    assert w1 < 0.7 * w0, (w0, w1)
    # the constraints are the same segments: each keeps its primitive id on the same vertex pairs
    def constrained(s):
        t, i = np.nonzero(s.tri_prim >= 0)
        a, b = s.tri_v[t, (i + 1) % 3], s.tri_v[t, (i + 2) % 3]
        return sorted(zip(s.tri_prim[t, i].tolist(), np.minimum(a, b).tolist(),
                          np.maximum(a, b).tolist()))
    assert constrained(an) == constrained(sc)


def test_grid_repeatable(ccsp, grid_annealed):
    sc, an, counts, temps = grid_annealed
    (tv, nbr, prim), counts2 = _gpu(ccsp, sc, temps, 0)
    assert list(counts2) == list(counts)
    assert np.array_equal(tv, an.tri_v) and np.array_equal(nbr, an.tri_nbr)
    assert np.array_equal(prim, an.tri_prim)


def test_grid_walk_on_annealed(ccsp, grid_annealed):
    """Hits and distances do not depend on the triangulation; steps fall."""
    sc, an, _, _ = grid_annealed
    rays = sg.sample_rays(sc, 1 << 20, seed=4)
    start_an = sg.locate(an, rays.o)
    keep = np.nonzero(start_an >= 0)[0]
    rays = rays.take(keep)
    res = []
    for tri, st in ((sc, rays.start), (an, start_an[keep].astype(np.int32))):
        with ccsp.Scene.from_arrays(tri) as scene:
            o = torch.from_numpy(rays.o).to(DEV)
            d = torch.from_numpy(rays.d).to(DEV)
            r = ccsp.trace(scene, o, d, torch.from_numpy(st).to(DEV), precision="fp64")
            torch.cuda.synchronize()
            res.append([x.cpu().numpy() for x in (r.hit_prim, r.hit_t, r.steps)])
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[1][2].mean() < 0.5 * res[0][2].mean()
    idx = np.arange(0, rays.n, 997)
    ref = oracle.walk(oracle.Triangulation.of(an), rays.o[idx], rays.d[idx],
                      start_an[keep][idx].astype(np.int32))
    assert np.array_equal(res[1][0][idx], ref[0]) and np.array_equal(res[1][2][idx], ref[2])


def _flat_case():
    A, B, Cv, X, Y = 0, 1, 2, 3, 4
    xy = np.array([[0, 0], [3, 0], [1.5, -2.0 ** -60], [1.5, 0.05], [1.5, -1]])
    tv = np.array([[X, A, Cv], [X, Cv, B], [Cv, A, Y], [Cv, Y, B]], dtype=np.int32)
    nbr = np.array([[2, 1, -1], [3, -1, 0], [-1, 3, 0], [-1, 1, 2]], dtype=np.int32)
    prim = np.array([[0, -1, -1], [0, -1, -1], [-1, -1, 0], [-1, 0, -1]], dtype=np.int32)
    line = np.array([-1, -1, 0, -1, -1], dtype=np.int32)
    return xy, tv, nbr, prim, line, np.array([[A, B]], dtype=np.int32)


def _gpu_lines(ccsp, xy, tv, nbr, prim, temps, seed, line=None, pv=None):
    X = torch.from_numpy(np.ascontiguousarray(xy)).to(DEV)
    arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)
            for a in (tv, nbr, prim)]
    extra = () if line is None else (torch.from_numpy(line).to(DEV), torch.from_numpy(pv).to(DEV))
    counts = ccsp.flip_anneal(X, *arrs, temps, seed, *extra)
    return [a.cpu().numpy() for a in arrs], counts


def test_flat_flip_refused_with_original_edges(ccsp):
    """The hand-built quad whose flip would make a triangle flat on an original edge: the GPU
    flips it without the vertices' original edges and refuses it with them, as the checker."""
    xy, tv, nbr, prim, line, pv = _flat_case()
    (tv1, _, _), c1 = _gpu_lines(ccsp, xy, tv, nbr, prim, [1e9], 5)
    assert list(c1) == [1] and not np.array_equal(tv1, tv)
    (tv2, _, _), c2 = _gpu_lines(ccsp, xy, tv, nbr, prim, [1e9, 1e9], 5, line, pv)
    assert list(c2) == [0, 0] and np.array_equal(tv2, tv)
    assert fl.anneal(xy, tv, nbr, prim, [1e9, 1e9], 5, line, pv)[3] == [0, 0]


@pytest.mark.parametrize("seed,eps", [(1, 0.02), (4, 0.1)])
def test_matches_checker_with_steiner_vertices(ccsp, seed, eps):
    """A clustered mesh contracted by the library (Steiner vertices on the original edges, each
    constrained edge its own primitive): GPU flips with the vertices' original edges equal the
    checker's bit for bit, and so do flips without them."""
    import sys
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_contract import _clustered_mesh
    from paper_2112_05570_amd import pipeline as pl
    mesh, xy0 = _clustered_mesh(seed, eps)
    r = ccsp.contract(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, xy0, eps)
    nbr, prim, _, _ = pl.walk_arrays(r["tri_v"], r["kind"], r["line"], mesh.prim_v, r["xy"])
    line = np.where(r["kind"] == 1, r["line"], -1).astype(np.int32)
    pv = np.ascontiguousarray(mesh.prim_v, dtype=np.int32)
    side = 1.0
    temps = list(side * np.geomspace(2e-2, 1e-4, 8)) + [0.0] * 8
    for with_lines in (True, False):
        args = (line, pv) if with_lines else (None, None)
        (tv, nb, pr), counts = _gpu_lines(ccsp, r["xy"], r["tri_v"], nbr, prim, temps, seed, *args)
        rv, rn, rp, rc = fl.anneal(r["xy"], r["tri_v"], nbr, prim, temps, seed, *args)
        assert list(counts) == list(rc) and sum(rc) > 0
        assert np.array_equal(tv, rv) and np.array_equal(nb, rn) and np.array_equal(pr, rp)
