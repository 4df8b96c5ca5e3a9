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
