"""The low-weight pipeline (paper_2112_05570_amd.pipeline.optimise) end to end on the tiny scene:
annealing with every single-vertex proposal on the GPU, the library's contraction, polishing and
greedy flips. The result is a valid constrained triangulation that keeps the original vertices,
weighs less than the subdivided input, and on which the GPU walk equals the checker's walk bit for
bit; hits match the CDT's primitives; two runs with one seed are identical."""
import numpy as np
import pytest

import oracle
import helpers
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


@pytest.fixture(scope="module")
def run(ccsp):
    from paper_2112_05570_amd import pipeline as pl
    sc = sg.make_scene("tiny")
    mesh = helpers.subdivided(sc)
    size = sc.box[1] - sc.box[0]
    sched = pl.Schedule(stages=9, t0_rel=1e-3, t1_rel=1e-5, e0_rel=2e-2, e1_rel=2e-3,
                        outer_max=4, flip_rounds=32, seed=3)
    r = pl.optimise(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy, size, sched)
    return sc, mesh, sched, r


def test_result_is_valid_and_lighter(ccsp, run):
    from paper_2112_05570_amd import pipeline as pl
    sc, mesh, _, r = run
    nbr, prim, prims, s2o = pl.walk_arrays(r.tri_v, r.kind, r.line, mesh.prim_v, r.xy)
    assert oracle.validate(oracle.Triangulation(r.xy, r.tri_v, nbr, prim, prims)) == ""
    assert (r.kind == 0).sum() == sc.n_vertices
    assert np.array_equal(r.xy[r.kind == 0], sc.xy)  # original vertices keep id order and place
    assert r.log["weight_final"] < r.log["weight_start"]
    assert r.log["weight_final"] == pl.weight(r.tri_v, r.xy)
    assert r.xy.shape[0] < mesh.n_vertices


def test_walk_on_result_equals_checker(ccsp, run):
    from paper_2112_05570_amd import pipeline as pl
    sc, mesh, _, r = run
    nbr, prim, prims, s2o = pl.walk_arrays(r.tri_v, r.kind, r.line, mesh.prim_v, r.xy)
    rays = sg.sample_rays(sc, 20000, seed=5)
    with ccsp.Scene(r.xy, r.tri_v, nbr, prim, prims) as s_opt, ccsp.Scene.from_arrays(sc) as s_cdt:
        o = torch.from_numpy(rays.o).to(DEV)
        d = torch.from_numpy(rays.d).to(DEV)
        st, stat = ccsp.locate(s_opt, o)
        keep = torch.nonzero(stat == 0).squeeze(1)
        assert keep.shape[0] > 19000
        o, d, st = o[keep].contiguous(), d[keep].contiguous(), st[keep].contiguous()
        got = ccsp.trace(s_opt, o, d, st, precision="fp32")
        cdt = ccsp.trace(s_cdt, o, d, torch.from_numpy(rays.start).to(DEV)[keep].contiguous(),
                         precision="fp64")
        torch.cuda.synchronize()
        g = [x.cpu().numpy() for x in (got.hit_prim, got.hit_t, got.steps)]
        c = [x.cpu().numpy() for x in (cdt.hit_prim, cdt.hit_t, cdt.steps)]
    k = keep.cpu().numpy()
    ref = oracle.walk(oracle.Triangulation(r.xy, r.tri_v, nbr, prim, prims), rays.o[k], rays.d[k],
                      st.cpu().numpy())
    assert np.array_equal(g[0], ref[0]) and np.array_equal(g[1], ref[1])
    assert np.array_equal(g[2], ref[2])
    mapped = np.where(g[0] >= 0, s2o[np.maximum(g[0], 0)], g[0])
    # every original edge survives as a chain of sub-edges, so each ray hits the same primitive
    _assert_chains(prims, s2o, mesh.prim_v, mesh.xy)
    assert np.array_equal(mapped, c[0]), np.nonzero(mapped != c[0])[0][:5]
    assert g[2].mean() < c[2].mean() * 1.5


def _assert_chains(prims, s2o, prim_v, xy):
    """The sub-edges mapped to original edge k, ordered along it, join end to end from one of its
    original vertices to the other: no original edge lost a piece."""
    for k in range(prim_v.shape[0]):
        a, b = xy[prim_v[k, 0]], xy[prim_v[k, 1]]
        segs = prims[s2o == k]
        assert segs.shape[0] >= 1, f"original edge {k} has no sub-edge"
        e = b - a
        # orient every sub-edge from a towards b, then order them along the edge
        t0 = (segs[:, :2] - a) @ e
        t1 = (segs[:, 2:] - a) @ e
        flip = t1 < t0
        segs = np.where(flip[:, None], segs[:, [2, 3, 0, 1]], segs)
        segs = segs[np.argsort(np.minimum(t0, t1))]
        assert np.array_equal(segs[0, :2], a) and np.array_equal(segs[-1, 2:], b), k
        assert np.array_equal(segs[1:, :2], segs[:-1, 2:]), k


def test_same_seed_same_result(ccsp, run):
    from paper_2112_05570_amd import pipeline as pl
    _, mesh, sched, r = run
    sc = sg.make_scene("tiny")
    r2 = pl.optimise(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy, sc.box[1] - sc.box[0],
                     sched)
    assert np.array_equal(r2.tri_v, r.tri_v) and np.array_equal(r2.xy, r.xy)


@pytest.mark.parametrize("name,kw,seed", [("tiny", {}, 7), ("large", dict(n_seg=2000), 1)])
def test_other_scenes_and_seeds(ccsp, name, kw, seed):
    """The pipeline on another seed and on an 8,002-triangle random-lines scene: valid result,
    original vertices kept, lighter than the subdivided input, and the GPU walk on it equal to the
    checker's on a sample of located rays, hitting the CDT's primitives."""
    from paper_2112_05570_amd import pipeline as pl
    sc = sg.make_scene(name, **kw)
    mesh = helpers.subdivided(sc)
    size = sc.box[1] - sc.box[0]
    sched = pl.Schedule(stages=8, t0_rel=1e-3, t1_rel=1e-5, e0_rel=5e-3, e1_rel=5e-4,
                        outer_max=3, flip_rounds=32, seed=seed)
    r = pl.optimise(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy, size, sched)
    nbr, prim, prims, s2o = pl.walk_arrays(r.tri_v, r.kind, r.line, mesh.prim_v, r.xy)
    tri = oracle.Triangulation(r.xy, r.tri_v, nbr, prim, prims)
    assert oracle.validate(tri) == ""
    assert (r.kind == 0).sum() == sc.n_vertices and np.array_equal(r.xy[r.kind == 0], sc.xy)
    assert r.log["weight_final"] < r.log["weight_start"]
    rays = sg.sample_rays(sc, 8192, seed=seed)
    with ccsp.Scene(r.xy, r.tri_v, nbr, prim, prims) as s_opt:
        o = torch.from_numpy(rays.o).to(DEV)
        d = torch.from_numpy(rays.d).to(DEV)
        st, stat = ccsp.locate(s_opt, o)
        keep = torch.nonzero(stat == 0).squeeze(1)
        got = ccsp.trace(s_opt, o[keep].contiguous(), d[keep].contiguous(),
                         st[keep].contiguous(), precision="fp64")
        torch.cuda.synchronize()
        g = [x.cpu().numpy() for x in (got.hit_prim, got.hit_t, got.steps)]
    k = keep.cpu().numpy()
    assert k.shape[0] > 8000
    ref = oracle.walk(tri, rays.o[k], rays.d[k], st.cpu().numpy()[k])
    assert all(np.array_equal(a, b) for a, b in zip(g, ref))
    cdt = oracle.walk(oracle.Triangulation.of(sc), rays.o[k], rays.d[k], rays.start[k])
    mapped = np.where(g[0] >= 0, s2o[np.maximum(g[0], 0)], g[0])
    _assert_chains(prims, s2o, mesh.prim_v, mesh.xy)
    assert np.array_equal(mapped, cdt[0]), np.nonzero(mapped != cdt[0])[0][:5]


def test_iterated_strategy(ccsp):
    """Sec. 3.5.3's iterated strategy, two rounds of subdivision and optimisation on the tiny
    scene: the second round starts from the first result subdivided (so it has more vertices than
    that result), the returned triangulation is the lighter round's and is valid, keeps the original
    vertices, and the GPU walk on it equals the checker's on a sample of located rays."""
    from paper_2112_05570_amd import pipeline as pl
    sc = sg.make_scene("tiny")
    xy, tv, kd, ln, pv = sg.movable_input(sc)
    size = sc.box[1] - sc.box[0]
    sched = pl.Schedule(stages=6, t0_rel=1e-3, t1_rel=1e-5, e0_rel=2e-2, e1_rel=2e-3,
                        outer_max=2, flip_rounds=16, seed=11)
    r = pl.optimise_iterated(tv, kd, ln, pv, xy, size, sched, rounds=2)
    logs = r.log["rounds"]
    assert len(logs) == 2
    w = [g["weight_final"] for g in logs]
    assert r.log["weight_final"] == min(w)
    assert logs[1]["subdivided_vertices"] > logs[0]["vertices"]
    nbr, prim, prims, s2o = pl.walk_arrays(r.tri_v, r.kind, r.line, pv, r.xy)
    tri = oracle.Triangulation(r.xy, r.tri_v, nbr, prim, prims)
    assert oracle.validate(tri) == ""
    assert (r.kind == 0).sum() == sc.n_vertices and np.array_equal(r.xy[r.kind == 0], sc.xy)
    assert r.log["weight_final"] == pl.weight(r.tri_v, r.xy)
    rays = sg.sample_rays(sc, 4096, seed=13)
    with ccsp.Scene(r.xy, r.tri_v, nbr, prim, prims) as s_opt:
        o = torch.from_numpy(rays.o).to(DEV)
        d = torch.from_numpy(rays.d).to(DEV)
        st, stat = ccsp.locate(s_opt, o)
        keep = torch.nonzero(stat == 0).squeeze(1)
        got = ccsp.trace(s_opt, o[keep].contiguous(), d[keep].contiguous(),
                         st[keep].contiguous(), precision="fp64")
        torch.cuda.synchronize()
        g = [x.cpu().numpy() for x in (got.hit_prim, got.hit_t, got.steps)]
    k = keep.cpu().numpy()
    assert k.shape[0] > 4000
    ref = oracle.walk(tri, rays.o[k], rays.d[k], st.cpu().numpy()[k])
    assert all(np.array_equal(a, b) for a, b in zip(g, ref))


def test_time_balanced_perturbations(ccsp):
    """Sec. 3.3.2's choice of perturbation types by equal computation time: every type runs
    (each first once, to be timed), the stages run the asked number of sweeps, and the result is
    a valid triangulation, lighter than the subdivided input, that keeps the original vertices."""
    from paper_2112_05570_amd import pipeline as pl
    sc = sg.make_scene("tiny")
    mesh = helpers.subdivided(sc)
    size = sc.box[1] - sc.box[0]
    sched = pl.Schedule(stages=4, t0_rel=1e-3, t1_rel=1e-5, e0_rel=2e-2, e1_rel=2e-3,
                        outer_max=2, flip_rounds=16, seed=5, balance_sweeps=6)
    r = pl.optimise(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy, size, sched)
    bal = r.log["balance"]
    assert sum(bal["sweeps"].values()) == 4 * 6
    assert all(c >= 1 for c in bal["sweeps"].values())
    nbr, prim, prims, s2o = pl.walk_arrays(r.tri_v, r.kind, r.line, mesh.prim_v, r.xy)
    assert oracle.validate(oracle.Triangulation(r.xy, r.tri_v, nbr, prim, prims)) == ""
    assert (r.kind == 0).sum() == sc.n_vertices and np.array_equal(r.xy[r.kind == 0], sc.xy)
    assert r.log["weight_final"] < r.log["weight_start"]
