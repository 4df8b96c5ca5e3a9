"""GPU parity of the 3D walk (trace_rays3d through the C ABI) with the checker's walk, bit for
bit in hit_prim, hit_t and steps:

* a 2,000-point tetrahedralisation with 15% of its interior faces as primitives, 20,000 rays,
  binned and in input order, under several launch shapes, and with a trace of another mesh on
  another stream in between;
* rays through vertices, edge midpoints, parallel to edges and along edge lines (every zero sign
  decided by the moved line on both sides);
* an open hull (misses), the step guard, invalid rays (zero direction, off the grid, start out of
  range, origin on a face);
* the benchmark's workload at full size (200,000 grid points, 1.35M tetrahedra, 5% primitives,
  4M rays), 30,000 sampled rays against the checker.
"""
import sys
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_tet import _degenerate_rays  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


def _run(ccsp, mesh, o, d, st, **kw):
    t = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV) for a in (o, d, st)]
    res = ccsp.trace3d(mesh, *t, **kw)
    torch.cuda.synchronize()
    return res.hit_prim.cpu().numpy(), res.hit_t.cpu().numpy(), res.steps.cpu().numpy()


def _same(got, ref, what):
    for name, g, r in zip(("prim", "t", "steps"), got, ref):
        ok = (g == r) | (np.isinf(g) & np.isinf(r)) if name == "t" else (g == r)
        bad = np.nonzero(~ok)[0]
        assert bad.size == 0, f"{what}: {name} differs at {bad[:5]}: {g[bad[:5]]} vs {r[bad[:5]]}"


def test_small_scene_vs_checker(ccsp):
    sc = sg.make_tet_scene(2000, seed=0)
    r = sg.sample_rays3(sc, 20_000, seed=1)
    ref = oracle.walk3(oracle.TetMesh.of(sc), r.o, r.d, r.start)[:3]
    print(f"{sc.n_tets} tetrahedra, mean steps {ref[2].mean():.1f}", flush=True)
    with ccsp.TetMesh.from_arrays(sc) as mesh:
        _same(_run(ccsp, mesh, r.o, r.d, r.start), ref, "default launch (binned)")
        _same(_run(ccsp, mesh, r.o, r.d, r.start, input_order=True), ref, "input order")
        for tune in ((64, 1, 64, 1, 1), (512, 8, 1024, 64, 2), (128, 64, 128, 32, 1)):
            t = ccsp.binding.Tune3d(*tune)
            _same(_run(ccsp, mesh, r.o, r.d, r.start, tune=t), ref, f"launch {tune}")
            _same(_run(ccsp, mesh, r.o, r.d, r.start, tune=t, input_order=True), ref,
                  f"launch {tune}, input order")
        # a ragged tail: fewer rays than one claim, and one ray
        for n in (1, 97):
            _same(_run(ccsp, mesh, r.o[:n], r.d[:n], r.start[:n]), tuple(x[:n] for x in ref), f"n={n}")
        # a second mesh traced in between on another stream, then this one again
        s2 = torch.cuda.Stream()
        with ccsp.TetMesh.from_arrays(sg.make_tet_scene(500, seed=9)) as other:
            r2 = sg.sample_rays3(sg.make_tet_scene(500, seed=9), 3000, seed=3)
            with torch.cuda.stream(s2):
                t2 = [torch.from_numpy(a).to(DEV) for a in (r2.o, r2.d, r2.start)]
                res2 = ccsp.trace3d(other, *t2, stream=s2)
            _same(_run(ccsp, mesh, r.o, r.d, r.start), ref, "after another stream")
            torch.cuda.synchronize()
            ref2 = oracle.walk3(oracle.TetMesh.of(sg.make_tet_scene(500, seed=9)), r2.o, r2.d, r2.start)[:3]
            _same((res2.hit_prim.cpu().numpy(), res2.hit_t.cpu().numpy(), res2.steps.cpu().numpy()),
                  ref2, "other stream")


def test_degenerate_rays_vs_checker(ccsp):
    sc = sg.make_tet_scene(2000, seed=0, frac_prims=0.02)
    m = oracle.TetMesh.of(sc)
    rays = _degenerate_rays(sc, np.random.default_rng(5), 600)
    with ccsp.TetMesh.from_arrays(sc) as mesh:
        for name, (o, d, st) in rays.items():
            ref = oracle.walk3(m, o, d, st)
            assert ref[3].sum() > 0 or name == "parallel"
            _same(_run(ccsp, mesh, o, d, st), ref[:3], name)


def test_open_hull_guard_and_bad_rays(ccsp):
    sc = sg.make_tet_scene(1500, seed=4, frac_prims=0.03, open_hull=True)
    m = oracle.TetMesh.of(sc)
    r = sg.sample_rays3(sc, 8000, seed=2)
    ref = oracle.walk3(m, r.o, r.d, r.start)[:3]
    assert (ref[0] == -1).sum() > 1000
    with ccsp.TetMesh.from_arrays(sc) as mesh:
        _same(_run(ccsp, mesh, r.o, r.d, r.start), ref, "open hull")
        for lim in (1, 2, 7):
            rl = oracle.walk3(m, r.o, r.d, r.start, max_steps=lim)[:3]
            assert (rl[0] == -2).sum() > 100
            _same(_run(ccsp, mesh, r.o, r.d, r.start, step_limit=lim), rl, f"step limit {lim}")
        # invalid rays: zero direction, origin and direction off the grid, start out of range,
        # origin on a vertex, origin inside another tetrahedron
        tv = sc.tet_v[r.start[0]]
        o = np.array([r.o[0], [-1, 5, 5], r.o[0], r.o[0], sc.xyz[tv[0]], r.o[1]], np.int64)
        d = np.array([[0, 0, 0], r.d[0], [1 << 19 | 1, 0, 0], r.d[0], r.d[0], r.d[1]], np.int64)
        st = np.array([r.start[0], r.start[0], r.start[0], sc.n_tets, r.start[0],
                       (r.start[1] + 1) % sc.n_tets], np.int64)
        ref = oracle.walk3(m, o, d, st)[:3]
        assert (ref[0] == -3).all()
        _same(_run(ccsp, mesh, o, d, st), ref, "invalid rays")


def test_bench_workload_vs_checker(ccsp):
    sc = sg.make_tet_scene(200_000, seed=0, frac_prims=0.05)
    r = sg.sample_rays3(sc, 1 << 22, seed=1)
    print(f"{sc.n_tets} tetrahedra, {sc.n_prims} primitives, {r.n} rays", flush=True)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(r.n, 30_000, replace=False), [0, r.n - 1]]))
    ref = oracle.walk3(oracle.TetMesh.of(sc), r.o[idx], r.d[idx], r.start[idx])[:3]
    with ccsp.TetMesh.from_arrays(sc) as mesh:
        got = _run(ccsp, mesh, r.o, r.d, r.start)
        got_io = _run(ccsp, mesh, r.o, r.d, r.start, input_order=True)
    _same(tuple(x[idx] for x in got), ref, "bench workload")
    for a, b, name in zip(got, got_io, ("prim", "t", "steps")):
        assert np.array_equal(a, b), f"binned and input-order {name} differ"
    assert (got[0] >= 0).all()
    assert 10 < got[2].mean() < 40
