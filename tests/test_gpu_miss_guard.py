"""GPU parity for the two non-hit outcomes of the walk (Sec. 5.1) and for per-launch validation.

* Miss: a ray that reaches a hull edge carrying no primitive has left the triangulation without
  meeting scene geometry (prim -1, t = +inf). Scenes with opened box sides reach it; the HIP walk
  must equal the checker bit for bit in both precision modes, in input order and binned, in
  trace_batch and in the continued (reflecting) walk.
* Step guard: with a step limit L, a walk that would enter triangle L + 1 stops with -2 and
  steps = L; every other ray is unchanged. The limit is set from the host, so every kernel still
  ends normally.
* Validation flags are per launch: validated traces on two host threads and two streams each
  report only their own bad rays.
"""
import json
import os
import threading

import numpy as np
import pytest

import helpers
import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


def _dev(r):
    return (torch.from_numpy(np.ascontiguousarray(r.o)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(r.d)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(r.start)).to(DEV))


def _host(res):
    torch.cuda.synchronize()
    return res.hit_prim.cpu().numpy(), res.hit_t.cpu().numpy(), res.steps.cpu().numpy()


def _same(got, ref, what):
    n = len(ref)
    for name, g, r in zip(("prim", "t", "steps", "bounces", "face")[:n], got[:n], ref):
        ok = (g == r) | (np.isinf(g) & np.isinf(r)) if name == "t" else (g == r)
        bad = np.nonzero(~ok)[0]
        assert bad.size == 0, f"{what}: {name} differs at {bad[:5]}: {g[bad[:5]]} vs {r[bad[:5]]}"


def _bounce_host(res, hits, face):
    torch.cuda.synchronize()
    return (res.hit_prim.cpu().numpy(), res.hit_t.cpu().numpy(), res.steps.cpu().numpy(),
            hits.cpu().numpy(), face.cpu().numpy())


class _Arrays:
    def __init__(self, g):
        self.xy = np.array(g["xy"], float)
        self.tri_v = np.array(g["tri_v"], np.int32)
        self.tri_nbr = np.array(g["tri_nbr"], np.int32)
        self.tri_prim = np.array(g["tri_prim"], np.int32)
        self.prims = np.array(g["prims"], float)


def _golden(name):
    g = json.load(open(os.path.join(GOLDEN, name)))
    r = sg.Rays(np.array([x["o"] for x in g["rays"]], float),
                np.array([x["d"] for x in g["rays"]], float),
                np.array([x["start"] for x in g["rays"]], np.int32))
    return g, _Arrays(g), r


def _tval(x):
    return np.inf if x == "inf" else float(x)


def test_golden_open_sides(ccsp):
    """The hand-derived unit square with two open sides: misses, hits, the guard at one triangle
    and a reflection that leaves through the open top side."""
    g, arr, r = _golden("unit_square_open_sides.json")
    want = (np.array([x["prim"] for x in g["rays"]], np.int32),
            np.array([_tval(x["t"]) for x in g["rays"]]),
            np.array([x["steps"] for x in g["rays"]], np.int32))
    guard = (np.array([x["prim"] for x in g["guard"]], np.int32),
             np.array([_tval(x["t"]) for x in g["guard"]]),
             np.array([x["steps"] for x in g["guard"]], np.int32))
    lim = ccsp.TuneParams(step_limit=g["guard_max_steps"])
    with ccsp.Scene(arr.xy, arr.tri_v, arr.tri_nbr, arr.tri_prim, arr.prims) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            _same(_host(ccsp.trace(scene, *dev, precision=prec)), want, f"golden {prec}")
            _same(_host(ccsp.trace(scene, *dev, precision=prec, tune=lim)), guard,
                  f"golden guard {prec}")
            res = ccsp.trace_batch([(scene, *dev), (scene, *dev)], precision=prec, tune=lim)
            for k in range(2):
                _same(_host(res[k]), guard, f"golden guard batch {prec} item {k}")
            got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 0, precision=prec))
            _same(got[:3], want, f"golden zero bounces {prec}")
            got = _bounce_host(*ccsp.trace_bounces(scene, *[x[3:4] for x in dev], 2, precision=prec))
            assert got[0].tolist() == [-1] and got[2].tolist() == [3] and got[3].tolist() == [1]
            assert got[4].tolist() == [-1] and np.isinf(got[1][0])


@pytest.mark.parametrize("sides", [(0, 1, 2, 3), (1, 2), (3,)])
def test_open_hull_tiny(ccsp, tiny_scene, tiny_rays, sides):
    sc = sg.open_hull(tiny_scene, sides)
    tri = oracle.Triangulation.of(sc)
    ref = oracle.walk(tri, tiny_rays.o, tiny_rays.d, tiny_rays.start)
    assert (ref[0] == -1).sum() > 1000
    with ccsp.Scene.from_arrays(sc) as scene:
        dev = _dev(tiny_rays)
        for prec in ("fp32", "fp64"):
            _same(_host(ccsp.trace(scene, *dev, precision=prec)), ref, f"open {sides} {prec}")
            cut = [0, 1, 4099, 30000, tiny_rays.n]
            parts = [tiny_rays.slice(a, b) for a, b in zip(cut[:-1], cut[1:])]
            res = ccsp.trace_batch([(scene, *_dev(p)) for p in parts], precision=prec)
            for (a, b), rs in zip(zip(cut[:-1], cut[1:]), res):
                _same(_host(rs), tuple(x[a:b] for x in ref), f"open {sides} batch {prec} [{a},{b})")
            got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 3, precision=prec))
            bref = oracle.bounce(tri, tiny_rays.o, tiny_rays.d, tiny_rays.start, 3)
            assert (bref[0] == -1).sum() > 1000
            _same(got, bref, f"open {sides} bounces {prec}")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_open_hull_degenerate_rays(ccsp, seed):
    """Rays through vertices, along edge lines and into the box corners of opened sides."""
    rng = np.random.default_rng(500 + seed)
    sc = sg.open_hull(helpers.integer_scene(rng, 12), ((0, 1, 2, 3), (1, 3), (2,))[seed])
    o, d, start = helpers.degenerate_rays(sc, rng, 3000)
    r = sg.Rays(o, d, start.astype(np.int32))
    tri = oracle.Triangulation.of(sc)
    ref = oracle.walk(tri, r.o, r.d, r.start)
    assert (ref[0] == -1).any()
    with ccsp.Scene.from_arrays(sc) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            _same(_host(ccsp.trace(scene, *dev, precision=prec)), ref, f"degenerate open {prec}")
            got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 2, precision=prec))
            _same(got, oracle.bounce(tri, r.o, r.d, r.start, 2), f"degenerate open bounces {prec}")


@pytest.fixture(scope="module")
def open_grid():
    sc = sg.open_hull(sg.make_scene("grid"), (1, 2))
    rays = sg.sample_rays(sc, 200_003, seed=3)
    return sc, rays


def test_open_hull_binned_grid(ccsp, open_grid):
    """Large enough to be binned: the binned walk and the input-order walk both equal the checker
    on every ray, misses included; so does the continued walk on a sample."""
    sc, r = open_grid
    tri = oracle.Triangulation.of(sc)
    ref = oracle.walk(tri, r.o, r.d, r.start)
    assert (ref[0] == -1).sum() > 100
    with ccsp.Scene.from_arrays(sc) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            _same(_host(ccsp.trace(scene, *dev, precision=prec)), ref, f"open grid binned {prec}")
            _same(_host(ccsp.trace(scene, *dev, precision=prec, input_order=True)), ref,
                  f"open grid input order {prec}")
        idx = np.arange(0, r.n, 23)
        got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 2))
        bref = oracle.bounce(tri, r.o[idx], r.d[idx], r.start[idx], 2)
        assert (bref[0] == -1).any()
        _same(tuple(x[idx] for x in got), bref, "open grid bounces")


@pytest.mark.parametrize("limit", [1, 2, 5, 17])
def test_step_limit(ccsp, tiny_scene, tiny_rays, limit):
    sc = sg.open_hull(tiny_scene, (1, 2))
    tri = oracle.Triangulation.of(sc)
    r = tiny_rays.slice(0, 20_000)
    ref = oracle.walk(tri, r.o, r.d, r.start, max_steps=limit)
    assert (ref[0] == -2).any() and (ref[0] != -2).any()
    tp = ccsp.TuneParams(step_limit=limit)
    with ccsp.Scene.from_arrays(sc) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            _same(_host(ccsp.trace(scene, *dev, precision=prec, tune=tp)), ref, f"limit {limit} {prec}")
            res = ccsp.trace_batch([(scene, *dev)], precision=prec, tune=tp)
            _same(_host(res[0]), ref, f"limit {limit} batch {prec}")
            res = ccsp.trace_batch([(scene, *dev)], precision=prec, tune=tp, graph=True)
            _same(_host(res[0]), ref, f"limit {limit} batch graph {prec}")
            got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 3, precision=prec, tune=tp))
            _same(got, oracle.bounce(tri, r.o, r.d, r.start, 3, max_steps=limit),
                  f"limit {limit} bounces {prec}")
        # no limit, or one at the triangle count: the plain walk
        plain = oracle.walk(tri, r.o, r.d, r.start)
        for lim in (0, sc.n_triangles, 2**31 - 1):
            _same(_host(ccsp.trace(scene, *dev, tune=ccsp.TuneParams(step_limit=lim))), plain,
                  f"limit {lim}")


def test_step_limit_binned(ccsp, open_grid):
    sc, r = open_grid
    tri = oracle.Triangulation.of(sc)
    ref = oracle.walk(tri, r.o, r.d, r.start, max_steps=9)
    assert (ref[0] == -2).mean() > 0.1
    with ccsp.Scene.from_arrays(sc) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            for binning in (1, 2):
                tp = ccsp.TuneParams(step_limit=9, bin=binning)
                _same(_host(ccsp.trace(scene, *dev, precision=prec, tune=tp)), ref,
                      f"binned ({binning}) limit {prec}")


def test_step_limit_rejected_when_negative(ccsp, tiny_scene, tiny_rays):
    r = tiny_rays.slice(0, 10)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        with pytest.raises(ccsp.CcspError):
            ccsp.trace(scene, *_dev(r), tune=ccsp.TuneParams(step_limit=-1))


def test_validation_flags_per_launch(ccsp, tiny_scene, tiny_rays):
    """Validated traces from two host threads on two streams at once: the one with a bad ray
    always reports it, the other never reports one."""
    r = tiny_rays.slice(0, 50_000)
    bad_start = r.start.copy()
    bad_start[12345] = np.roll(r.start, 1)[12345] if r.start[12344] != r.start[12345] else -1
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), r.o, r.d, r.start)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        o, d, st = _dev(r)
        st_bad = torch.from_numpy(bad_start).to(DEV)
        torch.cuda.synchronize()
        errors = []
        outcome = {"good": [], "bad": []}

        def run(which, start):
            try:
                s = torch.cuda.Stream()
                for _ in range(40):
                    try:
                        with torch.cuda.stream(s):
                            res = ccsp.trace(scene, o, d, start, stream=s, validate=True)
                        s.synchronize()
                        outcome[which].append(("ok", res))
                    except ccsp.CcspError as e:
                        outcome[which].append(("bad", e.code))
            except Exception as e:  # noqa: BLE001 - reported below
                errors.append(repr(e))

        ts = [threading.Thread(target=run, args=("good", st)),
              threading.Thread(target=run, args=("bad", st_bad))]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errors, errors
        assert all(k == "ok" for k, _ in outcome["good"]), "a valid trace reported a bad ray"
        assert all(k == "bad" and v == ccsp.binding.CCSP_E_BAD_RAY for k, v in outcome["bad"])
        _same(_host(outcome["good"][-1][1]), ref, "validated good trace")
