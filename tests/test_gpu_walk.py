"""GPU parity of the HIP walk against the checker (runs on an MI355X).

hit_prim and steps must match bit for bit; hit_t is computed by the same fixed binary64 formula on
both sides, so it is compared bit for bit as well (stricter than the 1e-12 / 1e-5 relative
tolerances stated for the two precision modes). Both precision modes must give identical results.
"""
import ctypes

import numpy as np
import pytest

import helpers
import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


DEV = "cuda:0"


def _dev(r):
    return (torch.from_numpy(np.ascontiguousarray(r.o)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(r.d)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(r.start)).to(DEV))


def _host(res):
    torch.cuda.synchronize()
    return res.hit_prim.cpu().numpy(), res.hit_t.cpu().numpy(), res.steps.cpu().numpy()


def _assert_same(got, ref, what=""):
    p, t, s = got
    rp, rt, rs = ref
    bad = np.nonzero((p != rp) | (s != rs) | ~((t == rt) | (np.isinf(t) & np.isinf(rt))))[0]
    assert bad.size == 0, (f"{what}: {bad.size} rays differ, first {bad[:5]}: "
                           f"gpu {p[bad[:5]]}, {s[bad[:5]]}, {t[bad[:5]]} vs "
                           f"ref {rp[bad[:5]]}, {rs[bad[:5]]}, {rt[bad[:5]]}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tiny_all_rays(ccsp, tiny_scene, tiny_rays, prec):
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), tiny_rays.o, tiny_rays.d, tiny_rays.start)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        got = _host(ccsp.trace(scene, *_dev(tiny_rays), precision=prec))
    _assert_same(got, ref, prec)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 127, 4099])
@pytest.mark.parametrize("tune", [(64, 64, 32, 1), (256, 128, 32, 16), (512, 256, 16, 64), (128, 64, 8, 32)])
def test_ragged_and_launch_shapes(ccsp, tiny_scene, tiny_rays, n, tune):
    r = tiny_rays.slice(0, n)
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), r.o, r.d, r.start)
    tp = ccsp.TuneParams(*tune)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        for prec in ("fp32", "fp64"):
            got = _host(ccsp.trace(scene, *_dev(r), precision=prec, tune=tp))
            _assert_same(got, ref, f"{prec} n={n} tune={tune}")


def test_empty_trace_is_noop(ccsp, tiny_scene):
    e = torch.empty((0, 2), dtype=torch.float64, device=DEV)
    s = torch.empty((0,), dtype=torch.int32, device=DEV)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        res = ccsp.trace(scene, e, e, s)
        torch.cuda.synchronize()
    assert res.hit_prim.numel() == 0


def test_bad_start_and_validation(ccsp, tiny_scene, tiny_rays):
    r = tiny_rays.slice(0, 300)
    start = r.start.copy()
    start[5] = -1
    start[17] = tiny_scene.n_triangles
    start[31] = 2**31 - 1
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        o, d, _ = _dev(r)
        st = torch.from_numpy(start).to(DEV)
        for prec in ("fp32", "fp64"):
            p, t, s = _host(ccsp.trace(scene, o, d, st, precision=prec))
            assert (p[[5, 17, 31]] == ccsp.CCSP_RAY_BAD).all() and (s[[5, 17, 31]] == 0).all()
            assert np.isinf(t[[5, 17, 31]]).all()
            ok = np.ones(300, bool)
            ok[[5, 17, 31]] = False
            assert (p[ok] >= 0).all()
        with pytest.raises(ccsp.CcspError) as ei:
            ccsp.trace(scene, o, d, st, validate=True)
        assert ei.value.code == ccsp.binding.CCSP_E_BAD_RAY
        # a valid start triangle that does not contain the origin is caught too
        wrong = torch.from_numpy(np.roll(r.start, 1)).to(DEV)
        with pytest.raises(ccsp.CcspError):
            ccsp.trace(scene, o, d, wrong, validate=True, precision="fp64")
        # and valid rays pass validation with the same results
        ref = oracle.walk(oracle.Triangulation.of(tiny_scene), r.o, r.d, r.start)
        got = _host(ccsp.trace(scene, *_dev(r), validate=True))
        _assert_same(got, ref, "validated")


def _integer_scene(seed):
    from helpers import degenerate_rays, integer_scene
    rng = np.random.default_rng(seed)
    sc = integer_scene(rng, 12)
    o, d, start = degenerate_rays(sc, rng, 3000)
    return sc, sg.Rays(o, d, start.astype(np.int32))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_degenerate_rays(ccsp, seed):
    sc, r = _integer_scene(seed)
    ref = oracle.walk(oracle.Triangulation.of(sc), r.o, r.d, r.start)
    assert (ref[0] >= 0).all()
    with ccsp.Scene.from_arrays(sc) as scene:
        for prec in ("fp32", "fp64"):
            ccsp.read_counters(reset=True)
            got = _host(ccsp.trace(scene, *_dev(r), precision=prec, count=True))
            _assert_same(got, ref, f"degenerate {prec}")
            steps, fb32, fb64, rays = ccsp.read_counters(reset=True)
            assert rays == r.n and steps == int(ref[2].sum())
            assert fb64 > 0  # exact ties really reached the exact expansion


@pytest.fixture(scope="module")
def grid_pair():
    sc = sg.make_scene("grid")
    an, _ = sg.anneal_flips(sc, seed=0)
    rays = sg.sample_rays(sc, sg.WORKLOADS["grid"]["rays"], seed=0)
    start_an = sg.locate(an, rays.o)
    keep = start_an >= 0
    rays = rays.take(np.nonzero(keep)[0])
    return sc, an, rays, start_an[keep].astype(np.int32)


def test_grid_cdt_and_annealed(ccsp, grid_pair):
    sc, an, rays, start_an = grid_pair
    ra = sg.Rays(rays.o, rays.d, start_an)
    ref_c = oracle.walk(oracle.Triangulation.of(sc), rays.o, rays.d, rays.start)
    ref_a = oracle.walk(oracle.Triangulation.of(an), ra.o, ra.d, ra.start)
    # the hit and its distance do not depend on the triangulation; the step count does
    assert np.array_equal(ref_c[0], ref_a[0]) and np.array_equal(ref_c[1], ref_a[1])
    assert ref_a[2].mean() < ref_c[2].mean()
    for tri, r, ref in ((sc, rays, ref_c), (an, ra, ref_a)):
        with ccsp.Scene.from_arrays(tri) as scene:
            for prec in ("fp32", "fp64"):
                _assert_same(_host(ccsp.trace(scene, *_dev(r), precision=prec)), ref, f"grid {prec}")


@pytest.mark.parametrize("n", [65535, 65536, 200_003])
def test_binned_equals_input_order(ccsp, grid_pair, n):
    sc, _, rays, _ = grid_pair
    r = rays.slice(0, n)
    with ccsp.Scene.from_arrays(sc) as scene:
        o, d, st = _dev(r)
        for prec in ("fp32", "fp64"):
            a = _host(ccsp.trace(scene, o, d, st, precision=prec))
            b = _host(ccsp.trace(scene, o, d, st, precision=prec, input_order=True))
            _assert_same(a, b, f"binned vs input order {prec} n={n}")
        idx = np.arange(0, n, 37)
        ref = oracle.walk(oracle.Triangulation.of(sc), r.o[idx], r.d[idx], r.start[idx])
        _assert_same((a[0][idx], a[1][idx], a[2][idx]), ref, "binned vs checker")


def test_stage_times(ccsp, grid_pair, tiny_scene, tiny_rays):
    """Timed traces record (binning, walk) durations; results are unchanged by timing."""
    sc, _, rays, _ = grid_pair
    ccsp.read_stage_times()  # forget older records
    r = rays.slice(0, 300_000)
    with ccsp.Scene.from_arrays(sc) as scene, ccsp.Scene.from_arrays(tiny_scene) as tiny:
        o, d, st = _dev(r)
        ref = _host(ccsp.trace(scene, o, d, st))
        for _ in range(3):
            got = ccsp.trace(scene, o, d, st, timed=True)
        ccsp.trace(tiny, *_dev(tiny_rays), timed=True, input_order=True)
        bin_ms, walk_ms, fin_ms = ccsp.read_stage_times()
        _assert_same(_host(got), ref, "timed trace")
        assert len(bin_ms) == len(walk_ms) == len(fin_ms) == 4
        assert all(w > 0 for w in walk_ms) and all(f > 0 for f in fin_ms)
        assert all(b > 0 for b in bin_ms[:3])      # the grid traces bin their rays
        assert bin_ms[3] < 0.5 * walk_ms[3] + 0.05  # the tiny trace does not
        assert ccsp.read_stage_times() == ([], [], [])  # reading forgets the records
        # the ring keeps the last 256 records
        o2, d2, st2 = _dev(tiny_rays.slice(0, 1000))
        for _ in range(300):
            ccsp.trace(tiny, o2, d2, st2, timed=True)
        b, w, f = ccsp.read_stage_times(1000)
        assert len(w) == 256
        b, w, f = ccsp.read_stage_times(0)
        assert w == []


def test_reserve_workspace_then_trace(ccsp, tiny_scene, tiny_rays):
    ccsp.reserve_workspace(1 << 17)
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), tiny_rays.o, tiny_rays.d, tiny_rays.start)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        _assert_same(_host(ccsp.trace(scene, *_dev(tiny_rays))), ref, "after reserve")
    with pytest.raises(ccsp.CcspError):
        ccsp.reserve_workspace(-1)


def test_large_bench_configuration_sampled(ccsp):
    """The 1M-segment scene and all 2^26 rays in the default launch: every ray checked for
    agreement between the two modes and for valid outputs, a sample against the checker."""
    sc = sg.make_scene("large")
    rays = sg.sample_rays(sc, sg.WORKLOADS["large"]["rays"], seed=0)
    idx = np.random.default_rng(7).choice(rays.n, 50_000, replace=False)
    idx = np.concatenate([idx, np.arange(rays.n - 1000, rays.n)])  # and the ragged end
    sub = rays.take(idx)
    ref = oracle.walk(oracle.Triangulation.of(sc), sub.o, sub.d, sub.start)
    with ccsp.Scene.from_arrays(sc) as scene:
        o, d, st = _dev(rays)
        del rays
        r32 = ccsp.trace(scene, o, d, st, precision="fp32")
        p32, t32, s32 = _host(r32)
        _assert_same((p32[idx], t32[idx], s32[idx]), ref, "large fp32 sample")
        assert (p32 >= 0).all() and (s32 >= 1).all() and np.isfinite(t32).all() and (t32 > 0).all()
        del r32
        r64 = ccsp.trace(scene, o, d, st, precision="fp64")
        p64, t64, s64 = _host(r64)
        assert np.array_equal(p32, p64) and np.array_equal(s32, s64) and np.array_equal(t32, t64)
        del r64
        ri = ccsp.trace(scene, o, d, st, precision="fp32", input_order=True)
        pi, ti, si = _host(ri)
        assert np.array_equal(p32, pi) and np.array_equal(s32, si) and np.array_equal(t32, ti)


def _batch_scenes(k=6, max_seg=20000):
    segs, nrays = sg.multi_sizes("batch", seed=0)
    out = []
    for i in range(k):
        ns = int(min(segs[i], max_seg))
        sc = sg.make_scene("batch", seed=0, n_seg=ns, index=i)
        r = sg.sample_rays(sc, int(min(nrays[i], 100_000)) + 17 * i, seed=i + 1)
        out.append((sc, r))
    return out


def test_batch_equals_single_and_graph_replays(ccsp):
    data = _batch_scenes()
    scenes = [ccsp.Scene.from_arrays(sc) for sc, _ in data]
    try:
        devr = [_dev(r) for _, r in data]
        refs = []
        for scene, (o, d, st) in zip(scenes, devr):
            refs.append(_host(ccsp.trace(scene, o, d, st)))
        # oracle on a sample of each item
        for (sc, r), ref in zip(data, refs):
            idx = np.arange(0, r.n, 97)
            rr = oracle.walk(oracle.Triangulation.of(sc), r.o[idx], r.d[idx], r.start[idx])
            _assert_same((ref[0][idx], ref[1][idx], ref[2][idx]), rr, "single vs checker")
        for prec in ("fp32", "fp64"):
            jobs = [(scene, *x) for scene, x in zip(scenes, devr)]
            res = ccsp.trace_batch(jobs, precision=prec)
            for k, rs in enumerate(res):
                _assert_same(_host(rs), refs[k], f"batch {prec} item {k}")
        # graph path: replay with changing item order and contents; every replay is checked
        for rep in range(4):
            order = np.random.default_rng(rep).permutation(len(scenes))
            jobs = [(scenes[k], *devr[k]) for k in order]
            res = ccsp.trace_batch(jobs, precision="fp32", graph=True)
            torch.cuda.synchronize()
            for k, rs in zip(order, res):
                _assert_same(_host(rs), refs[k], f"graph replay {rep} item {k}")
            # eager work between replays
            _assert_same(_host(ccsp.trace(scenes[0], *devr[0])), refs[0], "eager between replays")
    finally:
        for s in scenes:
            s.free()


def test_batch_with_empty_and_tiny_items(ccsp, tiny_scene, tiny_rays):
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        parts = [tiny_rays.slice(0, 0), tiny_rays.slice(0, 1), tiny_rays.slice(1, 130),
                 tiny_rays.slice(130, 130), tiny_rays.slice(130, 5000)]
        jobs = [(scene, *_dev(p)) for p in parts]
        res = ccsp.trace_batch(jobs, precision="fp64")
        for p, rs in zip(parts, res):
            ref = oracle.walk(oracle.Triangulation.of(tiny_scene), p.o, p.d, p.start)
            _assert_same(_host(rs), ref, f"batch part n={p.n}")


def test_binned_traces_on_two_streams(ccsp, grid_pair):
    """Binned traces share the per-device scratch; traces on two streams must still be right."""
    sc, _, rays, _ = grid_pair
    r1, r2 = rays.slice(0, 300_000), rays.slice(300_000, 700_000)
    with ccsp.Scene.from_arrays(sc) as scene:
        d1, d2 = _dev(r1), _dev(r2)
        ref1 = _host(ccsp.trace(scene, *d1, input_order=True))
        ref2 = _host(ccsp.trace(scene, *d2, input_order=True))
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        for _ in range(3):
            with torch.cuda.stream(s1):
                a = ccsp.trace(scene, *d1, stream=s1)
            with torch.cuda.stream(s2):
                b = ccsp.trace(scene, *d2, stream=s2, precision="fp64")
            torch.cuda.synchronize()
            _assert_same(_host(a), ref1, "binned stream 1")
            _assert_same(_host(b), ref2, "binned stream 2")


def test_concurrent_streams(ccsp, tiny_scene, tiny_rays):
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), tiny_rays.o, tiny_rays.d, tiny_rays.start)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        o, d, st = _dev(tiny_rays)  # 65,536 rays: both traces are binned, sharing the scratch
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            a = ccsp.trace(scene, o, d, st, stream=s1)
        with torch.cuda.stream(s2):
            b = ccsp.trace(scene, o, d, st, stream=s2, precision="fp64")
        torch.cuda.synchronize()
        _assert_same(_host(a), ref, "stream 1")
        _assert_same(_host(b), ref, "stream 2")


def test_autotune_single_batch_and_cache(ccsp, tiny_scene, tiny_rays, tmp_path):
    ref = oracle.walk(oracle.Triangulation.of(tiny_scene), tiny_rays.o, tiny_rays.d, tiny_rays.start)
    cache = str(tmp_path / "tune.json")
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        o, d, st = _dev(tiny_rays)
        best, ms = ccsp.autotune([(scene, o, d, st)], reps=1, cache_path=cache)
        assert ms is not None and ms > 0
        assert best.wg_size in (64, 128, 256, 512) and best.tile_rays in (64, 128, 256)
        assert 8 <= best.waves_per_cu <= 28 and best.xcd_chunks in (1, 8)
        # tune=None now uses the tuned parameters; the results do not depend on them
        _assert_same(_host(ccsp.trace(scene, o, d, st)), ref, "after autotune")
        # the JSON file is found again without measuring
        again, ms2 = ccsp.autotune([(scene, o, d, st)], cache_path=cache)
        assert ms2 is None and again.as_tuple() == best.as_tuple()
        parts = [tiny_rays.slice(0, 1000), tiny_rays.slice(1000, 5000), tiny_rays.slice(5000, 5001),
                 tiny_rays.slice(5001, 5001)]
        jobs = [(scene, *_dev(p)) for p in parts]
        bb, bms = ccsp.autotune(jobs, graph=True, reps=1)
        assert bms > 0
        for rep in range(3):
            res = ccsp.trace_batch(jobs, graph=True)
            for p, rs, a in zip(parts, res, (0, 1000, 5000, 5001)):
                _assert_same(_host(rs), tuple(x[a:a + p.n] for x in ref), f"tuned graph {rep}")


def test_concurrent_batches_and_graph_replays_on_two_streams(ccsp, grid_pair):
    """Batches in flight on two streams use separate item tables; replays of one graph on
    alternating streams are ordered."""
    sc, _, rays, _ = grid_pair
    parts = [rays.slice(k * 40_000, (k + 1) * 40_000 + 17 * k) for k in range(6)]
    with ccsp.Scene.from_arrays(sc) as scene:
        devp = [_dev(p) for p in parts]
        refs = [_host(ccsp.trace(scene, *x, input_order=True)) for x in devp]
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        for graph in (False, True):
            outs = []
            for rep in range(4):
                # the two streams alternate between two different item lists
                jobs = [(scene, *devp[k]) for k in ((0, 1, 2) if rep % 2 == 0 else (3, 4, 5))]
                s = s1 if rep % 2 == 0 else s2
                with torch.cuda.stream(s):
                    outs.append((rep, ccsp.trace_batch(jobs, stream=s, graph=graph)))
            torch.cuda.synchronize()
            for rep, res in outs:
                ks = (0, 1, 2) if rep % 2 == 0 else (3, 4, 5)
                for k, rs in zip(ks, res):
                    _assert_same(_host(rs), refs[k], f"graph={graph} rep {rep} item {k}")
        # one graph replayed on alternating streams
        jobs = [(scene, *devp[k]) for k in (0, 1, 2)]
        outs = []
        for rep in range(4):
            s = s1 if rep % 2 == 0 else s2
            with torch.cuda.stream(s):
                outs.append(ccsp.trace_batch(jobs, stream=s, graph=True))
        torch.cuda.synchronize()
        for rep, res in enumerate(outs):
            for k, rs in zip((0, 1, 2), res):
                _assert_same(_host(rs), refs[k], f"same graph rep {rep} item {k}")


def _pinned(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).pin_memory()


def test_server_alone_vs_mix(ccsp, tiny_scene, tiny_rays, grid_pair):
    """Requests of uneven sizes over three scenes, submitted while others run, through a small
    pool (admission waits for memory) and few slots: every result equals the same rays traced
    alone, bit for bit; launches coalesce requests and overlap."""
    sc_grid, sc_ann, grid_rays, start_ann = grid_pair
    scenes = [ccsp.Scene.from_arrays(tiny_scene), ccsp.Scene.from_arrays(sc_grid),
              ccsp.Scene.from_arrays(sc_ann)]
    m = 300_000
    pools = [tiny_rays, grid_rays.slice(0, m),
             sg.Rays(grid_rays.o[:m], grid_rays.d[:m], start_ann[:m])]
    host = [(_pinned(r.o, torch.float64), _pinned(r.d, torch.float64),
             _pinned(r.start, torch.int32)) for r in pools]
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(60):
        s = int(rng.integers(0, 3))
        n = int(np.exp(rng.uniform(np.log(1), np.log(60_000))))
        if k % 17 == 0:
            n = 0
        if 1 <= k <= 3:
            # three requests of 3.4 MB each, submitted back to back, do not fit the 8 MiB pool
            # together: the third waits for memory unless the first has already finished
            s, n = 1, 60_000
        off = int(rng.integers(0, pools[s].n - n + 1))
        reqs.append((s, off, n))
    # outputs allocated before any submission, so that requests arrive back to back
    outs = [ccsp.Result(torch.empty(n, dtype=torch.int32).pin_memory(),
                        torch.empty(n, dtype=torch.float64).pin_memory(),
                        torch.empty(n, dtype=torch.int32).pin_memory()) for _, _, n in reqs]
    try:
        with ccsp.Server(precision="fp32", slots=3, max_items=8, memory_bytes=8 << 20) as srv:
            ids, done = {}, []
            for k, (s, off, n) in enumerate(reqs):
                o, d, st = (x[off:off + n] for x in host[s])
                ids[srv.submit(scenes[s], o, d, st, outs[k])] = k
                if k % 10 == 9:
                    done += srv.poll()
            deadline = 60.0
            while len(done) < len(reqs):
                got = srv.poll(timeout_s=1.0)
                done += got
                deadline -= 1.0 if not got else 0.0
                assert deadline > 0, "server did not finish"
            st = srv.stats()
        assert sorted(ids[i] for i, *_ in done) == list(range(len(reqs)))
        assert all(status == 0 for _, status, *_ in done)
        assert all(t1 >= t0 for _, _, t0, t1 in done)
        assert st["launches"] < st["requests"] and st["max_items_per_launch"] > 1
        assert st["max_slots_busy"] >= 2 and st["admissions_stopped_by_memory"] > 0
        assert st["peak_pool_bytes"] <= 8 << 20
        for k, (s, off, n) in enumerate(reqs):
            o, d, stt = (x[off:off + n].to(DEV) for x in host[s])
            alone = _host(ccsp.trace(scenes[s], o, d, stt, input_order=True))
            got = (outs[k].hit_prim.numpy(), outs[k].hit_t.numpy(), outs[k].steps.numpy())
            _assert_same(got, alone, f"request {k} (scene {s}, {n} rays)")
    finally:
        for s in scenes:
            s.free()


def test_server_rejects_oversized_request(ccsp, tiny_scene, tiny_rays):
    with ccsp.Scene.from_arrays(tiny_scene) as scene, \
            ccsp.Server(memory_bytes=1 << 20) as srv:
        n = 60_000  # needs about 3 MB
        o = torch.zeros((n, 2), dtype=torch.float64)
        st = torch.zeros(n, dtype=torch.int32)
        out = ccsp.Result(torch.empty(n, dtype=torch.int32), torch.empty(n, dtype=torch.float64),
                          torch.empty(n, dtype=torch.int32))
        with pytest.raises(ccsp.CcspError, match="more than the server"):
            srv.submit(scene, o, o, st, out)


def _check_locate(tri_gpu, st_gpu, sc, q, what):
    """Statuses equal the checker's; triangles equal where the answer is unique; where the point
    is on an edge or vertex, the GPU's triangle must contain it in its closure."""
    ref_t, ref_s = oracle.locate(oracle.Triangulation.of(sc), q)
    assert np.array_equal(st_gpu, ref_s), f"{what}: status differs at {np.nonzero(st_gpu != ref_s)[0][:5]}"
    uniq = ref_s != 1
    assert np.array_equal(tri_gpu[uniq], ref_t[uniq]), f"{what}: triangle differs"
    for k in np.nonzero(~uniq)[0]:
        a, b, c = (sc.xy[v] for v in sc.tri_v[tri_gpu[k]])
        assert min(oracle.orient(b, c, q[k]), oracle.orient(c, a, q[k]),
                   oracle.orient(a, b, q[k])) == 0, f"{what}: point {k} not on triangle {tri_gpu[k]}"


def test_locate_tiny_and_degenerate_points(ccsp, tiny_scene, tiny_rays):
    rng = np.random.default_rng(3)
    scenes = [tiny_scene] + [helpers.integer_scene(rng, int(rng.integers(3, 12))) for _ in range(4)]
    for k, sc in enumerate(scenes):
        e = sc.tri_v[:, [0, 1, 1, 2, 2, 0]].reshape(-1, 2)
        mid = 0.5 * (sc.xy[e[:, 0]] + sc.xy[e[:, 1]])  # exact on the integer scenes
        lo, hi = sc.box
        pts = [sc.xy, mid, rng.uniform(lo, hi, (3000, 2)),
               np.array([[lo - 1, lo], [hi + 5, hi], [np.nan, lo], [lo, np.inf], [-1e300, 0.0]])]
        if k == 0:
            pts.append(tiny_rays.o)
        q = np.ascontiguousarray(np.concatenate(pts))
        with ccsp.Scene.from_arrays(sc) as scene:
            t, s = ccsp.locate(scene, torch.from_numpy(q).to(DEV))
            torch.cuda.synchronize()
            _check_locate(t.cpu().numpy(), s.cpu().numpy(), sc, q, f"scene {k}")


def test_locate_ray_origins_at_scale(ccsp, grid_pair):
    sc, an, rays, start_an = grid_pair
    q = torch.from_numpy(rays.o).to(DEV)
    for tri_sc, start in ((sc, rays.start), (an, start_an)):
        with ccsp.Scene.from_arrays(tri_sc) as scene:
            t, s = ccsp.locate(scene, q)
            torch.cuda.synchronize()
            assert (s.cpu().numpy() == 0).all() and np.array_equal(t.cpu().numpy(), start)
    large = sg.make_scene("large")
    r = sg.sample_rays(large, 1 << 22, seed=4)
    with ccsp.Scene.from_arrays(large) as scene:
        t, s = ccsp.locate(scene, torch.from_numpy(r.o).to(DEV))
        torch.cuda.synchronize()
        assert (s.cpu().numpy() == 0).all() and np.array_equal(t.cpu().numpy(), r.start)


def _bounce_host(res, hits, face):
    torch.cuda.synchronize()
    return (res.hit_prim.cpu().numpy(), res.hit_t.cpu().numpy(), res.steps.cpu().numpy(),
            hits.cpu().numpy(), face.cpu().numpy())


def _assert_bounce_same(got, ref, what):
    names = ("prim", "t", "steps", "bounces", "face")
    for name, g, r in zip(names, got, ref):
        bad = np.nonzero(~((g == r) | (np.isinf(g) & np.isinf(r)) if name == "t" else (g == r)))[0]
        assert bad.size == 0, f"{what}: {name} differs at {bad[:5]}: {g[bad[:5]]} vs {r[bad[:5]]}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_bounces_tiny_all_rays(ccsp, tiny_scene, tiny_rays, prec):
    tri = oracle.Triangulation.of(tiny_scene)
    with ccsp.Scene.from_arrays(tiny_scene) as scene:
        o, d, st = _dev(tiny_rays)
        plain = _host(ccsp.trace(scene, o, d, st, precision=prec))
        for mb in (0, 1, 3, 8):
            got = _bounce_host(*ccsp.trace_bounces(scene, o, d, st, mb, precision=prec))
            ref = oracle.bounce(tri, tiny_rays.o, tiny_rays.d, tiny_rays.start, mb)
            _assert_bounce_same(got, ref, f"{prec} max_bounces={mb}")
            if mb == 0:
                _assert_same(got[:3], plain, "zero bounces vs trace")
                hit = got[0] >= 0
                f = got[4][hit]
                assert np.array_equal(tiny_scene.tri_prim[f >> 2, f & 3], got[0][hit])
            else:
                assert (got[3] == mb).mean() > 0.9  # nearly every ray keeps hitting walls


def test_bounces_binned_grid_and_large_sampled(ccsp, grid_pair):
    sc, _, rays, _ = grid_pair
    r = rays.slice(0, 300_000)
    idx = np.arange(0, r.n, 37)
    with ccsp.Scene.from_arrays(sc) as scene:
        o, d, st = _dev(r)
        got = _bounce_host(*ccsp.trace_bounces(scene, o, d, st, 4))
        io = _bounce_host(*ccsp.trace_bounces(scene, o, d, st, 4, input_order=True))
        _assert_bounce_same(got, io, "grid binned vs input order")
        ref = oracle.bounce(oracle.Triangulation.of(sc), r.o[idx], r.d[idx], r.start[idx], 4)
        _assert_bounce_same(tuple(x[idx] for x in got), ref, "grid vs checker")
    large = sg.make_scene("large")
    r = sg.sample_rays(large, 1 << 21, seed=8)
    idx = np.arange(0, r.n, 211)
    with ccsp.Scene.from_arrays(large) as scene:
        o, d, st = _dev(r)
        for prec in ("fp32", "fp64"):
            got = _bounce_host(*ccsp.trace_bounces(scene, o, d, st, 3, precision=prec))
            ref = oracle.bounce(oracle.Triangulation.of(large), r.o[idx], r.d[idx], r.start[idx], 3)
            _assert_bounce_same(tuple(x[idx] for x in got), ref, f"large {prec} vs checker")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_split_primitives(ccsp, seed):
    """Every segment constrained as two sub-edges meeting at its midpoint: the hit reports the
    primitive and t its own segment's parameter, in both modes, with and without continuation;
    point location is exact on the split vertices too."""
    rng = np.random.default_rng(100 + seed)
    split = sg.triangulate(sg.split_segments(helpers.integer_scene(rng, 40, size=48)))
    o, d, start = helpers.degenerate_rays(split, rng, 6000)
    r = sg.Rays(o, d, start.astype(np.int32))
    tri = oracle.Triangulation.of(split)
    ref = oracle.walk(tri, r.o, r.d, r.start)
    with ccsp.Scene.from_arrays(split) as scene:
        dev = _dev(r)
        for prec in ("fp32", "fp64"):
            _assert_same(_host(ccsp.trace(scene, *dev, precision=prec)), ref, f"split {prec}")
            _assert_same(_host(ccsp.trace(scene, *dev, precision=prec, input_order=True)), ref,
                         f"split {prec} input order")
            got = _bounce_host(*ccsp.trace_bounces(scene, *dev, 3, precision=prec))
            _assert_bounce_same(got, oracle.bounce(tri, r.o, r.d, r.start, 3), f"split bounces {prec}")
        q = np.ascontiguousarray(np.concatenate([split.xy, r.o]))
        t, s = ccsp.locate(scene, torch.from_numpy(q).to(DEV))
        torch.cuda.synchronize()
        _check_locate(t.cpu().numpy(), s.cpu().numpy(), split, q, "split")
