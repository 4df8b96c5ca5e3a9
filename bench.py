"""Benchmark: stackless triangulation walk on one MI355X.

Workload: the large clutter scene (10^6 non-crossing segments, midpoints U[0,1000]^2, lengths
log-U[0.01, 1], box [-1,1001]^2, constrained Delaunay triangulation with 4,000,002 triangles) and
2^26 isotropic rays with known start triangles, synthetic and seeded. One step = one trace of all
rays (the whole walk: first triangle, steps, hit distance), inputs resident in HBM.

Prints one JSON line: rays/s of the binary32-filtered walk (value), steps/s, the binary64 walk's
rays/s on the same inputs, the roofline of the walk kernel (its own duration from HIP events the
library records on the trace's stream around it), the dependent-gather roofline measured on this
GPU, and the checker's throughput on the host cores for a bounded sample of the same rays.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
# Algorithmic bytes of the walk kernel: per step the exit word, the across vertex in binary32 and
# its id (16); per ray its input (origin, direction, start triangle: 36), the two first-triangle
# vertices beyond the one a step would read (16), the hit primitive's segment (32) and the parked
# result (16). The whole trace moves the same per-step bytes and 100 B per ray of its own (36 in,
# 16 out, 16 first-triangle vertices, 32 primitive segment).
BYTES_PER_STEP = 16
BYTES_PER_RAY = 100
TRACE_BYTES_PER_RAY = 100

# HBM traffic of one binary32 walk launch on the large workload, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE passes (profiles/walk_fp32_large_pmc.md), each scaled by what the same counter reports
# for a plain copy of known size. Valid only for the kernel sources and launch parameters it was
# taken with.
WALK_SOURCES = ("walk_kernels.hip", "walk.hpp", "decide.hpp", "exact.hpp")
MEASURED_TRAFFIC = {
    "sources_sha256": "e4892b4746b1801658487388c9c7b818be986a3d9f24828c765ffd64c18c9d57",
    "tune": [128, 64, 16, 8, 8, 8, 0],
    "bytes_per_launch": 17194156288,
}


def walk_sources_sha256():
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, "paper_2112_05570_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TUNE_TABLE = os.path.join(ROOT, "paper_2112_05570_amd", "tuned", "mi355x.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large",
                    choices=["large", "grid", "tiny", "batch", "serve", "objective", "flips",
                             "pipeline", "tet3d"],
                    help="batch: the 256-scene workload in one graph-replayed, autotuned launch; "
                         "serve: the request server under Poisson arrivals; objective: the "
                         "low-weight objective on the subdivided large scene; flips: edge-flip "
                         "annealing of the grid scene's CDT; pipeline: the low-weight pipeline "
                         "on the grid scene, walked by its rays")
    ap.add_argument("--requests", type=int, default=10_000, help="serve: requests per level")
    ap.add_argument("--slots", type=int, default=4, help="serve: launch slots")
    ap.add_argument("--tune-cache", default=TUNE_TABLE,
                    help="JSON file of autotuned launch parameters (the library's table for this "
                         "GPU by default); workloads missing from it are tuned by measurement")
    ap.add_argument("--rays", type=int, default=0, help="override the ray count")
    ap.add_argument("--scene", default="grid",
                    help="pipeline: 'grid', or 'lines:N' for N random segments drawn as in the "
                         "large scene")
    ap.add_argument("--pipeline-rounds", type=int, default=1,
                    help="pipeline: rounds of subdivision and optimisation (2 = the iterated "
                         "strategy with one intermediate subdivision)")
    ap.add_argument("--balance-sweeps", type=int, default=0,
                    help="pipeline: sweeps per stage with perturbation types drawn for equal time "
                         "(0: a displacement sweep and the next proposal type in turn)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the checker leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-objective", action="store_true",
                    help="leave out the objective leg (for profiler runs of the walk)")
    ap.add_argument("--no-multi", action="store_true",
                    help="leave out the batch and serving legs of the default run")
    ap.add_argument("--no-tet3d", action="store_true",
                    help="leave out the 3D tetrahedral walk leg of the default run")
    ap.add_argument("--multi-requests", type=int, default=3000,
                    help="requests per load level of the default run's serving leg")
    ap.add_argument("--tune", default="", help="wg,tile,waves_per_cu,refill_min")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for scaling HBM "
                         "counters of a profiler run)")
    ap.add_argument("--gather-sweep", action="store_true",
                    help="only measure the dependent-gather roofline over a range of buffer sizes")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gather_sweep:
        gather_sweep()
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; the walk would shard by "
                                   "replicating the scene on every GPU and splitting the rays",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "objective":
        print(json.dumps(objective_leg("large", args.steps, args.warmup)), flush=True)
        return
    if args.workload == "tet3d":
        print(json.dumps(tet3d_leg(args.steps, args.warmup,
                                   None if args.no_cpu else args.cpu_seconds / 2)), flush=True)
        return
    if args.workload == "pipeline":
        sc = (sg.make_scene("grid", seed=0) if args.scene == "grid"
              else sg.make_scene("large", seed=0, n_seg=int(args.scene.split(":")[1])))
        rays = sg.sample_rays(sc, args.rays or (1 << 20), seed=0)
        from paper_2112_05570_amd import pipeline as pl
        sched = pl.Schedule(balance_sweeps=args.balance_sweeps)
        print(json.dumps(pipeline_leg(sc, rays, verbose=True, schedule=sched,
                                      rounds=args.pipeline_rounds)), flush=True)
        return
    if args.workload == "flips":
        sc = sg.make_scene("grid", seed=0)
        print(json.dumps(flip_leg(sc, args.steps)[2]), flush=True)
        return
    dev = torch.device("cuda:0")
    t0 = time.time()
    sc = sg.make_scene(args.workload, seed=0)
    n = args.rays or sg.WORKLOADS[args.workload]["rays"]
    rays = sg.sample_rays(sc, n, seed=0)
    log(f"[bench] {args.workload}: {sc.n_prims} prims, {sc.n_triangles} triangles, {n} rays "
        f"built in {time.time() - t0:.1f}s")
    o = torch.from_numpy(rays.o).to(dev)
    d = torch.from_numpy(rays.d).to(dev)
    st = torch.from_numpy(rays.start).to(dev)
    scene = ccsp.Scene.from_arrays(sc)
    tune = None
    if args.tune:
        tune = ccsp.TuneParams(*[int(x) for x in args.tune.split(",")])
    out32 = ccsp.Result(torch.empty(n, dtype=torch.int32, device=dev),
                        torch.empty(n, dtype=torch.float64, device=dev),
                        torch.empty(n, dtype=torch.int32, device=dev))
    out64 = ccsp.Result(torch.empty_like(out32.hit_prim), torch.empty_like(out32.hit_t),
                        torch.empty_like(out32.steps))
    stream = torch.cuda.current_stream()
    tuned = {}
    if tune is None:
        # launch parameters from the library's autotuner (kept in its cache; tune=None below)
        for prec, out in (("fp32", out32), ("fp64", out64)):
            t_tune = time.perf_counter()
            best, _ = ccsp.autotune([(scene, o, d, st, out)], prec, reps=2,
                                    cache_path=args.tune_cache)
            tuned[prec] = best.as_tuple()
            log(f"[bench] autotune {prec}: {tuned[prec]} in {time.perf_counter() - t_tune:.1f}s")

    def timed(prec, out, k, w):
        for _ in range(w):
            ccsp.trace(scene, o, d, st, precision=prec, out=out, tune=tune, stream=stream)
        torch.cuda.synchronize()
        ccsp.read_stage_times()  # forget older records
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k)]
        t = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            ccsp.trace(scene, o, d, st, precision=prec, out=out, tune=tune, stream=stream,
                       timed=True)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        trace_s = [a.elapsed_time(b) / 1e3 for a, b in evs]
        bin_ms, walk_ms, fin_ms = ccsp.read_stage_times(k)
        assert len(walk_ms) == k
        return (wall, trace_s, [x / 1e3 for x in bin_ms], [x / 1e3 for x in walk_ms],
                [x / 1e3 for x in fin_ms])

    wall32, tr32, bin32, walk32, fin32 = timed("fp32", out32, args.steps, args.warmup)
    log(f"[bench] fp32 walk: {args.steps} steps in {wall32:.3f}s")
    wall64, tr64, bin64, walk64, fin64 = timed("fp64", out64, max(1, args.steps // 2), 1)
    log(f"[bench] fp64 walk: {len(tr64)} steps in {wall64:.3f}s")
    # the same walk without ray binning (rays walked in input order), for comparison
    for _ in range(1):
        ccsp.trace(scene, o, d, st, precision="fp32", out=out64, tune=tune, input_order=True)
    torch.cuda.synchronize()
    t_io = time.perf_counter()
    k_io = max(1, args.steps // 2)
    for _ in range(k_io):
        ccsp.trace(scene, o, d, st, precision="fp32", out=out64, tune=tune, input_order=True)
    torch.cuda.synchronize()
    ms_io = (time.perf_counter() - t_io) / k_io * 1e3

    # continued rays: up to 4 specular reflections per ray (Sec. 5.2 secondary rays)
    ccsp.trace_bounces(scene, o, d, st, 4)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    for _ in range(3):
        b_res, b_hits, _ = ccsp.trace_bounces(scene, o, d, st, 4)
    torch.cuda.synchronize()
    ms_bounce = (time.perf_counter() - t_b) / 3 * 1e3
    b_segments = n + int(b_hits.sum(dtype=torch.int64).item())
    b_steps = int(b_res.steps.sum(dtype=torch.int64).item())
    del b_res, b_hits

    # point location of the same origins (Sec. 5.2), timed on its own
    ccsp.locate(scene, o)
    torch.cuda.synchronize()
    t_loc = time.perf_counter()
    for _ in range(3):
        loc_tri, loc_st = ccsp.locate(scene, o)
    torch.cuda.synchronize()
    ms_locate = (time.perf_counter() - t_loc) / 3 * 1e3
    locate_ok = bool(torch.equal(loc_tri, st) and int((loc_st != 0).sum().item()) == 0)
    del loc_tri, loc_st

    # diagnostics outside the timed region
    steps_total = int(out32.steps.sum(dtype=torch.int64).item())
    # dependent loads of the binned walk: binning decides the first triangle, and each 32-B
    # record load then advances up to two steps, so a ray of k steps makes (k + 1) // 2 loads
    loads_total = int(((out32.steps.to(torch.int64) + 1) // 2).sum().item())
    steps_p99 = float(torch.quantile(out32.steps[: 1 << 24].double(), 0.99).item())
    t32_err = pure_binary32_t_error(sc, o, d, out32, torch)
    same = bool(torch.equal(out32.hit_prim, out64.hit_prim) and torch.equal(out32.steps, out64.steps)
                and torch.equal(out32.hit_t, out64.hit_t))
    ccsp.read_counters(reset=True)
    ccsp.trace(scene, o, d, st, precision="fp32", out=out64, count=True, tune=tune)
    c_steps, c_fb32, c_fb64, c_rays = ccsp.read_counters(reset=True)
    hp = out32.hit_prim
    n_bad = int((hp < 0).sum().item())

    ms = wall32 / args.steps * 1e3
    rays_s = n * args.steps / wall32
    walk_avg = float(np.mean(walk32))
    alg_bytes = BYTES_PER_STEP * steps_total + BYTES_PER_RAY * n
    achieved = alg_bytes / walk_avg / 1e9
    traffic = None
    if MEASURED_TRAFFIC["sources_sha256"] == walk_sources_sha256() and args.workload == "large" \
            and not args.rays and list(tuned.get("fp32", ())) == MEASURED_TRAFFIC["tune"]:
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]

    # dependent-gather roofline: 16-byte pointer chases over the walk's binary32 slot array size
    # and over an L2-sized buffer (what one XCD's share of binned rays touches at a time)
    ws_bytes = 48 * sc.n_triangles
    from paper_2112_05570_amd import binding as B
    g_scene = B.gather_roofline(ws_bytes, 16, 2048, stream.cuda_stream)
    g_l2 = B.gather_roofline(2 << 20, 16, 2048, stream.cuda_stream)
    walk_steps_s = steps_total / walk_avg
    walk_loads_s = loads_total / walk_avg

    objective = None if args.no_objective else objective_leg("grid", args.steps, args.warmup)
    low_weight = None
    if args.workload == "large" and not args.no_objective:
        low_weight = low_weight_leg(sc, scene, o, d, out32, args.steps)
    triangulations = None
    if args.workload == "grid":
        triangulations = grid_triangulations(sc, rays, scene, o, d, st, out32, args.steps)

    batch = serve = None
    if args.workload == "large" and not args.no_multi:
        del out64
        batch = batch_leg(3, 1, args.tune_cache)
        serve = serve_leg(args.multi_requests, args.slots)

    tet3d = None
    if args.workload == "large" and not args.no_tet3d:
        tet3d = tet3d_leg(args.steps, args.warmup, None if args.no_cpu else args.cpu_seconds / 2)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_leg(sc, rays, args.cpu_seconds)

    line = {
        "metric": "rays/s and traversal steps/s on 1 MI355X (FP32+filter vs FP64); p99 latency",
        "value": rays_s,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {sc.n_prims - 4} segments + 4 box sides, "
                        f"{sc.n_triangles} CDT triangles, {n} isotropic rays, seed 0",
            "rays": n, "triangles": sc.n_triangles, "primitives": sc.n_prims,
            "precision": "fp32 filtered, fp64 exact fallback",
        },
        "steps_per_s": steps_total * args.steps / wall32,
        "mean_steps_per_ray": steps_total / n,
        "p99_steps_per_ray": steps_p99,
        "pure_binary32_t_rel_error": t32_err,
        "ms_per_step_median": float(np.median(tr32)) * 1e3,
        "stages_ms": {"binning": float(np.mean(bin32)) * 1e3, "walk": walk_avg * 1e3,
                      "walk_median": float(np.median(walk32)) * 1e3,
                      "finish": float(np.mean(fin32)) * 1e3},
        "fp64": {"rays_per_s": n * len(tr64) / wall64, "ms_per_step": wall64 / len(tr64) * 1e3,
                 "steps_per_s": steps_total * len(tr64) / wall64,
                 "stages_ms": {"binning": float(np.mean(bin64)) * 1e3,
                               "walk": float(np.mean(walk64)) * 1e3,
                               "finish": float(np.mean(fin64)) * 1e3}},
        "fp32_input_order_ms_per_step": ms_io,
        "bounces": {"max_bounces": 4, "ms": ms_bounce, "rays_per_s": n / ms_bounce * 1e3,
                    "segments_per_s": b_segments / ms_bounce * 1e3,
                    "steps_per_s": b_steps / ms_bounce * 1e3},
        "locate": {"points_per_s": n / ms_locate * 1e3, "ms": ms_locate,
                   "equals_start_triangles": locate_ok},
        "tuned": {k: dict(zip(["wg_size", "tile_rays", "waves_per_cu", "refill_min",
                               "tiles_per_claim", "xcd_chunks", "bin"], v))
                  for k, v in tuned.items()},
        "fp32_equals_fp64": same,
        "fallback": {"fp32_to_fp64_per_step": c_fb32 / max(1, c_steps),
                     "fp64_to_exact_per_step": c_fb64 / max(1, c_steps)},
        "rays_not_hit": n_bad,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "walk_persistent (binary32)", "kernel_ms": walk_avg * 1e3,
                     "bytes_per_launch": alg_bytes,
                     "bytes_model": f"{BYTES_PER_STEP} B/step + {BYTES_PER_RAY} B/ray (algorithmic)",
                     "measured_GBs": (traffic / walk_avg / 1e9) if traffic else None,
                     "measured_frac": (traffic / walk_avg / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "note": "achieved counts algorithmic bytes, which caches partly serve; "
                             "measured_GBs is the rocprofv3 HBM traffic over the same time"},
        "trace_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "bytes_per_trace": BYTES_PER_STEP * steps_total + TRACE_BYTES_PER_RAY * n,
            "achieved": (BYTES_PER_STEP * steps_total + TRACE_BYTES_PER_RAY * n) / (ms / 1e3) / 1e9,
            "frac": (BYTES_PER_STEP * steps_total + TRACE_BYTES_PER_RAY * n) / (ms / 1e3) / 1e9
                    / HBM_PEAK_GBS,
            "what": "whole trace (binning, walk, copy) per step of the benchmark"},
        "gather_roofline": {
            "walk_steps_per_s": walk_steps_s, "walk_loads_per_s": walk_loads_s,
            "loads_per_ray": loads_total / n,
            "chase_loads_per_s_scene_sized": g_scene, "scene_sized_bytes": ws_bytes,
            "frac_scene_sized_per_load": walk_loads_s / g_scene,
            "chase_loads_per_s_l2_sized": g_l2, "l2_sized_bytes": 2 << 20,
            "frac_l2_sized_per_load": walk_loads_s / g_l2,
            "note": "one 32-B record load advances up to two steps; fractions compare loads "
                    "with the chase's loads"},
        "batch": batch,
        "serve": serve,
        "latency": None if serve is None else {
            "source": "serve leg, Poisson arrivals at 50% of capacity",
            "p50_ms": serve["levels"][1]["p50_ms"], "p99_ms": serve["levels"][1]["p99_ms"]},
        "objective": objective,
        "triangulations": triangulations,
        "low_weight": low_weight,
        "tet3d": tet3d,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    scene.free()


def subdivided(sc):
    """The scene's CDT subdivided once (Sec. 3.5.2) by the library (mesh_subdivide)."""
    from types import SimpleNamespace

    import paper_2112_05570_amd as ccsp
    import scenegen as sg
    xy, tv, kd, ln, pv = sg.movable_input(sc)
    tv, kd, ln, pv, xy = ccsp.subdivide(tv, kd, ln, pv, xy)
    return SimpleNamespace(xy=xy, tri_v=tv, kind=kd, line=ln, prim_v=pv, n_vertices=xy.shape[0],
                           n_triangles=tv.shape[0], name=sc.name + "/4")


def flip_leg(sc, steps, hot=300, cold=100, t0_rel=5e-3, t1_rel=1e-5, seed=0):
    """GPU edge-flip annealing (flip_anneal) of a scene's CDT with the weight as energy: `hot`
    rounds at temperatures falling geometrically from t0_rel to t1_rel of the box side, then
    `cold` rounds at 0. Each timed run starts from a fresh copy of the CDT (copied outside the
    timed region). The scene generator's sequential flip annealer is timed beside it for
    context. Returns (annealed Scene, results)."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    side = sc.box[1] - sc.box[0]
    temps = list(side * np.geomspace(t0_rel, t1_rel, hot)) + [0.0] * cold
    xy = torch.from_numpy(np.ascontiguousarray(sc.xy)).cuda()
    base = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
            for a in (sc.tri_v, sc.tri_nbr, sc.tri_prim)]
    times = []
    for _ in range(max(1, steps)):
        arrs = [a.clone() for a in base]
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        counts = ccsp.flip_anneal(xy, *arrs, temps, seed)  # synchronous
        times.append((time.perf_counter() - t_s) * 1e3)
    an = sc.copy_with(*[a.cpu().numpy() for a in arrs], name=sc.name + "/gpu-annealed")
    t_s = time.perf_counter()
    host, host_stats = sg.anneal_flips(sc, seed=0)
    host_s = time.perf_counter() - t_s
    ms = float(np.median(times))
    res = {"rounds": len(temps), "hot_rounds": hot, "temperature": [temps[0], temps[hot - 1]],
           "ms": ms, "us_per_round": ms * 1e3 / len(temps), "flips": int(counts.sum()),
           "last_round_with_flips": int(np.nonzero(counts)[0][-1]),
           "weight_cdt": sg.weight(sc), "weight": sg.weight(an),
           "host_sequential": {"s": host_s, "weight": sg.weight(host),
                               "proposals": int(host_stats["proposals"])}}
    return an, host, res


def low_weight_leg(sc, scene, o, d, out, steps, hot=300, cold=100, seed=0):
    """The paper's claim on this workload: the scene's CDT flip-annealed on the GPU with the
    weight as energy (flip_anneal; temperatures from 2.5 to 0.005 mean edge lengths over `hot`
    rounds, then `cold` rounds at 0), the rays' origins located in the result by the library's
    point location, and the same rays walked on it. `out` holds the CDT trace of these rays."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    from paper_2112_05570_amd import pipeline as pl

    w0 = pl.weight(sc.tri_v, sc.xy)
    mean_len = w0 / (sc.n_vertices + sc.n_triangles - 1)  # Euler: E = V + T - 1
    temps = list(mean_len * np.geomspace(2.5, 0.005, hot)) + [0.0] * cold
    xy = torch.from_numpy(np.ascontiguousarray(sc.xy)).to(o.device)
    arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(o.device)
            for a in (sc.tri_v, sc.tri_nbr, sc.tri_prim)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = ccsp.flip_anneal(xy, *arrs, temps, seed)
    ms_anneal = (time.perf_counter() - t0) * 1e3
    tv, nbr, prim = (a.cpu().numpy() for a in arrs)
    del arrs
    res = {"anneal": {"rounds": len(temps), "ms": ms_anneal, "flips": int(counts.sum()),
                      "last_round_with_flips": int(np.nonzero(counts)[0][-1])},
           "weight_cdt": w0, "weight": pl.weight(tv, sc.xy)}
    with ccsp.Scene(sc.xy, tv, nbr, prim, sc.prims) as an:
        st, stat = ccsp.locate(an, o)
        keep = torch.nonzero(stat == 0).squeeze(1)
        full = keep.shape[0] == o.shape[0]
        oo = o if full else o[keep].contiguous()
        dd = d if full else d[keep].contiguous()
        st = st if full else st[keep].contiguous()
        r = ccsp.trace(an, oo, dd, st, precision="fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ccsp.trace(an, oo, dd, st, precision="fp32", out=r)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        cdt_prim = out.hit_prim if full else out.hit_prim[keep]
        cdt_t = out.hit_t if full else out.hit_t[keep]
        cdt_steps = out.steps if full else out.steps[keep]
        res.update({"rays": int(oo.shape[0]), "ms_per_trace": ms,
                    "rays_per_s": oo.shape[0] / ms * 1e3,
                    "mean_steps_per_ray": float(r.steps.double().mean().item()),
                    "mean_steps_per_ray_cdt": float(cdt_steps.double().mean().item()),
                    "hits_identical": bool(torch.equal(r.hit_prim, cdt_prim)
                                           and torch.equal(r.hit_t, cdt_t))})
        del r
    return res


def grid_triangulations(sc, rays, scene, o, d, st, out, steps):
    """The grid scene's CDT and its low-weight triangulations by edge-flip annealing (the paper's
    claim: lower weight, fewer traversal steps), walked by the same rays: weight, mean steps per
    ray and rays/s. Annealed by the GPU (flip_anneal) and by the scene generator's sequential
    annealer."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    gpu_an, host_an, flips = flip_leg(sc, steps)
    res = {"flip_anneal": flips}
    hits = {}
    for name, sc_ in (("cdt", sc), ("gpu_annealed", gpu_an), ("host_annealed", host_an)):
        if name == "cdt":
            tri, s = scene, st
        else:
            start = sg.locate(sc_, rays.o)
            assert (start >= 0).all()
            s = torch.from_numpy(start.astype(np.int32)).to(o.device)
            tri = ccsp.Scene.from_arrays(sc_)
        try:
            ccsp.trace(tri, o, d, s, precision="fp32", out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ccsp.trace(tri, o, d, s, precision="fp32", out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
        finally:
            if tri is not scene:
                tri.free()
        res[name] = {"triangles": sc_.n_triangles, "weight": sg.weight(sc_),
                     "mean_steps_per_ray": float(out.steps.double().mean().item()),
                     "rays_per_s": rays.n / ms * 1e3, "ms_per_trace": ms}
        hits[name] = (out.hit_prim.clone(), out.hit_t.clone())
    res["hits_identical"] = all(torch.equal(hits["cdt"][0], h[0]) and torch.equal(hits["cdt"][1], h[1])
                                for h in hits.values())
    return res


def pipeline_leg(sc, rays, stages=24, verbose=False, schedule=None, rounds=1):
    """The paper's low-weight pipeline on a scene (``paper_2112_05570_amd.pipeline.optimise``:
    annealing with every single-vertex proposal, contraction, polishing and greedy flips, raised
    contraction lengths) from its CDT subdivided once (Sec. 3.5.2), then the CDT and the result
    walked by the same rays (origins located in the result by the library's point location).
    Returns weights, counts, times and the walk comparison: steps per ray, trace time, the share
    of rays hitting the same original primitive, and the largest relative difference of t (the
    result's constrained edges are sub-segments of the primitives, collinear to rounding). With
    rounds > 1, the iterated strategy of Sec. 3.5.3 (``pipeline.optimise_iterated``) from the CDT,
    reporting the lightest round and each round's weight."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg
    from paper_2112_05570_amd import pipeline as pl

    size = sc.box[1] - sc.box[0]
    t0 = time.perf_counter()
    mesh = subdivided(sc)
    t_sub = time.perf_counter() - t0
    if rounds > 1:
        xy0, tv0, kd0, ln0, pv0 = sg.movable_input(sc)
        r = pl.optimise_iterated(tv0, kd0, ln0, pv0, xy0, size,
                                 schedule or pl.Schedule(stages=stages), rounds, verbose=verbose)
    else:
        r = pl.optimise(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v, mesh.xy, size,
                        schedule or pl.Schedule(stages=stages), verbose=verbose)
    res = {"subdivided": {"vertices": mesh.n_vertices, "triangles": mesh.n_triangles,
                          "weight": r.log["weight_start"], "subdivide_s": t_sub},
           "stages": stages, "anneal_s": r.log["anneal_s"],
           "weight_annealed": r.log["weight_annealed"],
           "contract_polish_s": r.log["contract_polish_s"],
           "contract_polish": r.log["contract_polish"],
           "final": {"vertices": int(r.xy.shape[0]), "triangles": int(r.tri_v.shape[0]),
                     "steiner_vertices": int((r.kind != 0).sum()), "weight": r.log["weight_final"]},
           "total_s": time.perf_counter() - t0}
    if "balance" in r.log:
        res["balance"] = r.log["balance"]
    if rounds > 1:
        res["rounds"] = [{"subdivided_vertices": g["subdivided_vertices"],
                          "vertices": g["vertices"], "weight": g["weight_final"],
                          "anneal_s": g["anneal_s"], "contract_polish_s": g["contract_polish_s"]}
                         for g in r.log["rounds"]]
        res["rounds_stopped"] = r.log["stopped"]
    nbr, prim, prims, sub_to_orig = pl.walk_arrays(r.tri_v, r.kind, r.line, mesh.prim_v, r.xy)
    dev = torch.device("cuda:0")
    o = torch.from_numpy(rays.o).to(dev)
    d = torch.from_numpy(rays.d).to(dev)
    walks = {}
    with ccsp.Scene(sc.xy, sc.tri_v, sc.tri_nbr, sc.tri_prim, sc.prims) as s_cdt, \
            ccsp.Scene(r.xy, r.tri_v, nbr, prim, prims) as s_opt:
        st_opt, stat = ccsp.locate(s_opt, o)
        keep = torch.nonzero(stat == 0).squeeze(1)
        o, d = o[keep].contiguous(), d[keep].contiguous()
        st_cdt = torch.from_numpy(rays.start).to(dev)[keep].contiguous()
        st_opt = st_opt[keep].contiguous()
        for name, scene, st in (("cdt", s_cdt, st_cdt), ("pipeline", s_opt, st_opt)):
            out = ccsp.trace(scene, o, d, st, precision="fp32")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                out = ccsp.trace(scene, o, d, st, precision="fp32", out=out)
            torch.cuda.synchronize()
            walks[name] = (out.hit_prim.cpu().numpy(), out.hit_t.cpu().numpy(),
                           out.steps.cpu().numpy(), (time.perf_counter() - t1) / 5 * 1e3)
    # flip-only annealing of the same CDT (flip_anneal, as in the low-weight leg), walked too
    w_cdt = pl.weight(sc.tri_v, sc.xy)
    mean_len = w_cdt / (sc.n_vertices + sc.n_triangles - 1)
    temps = list(mean_len * np.geomspace(2.5, 0.005, 300)) + [0.0] * 100
    fxy = torch.from_numpy(np.ascontiguousarray(sc.xy)).to(dev)
    farr = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
            for a in (sc.tri_v, sc.tri_nbr, sc.tri_prim)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ccsp.flip_anneal(fxy, *farr, temps, 0)
    ms_flip = (time.perf_counter() - t1) * 1e3
    ftv, fnbr, fprim = (a.cpu().numpy() for a in farr)
    with ccsp.Scene(sc.xy, ftv, fnbr, fprim, sc.prims) as s_flip:
        st_f, stat_f = ccsp.locate(s_flip, o)
        okf = bool((stat_f == 0).all().item())
        out = ccsp.trace(s_flip, o, d, st_f, precision="fp32") if okf else None
        torch.cuda.synchronize()
        flip_only = {"weight": pl.weight(ftv, sc.xy), "anneal_ms": ms_flip,
                     "mean_steps_per_ray": float(out.steps.double().mean().item()) if okf else None,
                     "hits_identical": bool(torch.equal(out.hit_prim.cpu(),
                                                        torch.from_numpy(walks["cdt"][0])))
                     if okf else None}
    hp = walks["pipeline"][0]
    mapped = np.where(hp >= 0, sub_to_orig[np.maximum(hp, 0)], hp)
    same = mapped == walks["cdt"][0]
    tc, tp = walks["cdt"][1][same], walks["pipeline"][1][same]
    fin = np.isfinite(tc)
    rel = np.abs(tp[fin] - tc[fin]) / np.abs(tc[fin])
    res["walk"] = {"rays": int(o.shape[0]),
                   "cdt": {"weight": sg.weight(sc), "triangles": sc.n_triangles,
                           "mean_steps_per_ray": float(walks["cdt"][2].mean()),
                           "ms_per_trace": walks["cdt"][3]},
                   "pipeline": {"weight": r.log["weight_final"], "triangles": int(r.tri_v.shape[0]),
                                "mean_steps_per_ray": float(walks["pipeline"][2].mean()),
                                "ms_per_trace": walks["pipeline"][3]},
                   "flip_only": flip_only,
                   "same_primitive_hit": float(same.mean()),
                   "max_rel_t_difference": float(rel.max(initial=0.0))}
    return res


# Compulsory bytes of one objective evaluation (every array read once, scratch written and read
# back once): per vertex 16 (caller's position) + 4 (its internal slot) + 16 + 16 (position in
# internal order, written and read) + 8 (kind, line); per ORIGINAL vertex 16 (the position staged
# by the previous call, compared to find out whether the rule bits still hold); per edge 8 (ends)
# + 8 (opposite vertices) + 16 (neighbouring edges) + 4 (its 1-hop list offset) + 1 (rule bits)
# + 17 (length, c and contractibility written) + 17 (read back); per triangle 16 (vertices).
OBJ_BYTES_PER_VERTEX, OBJ_BYTES_PER_ORIGINAL, OBJ_BYTES_PER_EDGE, OBJ_BYTES_PER_TRIANGLE = (
    60, 16, 71, 16)


def objective_leg(scene_name, steps, warmup, moves=1 << 20):
    """The low-weight objective (Sec. 2.2) on a scene's CDT subdivided once (Sec. 3.5.2): full
    evaluations and batches of single-vertex moves (Sec. 3.2.2), parameters of the paper scaled from
    the unit square to the scene (eps = 1e-3 of its size, a point of the annealing schedule)."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    t0 = time.time()
    sc = sg.make_scene(scene_name, seed=0)
    mesh = subdivided(sc)
    size = sc.box[1] - sc.box[0]
    gm = ccsp.MovableMesh.from_mesh(mesh)
    log(f"[bench] objective on {mesh.name}: {mesh.n_vertices} vertices, {gm.n_edges} edges, "
        f"{mesh.n_triangles} triangles ({time.time() - t0:.1f}s to build)")
    p = ccsp.objective_params(1e-3 * size, None, 1e-10 * size, 1.0 * size, 10.0 * size)
    xy = torch.from_numpy(mesh.xy).cuda()
    v, q = sg.vertex_moves(mesh, moves, 0, 0.05)
    vid = torch.from_numpy(v).cuda()
    qd = torch.from_numpy(q).cuda()

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k, r

    ms_eval, out = timed(lambda: gm.eval(xy, p), steps, warmup)
    ms_delta, (d, st) = timed(lambda: gm.delta(xy, p, vid, qd), max(1, steps // 2), 1)
    # the same moves submitted in vertex order (neighbouring threads then share cache lines)
    srt = torch.argsort(vid)
    vid_s, q_s = vid[srt].contiguous(), qd[srt].contiguous()
    ms_delta_sorted, _ = timed(lambda: gm.delta(xy, p, vid_s, q_s), max(1, steps // 2), 1)
    log(f"[bench] objective: eval {ms_eval:.3f} ms, {moves} changes of f {ms_delta:.2f} ms")
    f, wc, pa, pl = out.cpu().tolist()
    ok = int((st == 1).sum().item())

    # Metropolis sweeps (Sec. 3.1): every movable vertex once per sweep, class by class, moves of
    # Sec. 3.2.2 with eta from the starting positions, at a fixed point of the schedule
    t1 = time.time()
    classes = gm.classes()
    t_classes = time.time() - t1
    order = torch.from_numpy(np.concatenate(classes).astype(np.int64)).cuda()
    n_mov = int(order.shape[0])
    tri = torch.from_numpy(mesh.tri_v.astype(np.int64)).cuda()
    pt = xy[tri]
    area = 0.5 * ((pt[:, 1, 0] - pt[:, 0, 0]) * (pt[:, 2, 1] - pt[:, 0, 1])
                  - (pt[:, 1, 1] - pt[:, 0, 1]) * (pt[:, 2, 0] - pt[:, 0, 0]))
    star = torch.zeros(mesh.n_vertices, dtype=torch.float64, device=xy.device)
    star.index_add_(0, tri.reshape(-1), area.repeat_interleave(3))
    eta = torch.sqrt(star[order]) * 0.05
    gen = torch.Generator(device=xy.device)
    gen.manual_seed(0)
    n_sweeps = max(2, steps // 2)
    draws = []
    for _ in range(n_sweeps + 1):
        r = torch.rand((n_mov, 3), generator=gen, device=xy.device, dtype=torch.float64)
        rad = torch.sqrt(r[:, 0]) * (1.0 - r[:, 2]) ** -2.0 * eta
        th = 2.0 * np.pi * r[:, 1]
        disp = torch.stack([rad * torch.cos(th), rad * torch.sin(th)], 1).contiguous()
        draws.append((disp, torch.rand(n_mov, generator=gen, device=xy.device,
                                       dtype=torch.float64)))
    X = xy.clone()
    temperature = 1e-3 * size
    gm.sweep(X, p, temperature, *draws[0])  # warm-up sweep
    f_before = gm.eval(X, p).cpu().tolist()[0]
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    accepted = torch.zeros((), dtype=torch.int64, device=xy.device)
    a.record()
    for k in range(n_sweeps):
        _, sst = gm.sweep(X, p, temperature, *draws[k + 1])
        accepted += (sst == 1).sum()
    b.record()
    torch.cuda.synchronize()
    ms_sweep = a.elapsed_time(b) / n_sweeps
    log(f"[bench] objective: displacement sweep {ms_sweep:.1f} ms")
    f_after = gm.eval(X, p).cpu().tolist()[0]
    del draws

    # sweeps of the proposals of Secs. 3.2.4-3.2.6 from the state the displacement sweeps left
    proposals = {}
    for kind in ("resample", "swap", "contract"):
        r = torch.rand((n_mov, 4), generator=gen, device=xy.device, dtype=torch.float64)
        if kind == "swap":
            rad = torch.sqrt(torch.rand(n_mov, generator=gen, device=xy.device,
                                        dtype=torch.float64))
            th = 2.0 * np.pi * torch.rand(n_mov, generator=gen, device=xy.device,
                                          dtype=torch.float64)
            r[:, 2], r[:, 3] = rad * torch.cos(th), rad * torch.sin(th)
        uk = torch.rand(n_mov, generator=gen, device=xy.device, dtype=torch.float64)
        XP = X.clone()
        f0k = gm.eval(XP, p).cpu().tolist()[0]
        torch.cuda.synchronize()
        a.record()
        _, pst = gm.propose(XP, p, temperature, kind, r, uk)
        b.record()
        torch.cuda.synchronize()
        ms_k = a.elapsed_time(b)
        log(f"[bench] objective: {kind} sweep {ms_k:.1f} ms")
        cnt = torch.bincount((pst + 2).long(), minlength=6).cpu().tolist()  # codes -2 .. 3
        proposals[kind] = {"sweep_ms": ms_k, "vertex_moves_per_s": n_mov / ms_k * 1e3,
                           "accepted": cnt[3], "rejected": cnt[4], "skipped": cnt[5],
                           "folded": cnt[2], "f_before": f0k,
                           "f_after": gm.eval(XP, p).cpu().tolist()[0]}
        del XP
    # group moves (Sec. 3.2.3): GROUP_CENTRES movable vertices drawn at random as centres, in
    # rounds of independent groups (the paper picks a group move's centre at random among the
    # vertices; a sweep over every vertex is not a step of its method)
    n_g = min(n_mov, GROUP_CENTRES)
    cen = gm.movable[np.sort(np.random.default_rng(7).choice(n_mov, n_g, replace=False))]
    r = torch.rand((n_g, 4), generator=gen, device=xy.device, dtype=torch.float64)
    rad = torch.sqrt(r[:, 0]) * (1.0 - r[:, 1]) ** -2.0
    th = 2.0 * np.pi * torch.rand(n_g, generator=gen, device=xy.device, dtype=torch.float64)
    r[:, 0], r[:, 1] = rad * torch.cos(th), rad * torch.sin(th)
    uk = torch.rand(n_g, generator=gen, device=xy.device, dtype=torch.float64)
    XP = X.clone()
    torch.cuda.synchronize()
    a.record()
    _, gst, gmem, grnd = gm.group_sweep(XP, p, temperature, 0.05, r, uk, centres=cen)
    b.record()
    torch.cuda.synchronize()
    ms_g = a.elapsed_time(b)
    log(f"[bench] objective: group sweep of {n_g} centres {ms_g:.1f} ms, "
        f"{int(grnd.max().item()) + 1} rounds")
    proposals["group"] = {"centres": n_g, "sweep_ms": ms_g, "vertex_moves_per_s": n_g / ms_g * 1e3,
                          "rounds": int(grnd.max().item()) + 1,
                          "max_group_size": int(gmem.max().item()),
                          "accepted": int((gst == 1).sum().item()),
                          "rejected": int((gst == 2).sum().item()),
                          "folded": int((gst == 0).sum().item()),
                          "mean_group_size": float(gmem.double().mean().item()),
                          "f_after": gm.eval(XP, p).cpu().tolist()[0]}
    del XP
    # joint moves (the second variant of Sec. 3.2.2): 2% of the movable vertices at once, one
    # Metropolis decision per move on the sum of every term's change; the step scale is far
    # below the single moves' (a joint move folds when any of its vertices does)
    n_j, jsteps = max(1, n_mov // 50), 8
    jrng = np.random.default_rng(9)
    XP = X.clone()
    jst = []
    t_j = time.perf_counter()
    for _ in range(jsteps):
        jv = torch.from_numpy(gm.movable[jrng.choice(n_mov, n_j, replace=False)]).to(xy.device)
        jx = torch.from_numpy(jrng.standard_normal((n_j, 2))).to(xy.device)
        jst.append(gm.joint(XP, p, temperature, 1e-5, jv, jx, float(jrng.random()))[1])
    ms_j = (time.perf_counter() - t_j) * 1e3 / jsteps
    log(f"[bench] objective: joint move of {n_j} vertices {ms_j:.2f} ms")
    proposals["joint"] = {"vertices": n_j, "ms_per_move": ms_j, "steps": jsteps,
                          "accepted": jst.count(1), "rejected": jst.count(2),
                          "folded": jst.count(0)}
    del XP

    # an annealing schedule (Secs. 3.2, 3.3.1): temperature and contraction length lowered together
    # by a factor of 10 over the sweeps, step scale adapted toward 23% acceptance
    n_sched = 10 if scene_name == "large" else 4
    ratio = np.geomspace(1.0, 0.1, n_sched)
    temps = 1e-3 * size * ratio
    epss = 1e-3 * size * ratio
    r1 = torch.sqrt(torch.rand((n_sched, n_mov), generator=gen, device=xy.device, dtype=torch.float64))
    th = 2.0 * np.pi * torch.rand((n_sched, n_mov), generator=gen, device=xy.device,
                                  dtype=torch.float64)
    fac = (1.0 - torch.rand((n_sched, n_mov), generator=gen, device=xy.device,
                            dtype=torch.float64)) ** -2.0
    xi = torch.stack([r1 * fac * torch.cos(th), r1 * fac * torch.sin(th)], -1).contiguous()
    us = torch.rand((n_sched, n_mov), generator=gen, device=xy.device, dtype=torch.float64)
    XS = xy.clone()
    start = gm.eval(XS, p).cpu().tolist()
    t_s = time.perf_counter()
    lam, acc = gm.schedule(XS, p, temps, epss, 0.05, xi, us)
    ms_sched = (time.perf_counter() - t_s) * 1e3
    p_end = ccsp.objective_params(epss[-1], None, 1e-10 * size, 1.0 * size, 10.0 * size)
    end = gm.eval(XS, p_end).cpu().tolist()
    start_at_end_eps = gm.eval(xy, p_end).cpu().tolist()
    del xi, us
    comp = (OBJ_BYTES_PER_VERTEX * mesh.n_vertices
            + OBJ_BYTES_PER_ORIGINAL * int((mesh.kind == sg.ORIGINAL).sum())
            + OBJ_BYTES_PER_EDGE * gm.n_edges + OBJ_BYTES_PER_TRIANGLE * mesh.n_triangles)
    achieved = comp / (ms_eval * 1e-3) / 1e9
    res = {
        "workload": f"{mesh.name}: {scene_name} CDT subdivided once, {mesh.n_vertices} vertices, "
                    f"{gm.n_edges} edges, {mesh.n_triangles} triangles; {moves} moves, seed 0",
        "eps": 1e-3 * size,
        "eval_ms": ms_eval, "edges_per_s": gm.n_edges / ms_eval * 1e3,
        "delta_ms": ms_delta, "moves_per_s": moves / ms_delta * 1e3,
        "delta_sorted_ms": ms_delta_sorted, "moves_sorted_per_s": moves / ms_delta_sorted * 1e3,
        "valid_moves": ok, "f": f, "w_contr": wc, "p_angle": pa, "p_len": pl,
        "anneal": {"classes": len(classes), "movable_vertices": n_mov,
                   "classes_host_s": t_classes, "temperature": temperature,
                   "sweep_ms": ms_sweep, "vertex_moves_per_s": n_mov / ms_sweep * 1e3,
                   "acceptance": int(accepted.item()) / (n_mov * n_sweeps), "sweeps": n_sweeps,
                   "f_before": f_before, "f_after": f_after, "proposals": proposals},
        "schedule": {"sweeps": n_sched, "ms_per_sweep": ms_sched / n_sched,
                     "temperature": [temps[0], temps[-1]], "eps": [epss[0], epss[-1]],
                     "acceptance": [int(a) / n_mov for a in acc],
                     "step_scale": [float(x) for x in lam],
                     "f_start": start[0], "w_contr_start": start[1],
                     "f_end_at_final_eps": end[0], "w_contr_end_at_final_eps": end[1],
                     "f_start_at_final_eps": start_at_end_eps[0],
                     "w_contr_start_at_final_eps": start_at_end_eps[1]},
        "roofline_eval": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                          "bytes_per_eval": comp},
    }
    gm.close()
    return res


def batch_bench(args):
    """The batch workload on its own line."""
    leg = batch_leg(args.steps, args.warmup, args.tune_cache)
    line = {
        "metric": "rays/s, 256-scene batch in one graph-replayed persistent launch (FP32+filter)",
        "value": leg["rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": leg["workload"], "items": leg["items"], "rays": leg["rays"],
                   "triangles": leg["triangles"]},
    }
    line.update({k: v for k, v in leg.items() if k not in ("workload",)})
    print(json.dumps(line), flush=True)


def batch_leg(steps, warmup, tune_cache):
    """256 scenes of uneven size and uneven ray counts traced in one persistent launch, replayed
    from a HIP graph, with launch parameters from the library's autotuner. Returns a dict."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    dev = torch.device("cuda:0")
    t0 = time.time()
    scenes, jobs = [], []
    for _, sc, r in sg.multi_workload("batch", seed=0):
        scenes.append(ccsp.Scene.from_arrays(sc))
        out = ccsp.Result(torch.empty(r.n, dtype=torch.int32, device=dev),
                          torch.empty(r.n, dtype=torch.float64, device=dev),
                          torch.empty(r.n, dtype=torch.int32, device=dev))
        jobs.append((scenes[-1], torch.from_numpy(r.o).to(dev), torch.from_numpy(r.d).to(dev),
                     torch.from_numpy(r.start).to(dev), out))
    n = sum(j[3].shape[0] for j in jobs)
    tris = sum(s.n_triangles for s in scenes)
    log(f"[bench] batch: {len(jobs)} scenes, {tris} triangles, {n} rays built in "
        f"{time.time() - t0:.1f}s")

    # reference results: one trace per item, default launch parameters
    refs = [ccsp.trace(s, o, d, st) for s, o, d, st, _ in jobs]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s, o, d, st, out in jobs:
        ccsp.trace(s, o, d, st, out=out)
    torch.cuda.synchronize()
    ms_items = (time.perf_counter() - t) * 1e3

    def timed(k, tune):
        for _ in range(2):
            ccsp.trace_batch(jobs, tune=tune, graph=True)
        torch.cuda.synchronize()
        ccsp.read_stage_times()
        t = time.perf_counter()
        for _ in range(k):
            ccsp.trace_batch(jobs, tune=tune, graph=True, timed=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return wall, ccsp.read_stage_times(k)

    wall_default, _ = timed(max(1, steps // 2), ccsp.TuneParams())
    t = time.perf_counter()
    best, tuned_ms = ccsp.autotune(jobs, "fp32", graph=True, reps=3, cache_path=tune_cache)
    tune_s = time.perf_counter() - t
    log(f"[bench] autotune: {best.as_tuple()} in {tune_s:.1f}s")
    for _ in range(warmup):
        ccsp.trace_batch(jobs, graph=True)
    wall, (bin_ms, walk_ms, fin_ms) = timed(steps, None)  # None: the tuned parameters
    torch.cuda.synchronize()
    same = all(torch.equal(j[4].hit_prim, r.hit_prim) and torch.equal(j[4].steps, r.steps)
               and torch.equal(j[4].hit_t, r.hit_t) for j, r in zip(jobs, refs))
    steps_total = int(sum(int(r.steps.sum(dtype=torch.int64).item()) for r in refs))
    ms = wall / steps * 1e3
    leg = {
        "workload": f"batch: {len(jobs)} scenes, segments log-U[100, 1e5], rays "
                    f"log-U[1024, 2^20], seed 0",
        "items": len(jobs), "rays": n, "triangles": tris,
        "rays_per_s": n * steps / wall, "ms_per_step": ms,
        "steps_per_s": steps_total * steps / wall,
        "mean_steps_per_ray": steps_total / n,
        "graph_replay_ms": float(np.mean(walk_ms)),
        "tuned": dict(zip(["wg_size", "tile_rays", "waves_per_cu", "refill_min",
                           "tiles_per_claim", "xcd_chunks", "bin"], best.as_tuple())),
        "autotune_seconds": tune_s,
        "default_params_ms_per_step": wall_default / max(1, steps // 2) * 1e3,
        "one_trace_per_item_ms": ms_items,
        "batch_equals_single_traces": same,
    }
    del refs, jobs
    for s in scenes:
        s.free()
    return leg


def serve_bench(args):
    """The serving workload on its own line."""
    leg = serve_leg(args.requests, args.slots)
    line = {
        "metric": "rays/s and p50/p99 request latency, 64 resident scenes, Poisson arrivals "
                  "(request server, FP32+filter)",
        "value": leg["capacity"]["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 0,
        "ms_per_step": leg["capacity"]["seconds"] / args.requests * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic", "config": leg["config"],
    }
    line.update({k: v for k, v in leg.items() if k != "config"})
    print(json.dumps(line), flush=True)


def serve_leg(n_requests, slots):
    """64 resident scenes; requests of log-U[256, 262144] rays, each naming a uniformly chosen
    scene, go through the library's request server (admission by device memory, coalescing across
    scenes, overlapping launch slots). Capacity: every request submitted at once. Then the same
    requests arrive as a Poisson process at 30/50/70/90% of the capacity's request rate; latency
    runs from a request's scheduled arrival to the completion the server reports."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    import scenegen as sg

    dev = torch.device("cuda:0")
    pool_rays = 262_144
    t0 = time.time()
    segs, _ = sg.multi_sizes("serve", seed=0)
    scenes, host = [], []
    for i in range(len(segs)):
        sc = sg.make_scene("serve", seed=0, n_seg=int(segs[i]), index=i)
        r = sg.sample_rays(sc, pool_rays, seed=sg.subseed(0, sg.TAG_RAYS, i + 1))
        scenes.append(ccsp.Scene.from_arrays(sc))
        host.append((torch.from_numpy(r.o).pin_memory(), torch.from_numpy(r.d).pin_memory(),
                     torch.from_numpy(r.start).pin_memory()))
    tris = sum(s.n_triangles for s in scenes)
    rng = np.random.default_rng(np.random.SeedSequence([0, 5]))
    N = n_requests
    req_scene = rng.integers(0, len(scenes), N)
    req_n = sg.log_uniform_int(rng.random(N), 256, pool_rays)
    req_off = (rng.random(N) * (pool_rays - req_n + 1)).astype(np.int64)
    gaps = rng.exponential(1.0, N)
    total_rays = int(req_n.sum())
    log(f"[bench] serve: {len(scenes)} scenes, {tris} triangles; {N} requests, {total_rays} rays; "
        f"built in {time.time() - t0:.1f}s")

    ring = 512  # pinned result buffers, reused as requests complete
    bufs = [ccsp.Result(torch.empty(pool_rays, dtype=torch.int32).pin_memory(),
                        torch.empty(pool_rays, dtype=torch.float64).pin_memory(),
                        torch.empty(pool_rays, dtype=torch.int32).pin_memory()) for _ in range(ring)]
    sample = set(range(0, N, 97))

    def run(rate):
        """rate None: all at once. Returns (latencies s, seconds, stats, stashed sample results)."""
        stash = {}
        with ccsp.Server("fp32", slots=slots, memory_bytes=2 << 30) as srv:
            start = time.monotonic() + 0.02
            arrive = np.full(N, start) if rate is None else start + np.cumsum(gaps) / rate
            free, inflight, lat = list(range(ring)), {}, np.zeros(N)
            i = done = 0
            t_end = start
            while done < N:
                now = time.monotonic()
                while i < N and arrive[i] <= now and free:
                    b, s, o, n = free.pop(), req_scene[i], req_off[i], req_n[i]
                    out = ccsp.Result(bufs[b].hit_prim[:n], bufs[b].hit_t[:n], bufs[b].steps[:n])
                    rid = srv.submit(scenes[s], host[s][0][o:o + n], host[s][1][o:o + n],
                                     host[s][2][o:o + n], out)
                    inflight[rid] = (i, b)
                    i += 1
                wait = 0.0 if (i < N and free and arrive[i] <= now) else 2e-4
                for rid, status, _, t_done in srv.poll(timeout_s=wait):
                    assert status == 0, f"request {rid} failed with {status}"
                    k, b = inflight.pop(rid)
                    lat[k] = t_done - arrive[k]
                    t_end = max(t_end, t_done)
                    if k in sample:
                        n = req_n[k]
                        stash[k] = (bufs[b].hit_prim[:n].clone(), bufs[b].hit_t[:n].clone(),
                                    bufs[b].steps[:n].clone())
                    free.append(b)
                    done += 1
            st = srv.stats()
        return lat, t_end - start, st, stash

    cap_lat, cap_s, cap_st, stash = run(None)
    cap_rays_s = total_rays / cap_s
    cap_req_s = N / cap_s
    log(f"[bench] serve capacity: {cap_rays_s / 1e9:.3f} G rays/s, {cap_req_s:.0f} requests/s")
    # the mix against the same rays traced alone (device-resident, default launch)
    same = True
    for k, (p, tt, s) in stash.items():
        sc_i, o, n = req_scene[k], req_off[k], req_n[k]
        r = ccsp.trace(scenes[sc_i], *(x[o:o + n].to(dev) for x in host[sc_i]))
        torch.cuda.synchronize()
        same &= bool(torch.equal(r.hit_prim.cpu(), p) and torch.equal(r.hit_t.cpu(), tt)
                     and torch.equal(r.steps.cpu(), s))
    levels = []
    for load in (0.3, 0.5, 0.7, 0.9):
        lat, secs, st, _ = run(load * cap_req_s)
        levels.append({"load": load, "offered_requests_per_s": load * cap_req_s,
                       "rays_per_s": total_rays / secs,
                       "p50_ms": float(np.percentile(lat, 50)) * 1e3,
                       "p99_ms": float(np.percentile(lat, 99)) * 1e3,
                       "launches": st["launches"],
                       "requests_per_launch": st["requests"] / max(1, st["launches"]),
                       "max_slots_busy": st["max_slots_busy"]})
        log(f"[bench] load {load}: p50 {levels[-1]['p50_ms']:.2f} ms, "
            f"p99 {levels[-1]['p99_ms']:.2f} ms")
    leg = {
        "config": {"workload": f"serve: {len(scenes)} resident scenes, segments log-U[1e3, 5e5]; "
                               f"{N} requests of log-U[256, 262144] rays, uniform scene, seed 0",
                   "triangles": tris, "rays": total_rays, "slots": slots,
                   "pool_bytes": 2 << 30, "host_buffers": "pinned"},
        "capacity": {"rays_per_s": cap_rays_s, "requests_per_s": cap_req_s, "seconds": cap_s,
                     "p50_ms": float(np.percentile(cap_lat, 50)) * 1e3,
                     "p99_ms": float(np.percentile(cap_lat, 99)) * 1e3,
                     "launches": cap_st["launches"],
                     "requests_per_launch": cap_st["requests"] / max(1, cap_st["launches"])},
        "levels": levels,
        "mix_equals_alone_sampled": same, "sampled_requests": len(stash),
    }
    for s in scenes:
        s.free()
    return leg


def copy_calibration(mib):
    """A plain copy of known size: the profiler's FETCH_SIZE / WRITE_SIZE for it give the
    counters' scale (bytes counted per byte moved)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def gather_sweep():
    """Sustained 16-byte dependent loads per second of persistent pointer-chasing waves, by buffer
    size (the memory pattern of one walk step) and resident waves per compute unit."""
    import torch  # noqa: F401  (binds the HIP runtime first)
    from paper_2112_05570_amd import binding as B
    for ws in (1 << 21, 1 << 22, 1 << 23, 1 << 25, 1 << 27, 1 << 30, 1 << 32):
        for wpc in (8, 16, 24, 32):
            r = B.gather_roofline(ws, wpc, 2048)
            print(json.dumps({"buffer_bytes": ws, "waves_per_cu": wpc, "loads_per_s": r}), flush=True)


def pure_binary32_t_error(sc, o, d, res, torch, sample=1 << 20):
    """Diagnostic only: relative error of the hit distance evaluated entirely in binary32 (ray and
    primitive segment rounded to binary32, the same formula) against the binary64 t the walk
    returns, on the first `sample` hits. The walk itself always finishes t in binary64."""
    import numpy as np
    prims = torch.from_numpy(sc.prims).to(o.device)
    p = res.hit_prim[:sample].long()
    hit = p >= 0
    seg = prims[p[hit]].float()
    oo, dd, t64 = o[:sample][hit].float(), d[:sample][hit].float(), res.hit_t[:sample][hit]
    ax, ay, bx, by = seg[:, 0], seg[:, 1], seg[:, 2], seg[:, 3]
    ex, ey = bx - ax, by - ay
    t32 = ((ax - oo[:, 0]) * ey - (ay - oo[:, 1]) * ex) / (dd[:, 0] * ey - dd[:, 1] * ex)
    rel = ((t32.double() - t64).abs() / t64.abs()).cpu().numpy()
    return {"p50": float(np.percentile(rel, 50)), "p99": float(np.percentile(rel, 99)),
            "max": float(rel.max()), "sample": int(rel.size)}


TET3D_POINTS, TET3D_FRAC, TET3D_RAYS = 200_000, 0.05, 1 << 22
GROUP_CENTRES = 1 << 13  # centres of the objective leg's group sweep


def tet3d_leg(steps, warmup, cpu_seconds):
    """The 3D walk (include/ccsp_tet.h): a Delaunay tetrahedralisation of 200,000 seeded grid
    points with every hull face and 5% of the interior faces as primitives, 4M rays with a start
    tetrahedron drawn by volume, an origin uniform in it and an isotropic direction. Whole traces
    (binning and start records, then the walk) timed with events on the stream; stage times from
    the library's own events; the walk's gather rate against the dependent-gather chase on a
    buffer the size of the face slots."""
    import numpy as np
    import torch

    import paper_2112_05570_amd as ccsp
    from paper_2112_05570_amd import binding as B
    import scenegen as sg

    t0 = time.perf_counter()
    sc = sg.make_tet_scene(TET3D_POINTS, seed=0, frac_prims=TET3D_FRAC)
    r = sg.sample_rays3(sc, TET3D_RAYS, seed=1)
    log(f"[bench] tet3d: {sc.n_tets} tetrahedra, {sc.n_prims} primitives, {r.n} rays "
        f"(built in {time.perf_counter() - t0:.1f}s)")
    dev = [torch.from_numpy(a).to("cuda:0") for a in (r.o, r.d, r.start)]
    stream = torch.cuda.current_stream()
    n = r.n
    with ccsp.TetMesh.from_arrays(sc) as mesh:
        res = ccsp.trace3d(mesh, *dev)

        def timed(k, **kw):
            for _ in range(warmup):
                ccsp.trace3d(mesh, *dev, out=res, **kw)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(k):
                ccsp.trace3d(mesh, *dev, out=res, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / k

        ms = timed(steps)
        ms_io = timed(max(1, steps // 2), input_order=True)
        stages = []
        for _ in range(max(3, steps // 2)):
            ccsp.trace3d(mesh, *dev, out=res, timed=True)
            stages.append(ccsp.trace3d_stage_times())
        bin_ms, walk_ms = (float(np.mean([x[i] for x in stages])) for i in range(2))
        steps_np = res.steps.cpu().numpy()
        prim_np = res.hit_prim.cpu().numpy()
        slot_bytes = 64 * sc.n_tets
        chase = B.gather_roofline(slot_bytes, 16, 2048, stream.cuda_stream)
    steps_total = int(steps_np.sum(dtype=np.int64))
    # the walk's algorithmic bytes: the 64-byte start record, one 16-byte face slot per visited
    # tetrahedron (its exit face), the 16 bytes of results
    walk_bytes = 64 * n + 16 * steps_total + 16 * n
    walk_gbs = walk_bytes / (walk_ms / 1e3) / 1e9
    loads_s = steps_total / (walk_ms / 1e3)
    out = {
        "workload": f"tets: {TET3D_POINTS} seeded grid points (Delaunay), {sc.n_tets} tetrahedra, "
                    f"hull + {int(TET3D_FRAC * 100)}% of interior faces as {sc.n_prims} primitives, "
                    f"{n} rays (origin uniform in a volume-drawn start, isotropic direction), seed 0",
        "rays": n, "tetrahedra": sc.n_tets, "primitives": sc.n_prims,
        "value": n / ms * 1e3, "unit": "rays/s", "ms_per_trace": ms,
        "ms_per_trace_input_order": ms_io,
        "stages_ms": {"binning_and_start": bin_ms, "walk": walk_ms},
        "mean_steps_per_ray": steps_total / n,
        "p99_steps_per_ray": float(np.percentile(steps_np, 99)),
        "steps_per_s": steps_total / ms * 1e3,
        "rays_not_hit": int((prim_np < 0).sum()),
        "dtype": "int32 coordinates, f64 filter + exact int64",
        "roofline": {"bound": "hbm", "kernel": "walk3d", "kernel_ms": walk_ms,
                     "achieved": walk_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": walk_gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": walk_bytes,
                     "bytes_model": "64 B/ray start record + 16 B per visited tetrahedron (its "
                                    "exit slot) + 16 B/ray results (algorithmic)"},
        "gather": {"slot_loads_per_s": loads_s, "chase_loads_per_s_slot_sized": chase,
                   "slot_bytes": slot_bytes, "frac_of_chase": loads_s / chase},
    }
    if cpu_seconds:
        out["cpu_baseline"] = tet3d_cpu_leg(sc, r, cpu_seconds)
    return out


def tet3d_cpu_leg(sc, r, budget_s):
    """The 3D checker's walk, as it stands, on the host cores: a bounded prefix of the same rays."""
    import numpy as np

    import oracle

    m3 = oracle.TetMesh.of(sc)
    threads = oracle.num_threads()
    m = 1 << 14
    while True:
        t = time.perf_counter()
        oracle.walk3(m3, r.o[:m], r.d[:m], r.start[:m], threads)
        dt = time.perf_counter() - t
        if dt >= 1.0 or m >= r.n:
            break
        m = min(r.n, m * 4)
    m = int(min(r.n, max(m, m * budget_s / dt)))
    t = time.perf_counter()
    _, _, s, _ = oracle.walk3(m3, r.o[:m], r.d[:m], r.start[:m], threads)
    dt = time.perf_counter() - t
    log(f"[bench] 3D checker walk: {m} rays on {threads} threads in {dt:.1f}s")
    return {"value": m / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} of the same rays (exact int64 checker walk, OpenMP over rays)",
            "steps_per_s": float(np.sum(s, dtype=np.int64)) / dt, "cpu": cpu_model()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(sc, rays, budget_s):
    """The checker's walk, as it stands, on the host cores: a bounded prefix of the same rays."""
    import numpy as np

    import oracle

    tri = oracle.Triangulation.of(sc)
    threads = oracle.num_threads()
    m = 1 << 14
    while True:  # calibrate on growing prefixes until a run takes at least a second
        t = time.perf_counter()
        oracle.walk(tri, rays.o[:m], rays.d[:m], rays.start[:m], threads)
        dt = time.perf_counter() - t
        if dt >= 1.0 or m >= rays.n:
            break
        m = min(rays.n, m * 4)
    m = int(min(rays.n, max(m, m * budget_s / dt)))
    t = time.perf_counter()
    _, _, s = oracle.walk(tri, rays.o[:m], rays.d[:m], rays.start[:m], threads)
    dt = time.perf_counter() - t
    log(f"[bench] checker walk: {m} rays on {threads} threads in {dt:.1f}s")
    return {"value": m / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} of the same rays (exact integer-arithmetic checker walk, "
                      f"OpenMP over rays)",
            "steps_per_s": float(np.sum(s, dtype=np.int64)) / dt,
            "rays_per_s_per_core": m / dt / threads, "cpu": cpu_model()}


if __name__ == "__main__":
    main()
