"""Pins for the checker's walk (paper Sec. 5.1) against things other than itself.

* a hand-derived closed-form fixture (unit square split by its diagonal);
* the textbook distance to a square and the diagonal test on random rays;
* brute force over every edge and over every primitive (the definition of the result), on the
  whole tiny workload and on scenes built to hit every degenerate case exactly: rays through
  vertices, along edges and through box corners;
* Cauchy-Crofton: the mean number of interior edges crossed by isotropic lines equals
  2 * (interior edge length) / (box perimeter) (the weight/cost relation of Sec. 1.4);
* invariance of hit and distance across two triangulations of one scene;
* the miss outcome (a hull edge that is not scene geometry): a hand-derived fixture, and brute
  force on scenes whose box sides are opened, degenerate rays included;
* the step guard against the unlimited walk: rays that need more triangles than the limit stop
  there, every other ray is unchanged.
"""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import scenegen as sg
from helpers import degenerate_rays as _degenerate_rays, integer_scene as _integer_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tri(sc):
    return oracle.Triangulation.of(sc)


def test_golden_unit_square():
    g = json.load(open(os.path.join(GOLDEN, "unit_square_diagonal.json")))
    tri = oracle.Triangulation(g["xy"], g["tri_v"], g["tri_nbr"], g["tri_prim"], g["prims"])
    assert oracle.validate(tri, delaunay=True) == ""
    o = np.array([r["o"] for r in g["rays"]], float)
    d = np.array([r["d"] for r in g["rays"]], float)
    s = np.array([r["start"] for r in g["rays"]], np.int32)
    prim, t, steps = oracle.walk(tri, o, d, s)
    assert prim.tolist() == [r["prim"] for r in g["rays"]]
    assert t.tolist() == [r["t"] for r in g["rays"]]
    assert steps.tolist() == [r["steps"] for r in g["rays"]]


def _square():
    g = json.load(open(os.path.join(GOLDEN, "unit_square_diagonal.json")))
    return g, oracle.Triangulation(g["xy"], g["tri_v"], g["tri_nbr"], g["tri_prim"], g["prims"])


def test_square_closed_form_random_rays():
    g, tri = _square()
    rng = np.random.default_rng(5)
    n = 20000
    o = rng.uniform(0, 1, (n, 2))
    o = o[o[:, 0] != o[:, 1]]
    th = rng.uniform(0, 2 * np.pi, o.shape[0])
    d = np.stack([np.cos(th), np.sin(th)], 1)
    start = (o[:, 1] > o[:, 0]).astype(np.int32)  # above the diagonal: triangle 1
    prim, t, steps = oracle.walk(tri, o, d, start)
    # textbook: distance to each side along d, the smallest positive one wins
    with np.errstate(divide="ignore"):
        tx = np.where(d[:, 0] > 0, (1 - o[:, 0]) / d[:, 0], -o[:, 0] / d[:, 0])
        ty = np.where(d[:, 1] > 0, (1 - o[:, 1]) / d[:, 1], -o[:, 1] / d[:, 1])
    side = np.where(tx < ty, np.where(d[:, 0] > 0, 1, 3), np.where(d[:, 1] > 0, 2, 0))
    tt = np.minimum(tx, ty)
    assert (prim == side).all()
    np.testing.assert_allclose(t, tt, rtol=1e-13)
    # the exit point lies on the other triangle's sides iff the diagonal was crossed
    x = o + tt[:, None] * d
    other = np.where(start == 0, x[:, 1] > x[:, 0], x[:, 1] < x[:, 0])
    assert (steps == 1 + other).all()


def test_tiny_walk_equals_brute_force(tiny_scene, tiny_rays):
    tri = _tri(tiny_scene)
    r = tiny_rays
    p, t, s = oracle.walk(tri, r.o, r.d, r.start)
    assert (p >= 0).all() and (s >= 1).all()
    pb, tb, sb, status = oracle.brute_edges(tri, r.o, r.d)
    assert status == 0
    assert (p == pb).all() and (s == sb).all()
    assert np.array_equal(t, tb)
    pp, tp, status = oracle.brute_prims(tiny_scene.prims, r.o, r.d)
    assert status == 0 and (pp == p).all() and np.array_equal(tp, t)


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_degenerate_rays_walk_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    sc = _integer_scene(rng, int(rng.integers(3, 14)))
    tri = _tri(sc)
    assert oracle.validate(tri, delaunay=True) == ""
    o, d, start = _degenerate_rays(sc, rng, 200)
    assert o.shape[0] > 20
    # the cases are really degenerate: some vertex lies exactly on many rays
    zero = sum(oracle.side_sign(o[k], d[k], v) == 0 for k in range(10) for v in sc.xy)
    assert zero >= 10
    p, t, s = oracle.walk(tri, o, d, start)
    assert (p >= 0).all()
    pb, tb, sb, status = oracle.brute_edges(tri, o, d)
    assert status == 0
    assert (p == pb).all() and (s == sb).all() and np.array_equal(t, tb)
    pp, tp, status = oracle.brute_prims(sc.prims, o, d)
    assert (pp == p).all() and np.array_equal(tp, t)


def _crofton_lines(lo, hi, n, rng):
    """Lines from the motion-invariant measure that hit the box, and a point uniform on each
    chord. Returns (origin, direction, chord length)."""
    c = 0.5 * (lo + hi)
    R = (hi - lo) * math.sqrt(0.5)
    o_all, d_all, L_all = [], [], []
    while sum(x.shape[0] for x in o_all) < n:
        m = 2 * n
        th = rng.uniform(0, np.pi, m)
        p = rng.uniform(-R, R, m)
        d = np.stack([np.cos(th), np.sin(th)], 1)
        nrm = np.stack([-np.sin(th), np.cos(th)], 1)
        foot = c + p[:, None] * nrm
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (lo - foot) / d
            t2 = (hi - foot) / d
        tmin = np.nanmax(np.minimum(t1, t2), axis=1)
        tmax = np.nanmin(np.maximum(t1, t2), axis=1)
        ok = tmax > tmin
        u = rng.uniform(0, 1, m)
        s = tmin + u * (tmax - tmin)
        o = foot + s[:, None] * d
        o_all.append(o[ok])
        d_all.append(d[ok])
        L_all.append((tmax - tmin)[ok])
    return (np.concatenate(o_all)[:n], np.concatenate(d_all)[:n], np.concatenate(L_all)[:n])


def _crofton_check(sc, n_lines, seed):
    rng = np.random.default_rng(seed)
    lo, hi = sc.box
    # interior constraints removed: a ray then crosses the whole chord; box sides stay primitives
    hull = sc.tri_nbr < 0
    prim = np.where(hull, sc.tri_prim, -1).astype(np.int32)
    tri = oracle.Triangulation(sc.xy, sc.tri_v, sc.tri_nbr, prim, sc.prims)
    o, d, chord = _crofton_lines(lo, hi, n_lines, rng)
    start = sg.locate(sc, o)
    keep = start >= 0
    o, d, chord, start = o[keep], d[keep], chord[keep], start[keep]
    pf, tf, sf = oracle.walk(tri, o, d, start)
    pbk, tbk, sbk = oracle.walk(tri, o, -d, start)
    assert (pf >= 0).all() and (pbk >= 0).all()
    ncross = (sf + sbk - 2).astype(np.float64)
    # interior edge length
    e = []
    for i in range(3):
        a = sc.xy[sc.tri_v[:, (i + 1) % 3]]
        b = sc.xy[sc.tri_v[:, (i + 2) % 3]]
        inner = (sc.tri_nbr[:, i] >= 0) & (sc.tri_nbr[:, i] > np.arange(sc.n_triangles))
        e.append(np.hypot(*(b - a).T)[inner])
    L_int = float(np.concatenate(e).sum())
    expect = 2.0 * L_int / (4.0 * (hi - lo))
    mean = ncross.mean()
    se = ncross.std(ddof=1) / math.sqrt(ncross.size)
    np.testing.assert_allclose(tf + tbk, chord, rtol=1e-12, atol=1e-13 * (hi - lo))
    return mean, se, expect


def test_crofton_unit_square():
    g, _ = _square()
    sc = sg.Scene(np.array(g["xy"], float), np.array(g["prims"], float), np.zeros((0, 2), np.int32),
                  (0.0, 1.0), np.array(g["tri_v"], np.int32), np.array(g["tri_nbr"], np.int32),
                  np.array(g["tri_prim"], np.int32))
    mean, se, expect = _crofton_check(sc, 1 << 18, 11)
    assert abs(expect - g["crofton_mean_interior_crossings"]) < 1e-15
    assert abs(mean - expect) < 5 * se, (mean, se, expect)


def test_crofton_tiny(tiny_scene):
    mean, se, expect = _crofton_check(tiny_scene, 1 << 20, 12)
    assert abs(mean - expect) < 5 * se, (mean, se, expect)
    assert se < 0.01 * expect  # the statistic is sharp enough to catch a dropped edge class


def test_invariance_cdt_vs_annealed(tiny_scene, tiny_rays):
    an, stats = sg.anneal_flips(tiny_scene, seed=0)
    assert stats["w_end"] <= stats["w_start"]
    tri_a = _tri(an)
    assert oracle.validate(tri_a) == ""
    r = tiny_rays
    start = sg.locate(an, r.o)
    keep = start >= 0
    p1, t1, s1 = oracle.walk(_tri(tiny_scene), r.o[keep], r.d[keep], r.start[keep])
    p2, t2, s2 = oracle.walk(tri_a, r.o[keep], r.d[keep], start[keep])
    assert (p1 == p2).all() and np.array_equal(t1, t2)
    assert (s1 != s2).any()


def _golden(name):
    g = json.load(open(os.path.join(GOLDEN, name)))
    tri = oracle.Triangulation(g["xy"], g["tri_v"], g["tri_nbr"], g["tri_prim"], g["prims"])
    o = np.array([r["o"] for r in g["rays"]], float)
    d = np.array([r["d"] for r in g["rays"]], float)
    s = np.array([r["start"] for r in g["rays"]], np.int32)
    return g, tri, o, d, s


def _tval(x):
    return math.inf if x == "inf" else float(x)


def test_golden_open_sides_miss_and_guard():
    g, tri, o, d, s = _golden("unit_square_open_sides.json")
    assert oracle.validate(tri, delaunay=True) == ""
    prim, t, steps = oracle.walk(tri, o, d, s)
    assert prim.tolist() == [r["prim"] for r in g["rays"]]
    assert t.tolist() == [_tval(r["t"]) for r in g["rays"]]
    assert steps.tolist() == [r["steps"] for r in g["rays"]]
    assert (prim == -1).sum() == 5
    pb, tb, sb, status = oracle.brute_edges(tri, o, d)
    assert status == 0
    assert np.array_equal(pb, prim) and np.array_equal(tb, t) and np.array_equal(sb, steps)
    # the guard: a limit of one triangle
    prim, t, steps = oracle.walk(tri, o, d, s, max_steps=g["guard_max_steps"])
    assert prim.tolist() == [r["prim"] for r in g["guard"]]
    assert t.tolist() == [_tval(r["t"]) for r in g["guard"]]
    assert steps.tolist() == [r["steps"] for r in g["guard"]]
    # zero bounces is the walk; a reflection off the bottom side then leaves through the top
    pr, tr, sr, hits, face = oracle.bounce(tri, o, d, s, 0)
    p0, t0, s0 = oracle.walk(tri, o, d, s)
    assert np.array_equal(pr, p0) and np.array_equal(tr, t0) and np.array_equal(sr, s0)
    pr, tr, sr, hits, face = oracle.bounce(tri, o[3:4], d[3:4], s[3:4], 2)
    # o = (0.75, 0.25) straight down: hits the bottom at (0.75, 0) in triangle 0, reflects
    # straight up, crosses the diagonal at (0.75, 0.75) and leaves through the open top side
    assert pr.tolist() == [-1] and hits.tolist() == [1] and sr.tolist() == [3] and face.tolist() == [-1]
    assert math.isinf(tr[0])


@pytest.mark.parametrize("sides", [(0, 1, 2, 3), (1, 2), (3,)])
def test_open_hull_walk_equals_brute_force(tiny_scene, tiny_rays, sides):
    sc = sg.open_hull(tiny_scene, sides)
    tri = _tri(sc)
    assert oracle.validate(tri, delaunay=True) == ""
    r = tiny_rays.slice(0, 8192)
    p, t, s = oracle.walk(tri, r.o, r.d, r.start)
    miss = p == -1
    assert miss.sum() > 100 and (p >= -1).all()
    assert np.isinf(t[miss]).all() and np.isfinite(t[~miss]).all()
    pb, tb, sb, status = oracle.brute_edges(tri, r.o, r.d)
    assert status == 0
    assert np.array_equal(p, pb) and np.array_equal(s, sb) and np.array_equal(t, tb)
    # brute force over the remaining primitives alone: -1 exactly when no primitive is ahead
    pp, tp, status = oracle.brute_prims(sc.prims, r.o, r.d)
    assert status == 0 and np.array_equal(pp, p) and np.array_equal(tp, t)
    # hits on primitives that stayed scene geometry are unchanged by opening the others
    p0, t0, s0 = oracle.walk(_tri(tiny_scene), r.o, r.d, r.start)
    S = tiny_scene.n_prims - 4
    seg_hit = p0 < S
    assert np.array_equal(p[seg_hit], p0[seg_hit]) and np.array_equal(t[seg_hit], t0[seg_hit])
    assert np.array_equal(s[seg_hit], s0[seg_hit])


@settings(max_examples=25, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_open_hull_degenerate_rays(seed):
    rng = np.random.default_rng(seed)
    sc = sg.open_hull(_integer_scene(rng, int(rng.integers(3, 14))),
                      tuple(k for k in range(4) if rng.random() < 0.6) or (0,))
    tri = _tri(sc)
    o, d, start = _degenerate_rays(sc, rng, 200)
    p, t, s = oracle.walk(tri, o, d, start)
    pb, tb, sb, status = oracle.brute_edges(tri, o, d)
    assert status == 0
    assert np.array_equal(p, pb) and np.array_equal(s, sb) and np.array_equal(t, tb)


@pytest.mark.parametrize("limit", [1, 2, 5, 17])
def test_guard_against_unlimited_walk(tiny_scene, tiny_rays, limit):
    tri = _tri(sg.open_hull(tiny_scene, (1, 2)))
    r = tiny_rays.slice(0, 8192)
    p, t, s = oracle.walk(tri, r.o, r.d, r.start)
    pg, tg, sg_ = oracle.walk(tri, r.o, r.d, r.start, max_steps=limit)
    long = s > limit
    assert long.any() and (~long).any()
    assert np.array_equal(pg[~long], p[~long]) and np.array_equal(tg[~long], t[~long])
    assert np.array_equal(sg_[~long], s[~long])
    assert (pg[long] == -2).all() and (sg_[long] == limit).all() and np.isinf(tg[long]).all()
    # a limit at or above the triangle count changes nothing
    pn, tn, sn = oracle.walk(tri, r.o, r.d, r.start, max_steps=tri.tri_v.shape[0])
    assert np.array_equal(pn, p) and np.array_equal(tn, t) and np.array_equal(sn, s)
