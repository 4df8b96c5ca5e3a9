"""Larger pins of the checker (marked slow; still CPU-only and run by default).

* the side predicate against exact rationals (``fractions.Fraction``) on 10^6 adversarial cases;
* the walk against brute force (every edge, every primitive) on random rays of the grid scene and
  of the 10^6-segment scene, i.e. at the bench's scale of scene.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from test_oracle_predicates import _side_cases, side_exact

pytestmark = pytest.mark.slow


def test_side_sign_many_cases():
    rng = np.random.default_rng(11)
    cases = _side_cases(rng, 300_000)
    signs = {-1: 0, 0: 0, 1: 0}
    for o, d, v in cases:
        e = side_exact(o, d, v)
        signs[e] += 1
        assert oracle.side_sign(o, d, v) == e, (o, d, v)
    assert min(signs.values()) > 3_000


@pytest.mark.parametrize("name, n_edges_rays, n_prims_rays", [("grid", 24, 120), ("large", 3, 12)])
def test_walk_equals_brute_force_at_scale(name, n_edges_rays, n_prims_rays):
    sc = sg.make_scene(name, seed=0)
    tri = oracle.Triangulation.of(sc)
    r = sg.sample_rays(sc, n_prims_rays, seed=17)
    p, t, s = oracle.walk(tri, r.o, r.d, r.start)
    pp, tp, status = oracle.brute_prims(sc.prims, r.o, r.d)
    assert status == 0 and np.array_equal(pp, p) and np.array_equal(tp, t)
    k = n_edges_rays
    pb, tb, sb, status = oracle.brute_edges(tri, r.o[:k], r.d[:k])
    assert status == 0
    assert np.array_equal(pb, p[:k]) and np.array_equal(sb, s[:k]) and np.array_equal(tb, t[:k])
