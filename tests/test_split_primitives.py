"""Primitives covered by several constrained edges (a segment split at an interior vertex): the
hit is the primitive, t comes from the primitive's own segment (so it does not depend on the
split), and the steps count the extra triangles. Checker pins on CPU."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from helpers import degenerate_rays, integer_scene


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_split_scene_walk_equals_brute_force_and_unsplit(seed):
    rng = np.random.default_rng(seed)
    whole = integer_scene(rng, int(rng.integers(4, 12)))
    split = sg.triangulate(sg.split_segments(whole))
    # two constrained edges per segment primitive, each seen from both of its triangles
    S = whole.prims.shape[0] - 4
    assert (np.bincount(split.tri_prim[split.tri_prim >= 0])[:S] == 4).all()
    tw, ts = oracle.Triangulation.of(whole), oracle.Triangulation.of(split)
    assert oracle.validate(ts) == ""
    o, d, start_w = degenerate_rays(whole, rng, 400)
    start_s = sg.locate(split, o)
    keep = start_s >= 0
    o, d, start_w, start_s = o[keep], d[keep], start_w[keep], start_s[keep]
    pw, tw_, sw = oracle.walk(tw, o, d, start_w)
    ps, ts_, ss = oracle.walk(ts, o, d, start_s)
    assert np.array_equal(pw, ps) and np.array_equal(tw_, ts_)
    pb, tb, sb, status = oracle.brute_edges(ts, o, d)
    assert status == 0 and np.array_equal(ps, pb) and np.array_equal(ss, sb) and np.array_equal(ts_, tb)
    assert (ss != sw).any()  # the split vertices add triangles along some rays
