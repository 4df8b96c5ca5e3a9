"""Shared test inputs: small integer scenes and rays built to hit degenerate cases exactly."""
import numpy as np

import scenegen as sg


def integer_scene(rng, n_seg, size=16):
    segs = []
    while len(segs) < n_seg:
        a = rng.integers(1, size, 2)
        b = a + rng.integers(-3, 4, 2)
        if (b <= 0).any() or (b >= size).any() or (a == b).all():
            continue
        s = np.concatenate([a, b]).astype(float)
        if all(not _touch(s, q) for q in segs):
            segs.append(s)
    return sg.triangulate(sg.scene_from_segments(np.array(segs), 0.0, float(size)))


def _touch(s, q):
    # integer data: exact signs in binary64
    def o(a, b, c):
        return np.sign((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
    A, B, C, D = s[:2], s[2:], q[:2], q[2:]
    o1, o2, o3, o4 = o(A, B, C), o(A, B, D), o(C, D, A), o(C, D, B)
    if o1 * o2 > 0 or o3 * o4 > 0:
        return False
    if o1 == 0 and o2 == 0:
        k = 0 if abs(B[0] - A[0]) >= abs(B[1] - A[1]) else 1
        return not (max(A[k], B[k]) < min(C[k], D[k]) or max(C[k], D[k]) < min(A[k], B[k]))
    return True


def degenerate_rays(sc, rng, n):
    """Dyadic origins strictly inside a triangle, aimed exactly at vertices, along edge lines
    and at the box corners."""
    V = sc.xy
    o_list, d_list = [], []
    T = sc.n_triangles
    while len(o_list) < n:
        kind = rng.integers(0, 3)
        if kind == 2:  # along the line of an edge, from outside the edge
            t = rng.integers(0, T)
            i = rng.integers(0, 3)
            p, q = V[sc.tri_v[t, (i + 1) % 3]], V[sc.tri_v[t, (i + 2) % 3]]
            lam = rng.choice([-0.5, -0.25, 1.25, 1.5, 2.0])
            o = p + lam * (q - p)
            d = (q - p) * rng.choice([-1.0, 1.0])
        else:
            o = rng.integers(0, 64, 2) / 4.0 + 0.125
            tgt = V[rng.integers(0, 4)] if kind == 1 else V[rng.integers(0, V.shape[0])]
            d = tgt - o
        if (d == 0).all():
            continue
        o_list.append(o)
        d_list.append(d)
    o = np.array(o_list)
    d = np.array(d_list)
    start = sg.locate(sc, o)
    keep = start >= 0
    return o[keep], d[keep], start[keep]


