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




def rules_mesh(seed):
    """A movable mesh on which the conditioning and flat-triangle restrictions of Sec. 2.2.2 are
    at work: inside an ORIGINAL square frame, six original edges each carrying three CONSTRAINED
    vertices with a FREE vertex just above its middle (fanned over the edge, the flat-triangle
    setting), and pairs of collinear original edges with a FREE vertex over their gap (snapping
    it onto one end makes three ORIGINAL vertices collinear), plus scattered FREE vertices. The
    Delaunay triangulation of the points (scipy) is kept only if it contains every piece of every
    original edge. Returns (tri_v, kind, line, prim_v, xy)."""
    from scipy.spatial import Delaunay
    ORIG, CONS, FREE = 0, 1, 2
    rng = np.random.default_rng(seed)
    while True:
        pts, kind, line, prims = [], [], [], []

        def add(p, k, ln=0):
            pts.append(p)
            kind.append(k)
            line.append(ln)
            return len(pts) - 1
        corners = [add((0.0, 0.0), ORIG), add((20.0, 0.0), ORIG), add((20.0, 20.0), ORIG),
                   add((0.0, 20.0), ORIG)]
        for i in range(4):
            prims.append((corners[i], corners[(i + 1) % 4]))
        for i in range(6):
            y = 2.0 + 3.0 * i + rng.uniform(-0.3, 0.3)
            a, b = add((2.0, y), ORIG), add((8.0, y), ORIG)
            prims.append((a, b))
            for x in (3.5, 5.0, 6.5):
                add((x + rng.uniform(-0.2, 0.2), y), CONS, len(prims) - 1)
            add((5.0 + rng.uniform(-0.3, 0.3), y + rng.uniform(0.3, 0.5)), FREE)
        for i in range(3):
            y = 3.5 + 5.0 * i + rng.uniform(-0.3, 0.3)
            p = [add((x, y), ORIG) for x in (11.0, 14.0, 15.0, 18.0)]
            prims += [(p[0], p[1]), (p[2], p[3])]
            add((14.5 + rng.uniform(-0.1, 0.1), y + rng.uniform(0.4, 0.6)), FREE)
        for _ in range(40):
            q = rng.uniform(0.5, 19.5, 2)
            if min(abs(q[1] - np.array(pts)[:, 1]).min(), 10) > 0.8:
                add(tuple(q), FREE)
        xy = np.array(pts)
        tri = Delaunay(xy).simplices.astype(np.int64)
        a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
        cw = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
        tri[cw] = tri[cw][:, [0, 2, 1]]
        edges = {tuple(sorted((int(t[i]), int(t[(i + 1) % 3])))) for t in tri for i in range(3)}
        kind_a, line_a = np.array(kind), np.array(line)
        ok = True
        for k, (a0, b0) in enumerate(prims):
            on = [a0, b0] + [v for v in range(len(pts)) if kind_a[v] == CONS and line_a[v] == k]
            on.sort(key=lambda v: (xy[v, 0], xy[v, 1]))
            ok = ok and all(tuple(sorted((on[j], on[j + 1]))) in edges for j in range(len(on) - 1))
        if ok:
            return (tri.astype(np.int32), kind_a.astype(np.int32), line_a.astype(np.int32),
                    np.array(prims, dtype=np.int32), xy)


def subdivided(sc):
    """The scene's CDT subdivided once (Sec. 3.5.2) by the checker's subdivision: the input of
    the objective's tests on both sides."""
    from oracle.subdivide import subdivide
    return subdivide(*sg.movable_input(sc), name=sc.name + "/4")
