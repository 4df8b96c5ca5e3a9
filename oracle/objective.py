"""Objective with fuzzy contraction and its change under vertex moves: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU leg may import this module. The
GPU library never does and shares no code with it.

What is computed (paper Sec. 2.2):
- the contractible weight w_contr = sum over edges of w_eps(e) * |e| (Sec. 2.2.1), where
  w_eps(e) = x * M(x) with x the product of c_eps over the other edges of the one or two
  triangles holding e, c_eps(e) = 1/2 + min(1, |e|/eps)/2 for a contractible edge and 1 otherwise,
  and M the correction for multiply merged edges (0 below 1/4, 4x - 1 up to 1/2, then 1);
- which edges are contractible (Sec. 2.2.2): the restrictions from the original geometry (vertex
  kinds) and the 1-hop topology rule;
- the angle penalty (Sec. 2.2.3): over the three corners of every triangle, the ramp
  max(0, -1 + delta - cos)/delta on the cosine between the corner's two edges (in polishing, the
  ramp max(0, cos - (1 - delta))/delta on sharp corners instead, and every edge weight 1);
- the length penalty (Sec. 2.2.3): over edges, max(0, eps0 - |e|)/eps0;
- f = w_contr + mu_angle * P_angle + mu_len * P_len (Sec. 2.2.4);
- for a proposed single-vertex move (Sec. 3.2.1, 3.2.2), its validity (the triangulation keeps
  every triangle strictly counter-clockwise, decided exactly) and
  delta_f = f(moved) - f(current), summed term by term over every term of f;
- the proposals of Secs. 3.2.4-3.2.6 for one vertex at a time: a position uniform by area over
  its triangles (resampling), a position near one of its neighbours for a vertex on an edge
  shorter than a drawn length (swapping a contracted edge), and a resampling kept only when it
  changes whether the vertex is contracted (contracting to a neighbour).

Every value is binary64, evaluated in the operation order written below with no fused operations
(numpy does not fuse), so that each term is a fixed function of the coordinates.

Readings of points the paper leaves open:
- Edge weight: the equation of Sec. 2.2.1 writes M(x), but the worked example of its figure (a
  merged pair weighs 1/2, an edge with two contracted neighbours weighs 0) and the remark that an
  identity M would already handle isolated contractions fix w_eps = x * M(x).
- 1-hop rule: a nontrivial common neighbour H of the edge's endpoints is harmless when its
  distance to one of the edge's opposite vertices is strictly below eps (the figure's
  ||V3 H|| < eps).
- Restrictions from the original geometry (Sec. 2.2.2): an edge is incontractible when both ends
  are original vertices; when one end is original and the other constrained to an original edge
  that does not end at it; or when both are constrained to different original edges.
- Conditioning and flat-triangle restrictions (Sec. 2.2.2): see conditioning_ok and flat_ok.
  Near-collinearity compares a triangle's area with the square of equal perimeter against
  COLLINEAR = 0.01 (the paper gives no value). Trapped vertices count as already contracted when
  a path of edges shorter than eps along their original edge, through the free vertex's fan,
  reaches the vertex contracted to or an original end of that edge.
- A corner with a zero-length edge contributes no angle penalty (its cosine is undefined; the
  length penalty covers it).
- Edges are numbered by (lower vertex id, higher vertex id); the product x runs over the
  neighbouring edges of the edge's triangles in increasing triangle id, each triangle's two edges
  in its local order after the edge itself, multiplied left to right.
"""
from __future__ import annotations

import math

import numpy as np

from . import orient

ORIGINAL, CONSTRAINED, FREE = 0, 1, 2


class Params:
    """eps: contraction length; delta: angle-cosine threshold; eps0: minimum edge length;
    mu_angle, mu_len: penalty weights; polish: fixed topology (no fuzzy contraction)."""

    def __init__(self, eps, delta=None, eps0=1e-10, mu_angle=1.0, mu_len=10.0, polish=False):
        self.eps = float(eps)
        self.delta = float(np.cos(np.radians(179.0)) + 1.0) if delta is None else float(delta)
        self.eps0 = float(eps0)
        self.mu_angle = float(mu_angle)
        self.mu_len = float(mu_len)
        self.polish = bool(polish)


class Mesh:
    """A triangulation with movable vertices. kind[v] is ORIGINAL, CONSTRAINED (on original edge
    line[v], an index into prim_v) or FREE; prim_v[k] are the two original vertices ending
    original edge k. Triangles are counter-clockwise."""

    def __init__(self, tri_v, kind, line, prim_v):
        self.tri_v = np.ascontiguousarray(tri_v, dtype=np.int64)
        self.kind = np.ascontiguousarray(kind, dtype=np.int64)
        self.line = np.ascontiguousarray(line, dtype=np.int64)
        self.prim_v = np.ascontiguousarray(prim_v, dtype=np.int64).reshape(-1, 2)
        self.nv = self.kind.shape[0]
        T = self.tri_v.shape[0]
        # edge i of a triangle joins v[i+1] and v[i+2]
        a = self.tri_v[:, [1, 2, 0]]
        b = self.tri_v[:, [2, 0, 1]]
        key = (np.minimum(a, b) * self.nv + np.maximum(a, b)).ravel()
        # edges = distinct keys in increasing order; a stable sort keeps, for each edge, its
        # triangles in increasing id (flattened index = 3 t + i)
        order = np.argsort(key, kind="stable")
        sk = key[order]
        first_of = np.ones(sk.shape[0], dtype=bool)
        first_of[1:] = sk[1:] != sk[:-1]
        uniq = sk[first_of]
        inv = np.empty(sk.shape[0], dtype=np.int64)
        inv[order] = np.cumsum(first_of) - 1
        lo = uniq // self.nv
        self.edge_v = np.stack([lo, uniq - lo * self.nv], axis=1)
        self.edge_key = uniq
        self.tri_edge = inv.reshape(T, 3)
        E = uniq.shape[0]
        cnt = np.bincount(inv, minlength=E)
        if (cnt > 2).any():
            raise ValueError("an edge is shared by more than two triangles")
        # triangles of each edge, increasing id, with the edge's local index there
        first = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        self.edge_tri = -np.ones((E, 2), dtype=np.int64)
        self.edge_loc = -np.ones((E, 2), dtype=np.int64)
        for j in range(2):
            has = cnt > j
            f = order[first[has] + j]
            self.edge_tri[has, j] = f // 3
            self.edge_loc[has, j] = f % 3
        # opposite vertices and neighbouring edges in the order stated above
        self.edge_opp = -np.ones((E, 2), dtype=np.int64)
        self.edge_nbr = -np.ones((E, 4), dtype=np.int64)
        for j in range(2):
            has = self.edge_tri[:, j] >= 0
            t, i = self.edge_tri[has, j], self.edge_loc[has, j]
            self.edge_opp[has, j] = self.tri_v[t, i]
            self.edge_nbr[has, 2 * j] = self.tri_edge[t, (i + 1) % 3]
            self.edge_nbr[has, 2 * j + 1] = self.tri_edge[t, (i + 2) % 3]
        # vertex neighbours (sorted) as CSR
        both = np.concatenate([self.edge_v, self.edge_v[:, ::-1]])
        both = both[np.argsort(both[:, 0] * self.nv + both[:, 1])]
        self.nbr = both[:, 1]
        self.nbr_off = np.concatenate([[0], np.cumsum(np.bincount(both[:, 0], minlength=self.nv))])

    @property
    def n_edges(self):
        return self.edge_v.shape[0]

    def has_edge(self, a, b):
        key = np.minimum(a, b) * self.nv + np.maximum(a, b)
        pos = np.clip(np.searchsorted(self.edge_key, key), 0, self.n_edges - 1)
        return self.edge_key[pos] == key


def lengths(xy, a, b):
    dx = xy[b, 0] - xy[a, 0]
    dy = xy[b, 1] - xy[a, 1]
    return np.sqrt(dx * dx + dy * dy)


def direct_contractible(m: Mesh) -> np.ndarray:
    """Restrictions of the original geometry (Sec. 2.2.2, first paragraph)."""
    a, b = m.edge_v[:, 0], m.edge_v[:, 1]
    ka, kb = m.kind[a], m.kind[b]
    ok = np.ones(m.n_edges, dtype=bool)
    ok[(ka == ORIGINAL) & (kb == ORIGINAL)] = False
    for o, c in ((a, b), (b, a)):
        sel = (m.kind[o] == ORIGINAL) & (m.kind[c] == CONSTRAINED)
        ends = m.prim_v[m.line[c[sel]]]
        ok[np.nonzero(sel)[0]] = (ends[:, 0] == o[sel]) | (ends[:, 1] == o[sel])
    sel = (ka == CONSTRAINED) & (kb == CONSTRAINED)
    ok[sel] = m.line[a[sel]] == m.line[b[sel]]
    return ok


def one_hop_contractible(m: Mesh, xy, eps) -> np.ndarray:
    """1-hop topology rule (Sec. 2.2.2): every common neighbour of the edge's endpoints that is
    not one of its opposite vertices must lie strictly closer than eps to an opposite vertex."""
    a = m.edge_v[:, 0]
    deg = m.nbr_off[a + 1] - m.nbr_off[a]
    e = np.repeat(np.arange(m.n_edges), deg)
    start = np.repeat(m.nbr_off[a], deg)
    x = m.nbr[start + (np.arange(e.shape[0]) - np.repeat(np.cumsum(deg) - deg, deg))]
    b = m.edge_v[e, 1]
    o0, o1 = m.edge_opp[e, 0], m.edge_opp[e, 1]
    common = m.has_edge(x, b) & (x != b)
    nontrivial = common & (x != o0) & (x != o1)
    e, x, o0, o1 = e[nontrivial], x[nontrivial], o0[nontrivial], o1[nontrivial]
    close = lengths(xy, x, o0) < eps
    has1 = o1 >= 0
    close[has1] |= lengths(xy, x[has1], o1[has1]) < eps
    ok = np.ones(m.n_edges, dtype=bool)
    ok[e[~close]] = False
    return ok


# Collinearity (Sec. 2.2.2): three points are near-collinear when the area of their triangle is
# below this fraction of the area of the square with the triangle's perimeter (the paper calls
# it a small critical value without giving it; 0.01 is the ratio of a triangle with a 179-degree
# corner between two equal sides, where the angle penalty starts).
COLLINEAR = 0.01


def near_collinear(a, b, c) -> bool:
    """16 * area / perimeter^2 below COLLINEAR (a zero perimeter counts as collinear). Lengths as
    for edges; cross product (b - a) x (c - a)."""
    cross = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    area = 0.5 * abs(cross)

    def ln(u, w):
        dx = w[0] - u[0]
        dy = w[1] - u[1]
        return math.sqrt(dx * dx + dy * dy)
    per = (ln(a, b) + ln(b, c)) + ln(c, a)
    if not per > 0.0:
        return True
    return (16.0 * area) / (per * per) < COLLINEAR


def _dof(kind):
    return {ORIGINAL: 0, CONSTRAINED: 1, FREE: 2}[int(kind)]


def _vertex_triangles(m: Mesh):
    if not hasattr(m, "_vtri"):
        vt = [[] for _ in range(m.nv)]
        for t, tv in enumerate(m.tri_v.tolist()):
            for v in tv:
                vt[v].append(t)
        m._vtri = vt
        m._nbrs = [set(m.nbr[m.nbr_off[v]:m.nbr_off[v + 1]].tolist()) for v in range(m.nv)]
    return m._vtri, m._nbrs


def conditioning_bad(m: Mesh, xy, lo, tri) -> bool:
    """Sec. 2.2.2, conditioning: the triangle `tri` (three vertex ids, the contracted vertex
    already replaced by `lo`) is badly conditioned for good. Only ORIGINAL positions and the
    original edges of CONSTRAINED vertices are used (fixed during optimisation):
    - a FREE vertex: never;
    - three ORIGINAL: near-collinear;
    - two ORIGINAL o1, o2 and a CONSTRAINED s: near-collinear with s at each end of its original
      edge and at its middle ((a + b) * 0.5), all three;
    - one ORIGINAL o and CONSTRAINED s1, s2: their original edges are collinear with each other
      (both ends of the second near-collinear with the first) and with o;
    - three CONSTRAINED: all their original edges collinear with the first one.
    A triangle whose three vertices lie on one original edge is the flat-triangle case, judged by
    flat_ok instead (its trapped vertices may still be contracted away, as the paper's figure
    of that rule allows)."""
    kinds = [int(m.kind[v]) for v in tri]
    if FREE in kinds:
        return False
    for v, k in zip(tri, kinds):
        if k == CONSTRAINED and all(_on_line(m, x, int(m.line[v])) for x in tri):
            return False
    orig = [v for v, k in zip(tri, kinds) if k == ORIGINAL]
    cons = [v for v, k in zip(tri, kinds) if k == CONSTRAINED]
    P = lambda v: xy[v]
    ends = lambda s: (xy[m.prim_v[m.line[s], 0]], xy[m.prim_v[m.line[s], 1]])
    if len(orig) == 3:
        return near_collinear(*(P(v) for v in orig))
    if len(orig) == 2:
        a, b = ends(cons[0])
        mid = np.array([(a[0] + b[0]) * 0.5, (a[1] + b[1]) * 0.5])
        o1, o2 = P(orig[0]), P(orig[1])
        return all(near_collinear(o1, o2, q) for q in (a, b, mid))
    a1, b1 = ends(cons[0])
    lines_collinear = all(near_collinear(a1, b1, q) for s in cons[1:] for q in ends(s))
    if len(orig) == 1:
        return lines_collinear and near_collinear(a1, b1, P(orig[0]))
    return lines_collinear


def conditioning_ok(m: Mesh, xy, a, b) -> bool:
    """Sec. 2.2.2, conditioning restriction: when the contraction of edge (a, b) snaps the vertex
    with more degrees of freedom (FREE 2, CONSTRAINED 1, ORIGINAL 0) onto the other, every
    triangle of that vertex that does not hold the other becomes the triangle with the other in
    its place; the edge is not contractible if one of those is badly conditioned for good. Edges
    whose ends have equal degrees of freedom lose none and are not restricted here."""
    da, db = _dof(m.kind[a]), _dof(m.kind[b])
    if da == db:
        return True
    hi, lo = (a, b) if da > db else (b, a)
    vtri, _ = _vertex_triangles(m)
    for t in vtri[hi]:
        tv = [int(x) for x in m.tri_v[t]]
        if lo in tv:
            continue
        if conditioning_bad(m, xy, lo, [lo if x == hi else x for x in tv]):
            return False
    return True


def _on_line(m: Mesh, v, line) -> bool:
    k = int(m.kind[v])
    if k == CONSTRAINED:
        return int(m.line[v]) == line
    if k == ORIGINAL:
        return int(v) in (int(m.prim_v[line, 0]), int(m.prim_v[line, 1]))
    return False


def _length(xy, u, w):
    dx = xy[w, 0] - xy[u, 0]
    dy = xy[w, 1] - xy[u, 1]
    return math.sqrt(dx * dx + dy * dy)


def flat_ok(m: Mesh, xy, a, b, eps) -> bool:
    """Sec. 2.2.2, flat triangles (the paper's figure of a free vertex F fanned over an original
    edge): for an edge joining a FREE vertex F and a CONSTRAINED or ORIGINAL vertex C, the
    contraction would snap F onto C, and each triangle (F, X, Y) of F without C whose X and Y lie
    on an original edge L through C becomes the zero-area (C, X, Y). Its CONSTRAINED vertices are
    trapped. The edge is contractible only if every trapped vertex is already contracted to C or
    to an ORIGINAL vertex of L: joined to it by a path along L of edges shorter than eps through
    vertices of F's fan (F's neighbours on L, and C). 'On L': CONSTRAINED to L, or an ORIGINAL end
    of L."""
    ka, kb = int(m.kind[a]), int(m.kind[b])
    if ka == FREE and kb != FREE:
        F, C = a, b
    elif kb == FREE and ka != FREE:
        F, C = b, a
    else:
        return True
    vtri, nbrs = _vertex_triangles(m)
    for t in vtri[F]:
        tv = [int(x) for x in m.tri_v[t]]
        if C in tv:
            continue
        X, Y = [x for x in tv if x != F]
        cx = [x for x in (X, Y) if int(m.kind[x]) == CONSTRAINED]
        if not cx:
            continue
        L = int(m.line[cx[0]])
        if not (_on_line(m, X, L) and _on_line(m, Y, L) and _on_line(m, C, L)):
            continue
        fan = {x for x in nbrs[F] if _on_line(m, x, L)} | {C}
        for T in cx:
            # walk along L through the fan over edges shorter than eps
            seen, todo, reached = {T}, [T], False
            while todo and not reached:
                u = todo.pop()
                for w in nbrs[u]:
                    if w in fan and w not in seen and _length(xy, u, w) < eps:
                        if w == C or int(m.kind[w]) == ORIGINAL:
                            reached = True
                            break
                        seen.add(w)
                        todo.append(w)
            if not reached:
                return False
    return True


def _near_collinear_v(a, b, c):
    """near_collinear over arrays of points (rows), the same operations in the same order."""
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    area = 0.5 * np.abs(cross)

    def ln(u, w):
        dx = w[:, 0] - u[:, 0]
        dy = w[:, 1] - u[:, 1]
        return np.sqrt(dx * dx + dy * dy)
    per = (ln(a, b) + ln(b, c)) + ln(c, a)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = (16.0 * area) / (per * per)
    return ~(per > 0.0) | (r < COLLINEAR)


def _on_line_v(m: Mesh, v, L):
    k = m.kind[v]
    return (((k == CONSTRAINED) & (m.line[v] == L)) |
            ((k == ORIGINAL) & ((m.prim_v[L, 0] == v) | (m.prim_v[L, 1] == v))))


def _star_pairs(m: Mesh, edges, centre, other):
    """(edge index, triangle) for every triangle of centre[k] that does not hold other[k]."""
    T = m.tri_v.shape[0]
    flat_v = m.tri_v.ravel()
    order = np.argsort(flat_v, kind="stable")
    vt = order // 3
    off = np.concatenate([[0], np.cumsum(np.bincount(flat_v, minlength=m.nv))])
    deg = off[centre + 1] - off[centre]
    k = np.repeat(np.arange(edges.shape[0]), deg)
    start = np.repeat(off[centre], deg)
    t = vt[start + (np.arange(k.shape[0]) - np.repeat(np.cumsum(deg) - deg, deg))]
    keep = ~(m.tri_v[t] == other[k][:, None]).any(axis=1)
    return k[keep], t[keep]


def conditioning_contractible(m: Mesh, xy) -> np.ndarray:
    """conditioning_ok of every edge, vectorised (the same decisions)."""
    ok = np.ones(m.n_edges, dtype=bool)
    a, b = m.edge_v[:, 0], m.edge_v[:, 1]
    dof = np.where(m.kind == ORIGINAL, 0, np.where(m.kind == CONSTRAINED, 1, 2))
    cand = np.nonzero(dof[a] != dof[b])[0]
    if cand.size == 0 or m.prim_v.shape[0] == 0:
        return ok
    hi = np.where(dof[a[cand]] > dof[b[cand]], a[cand], b[cand])
    lo = np.where(dof[a[cand]] > dof[b[cand]], b[cand], a[cand])
    k, t = _star_pairs(m, cand, hi, lo)
    tri = np.where(m.tri_v[t] == hi[k][:, None], lo[k][:, None], m.tri_v[t])
    kinds = m.kind[tri]
    sel = ~(kinds == FREE).any(axis=1)
    k, tri, kinds = k[sel], tri[sel], kinds[sel]
    # three vertices on the line of one of its constrained vertices: the flat-triangle case
    flat = np.zeros(k.shape[0], dtype=bool)
    for j in range(3):
        cj = kinds[:, j] == CONSTRAINED
        Lj = np.where(cj, m.line[tri[:, j]], 0)
        flat |= cj & _on_line_v(m, tri[:, 0], Lj) & _on_line_v(m, tri[:, 1], Lj) & \
            _on_line_v(m, tri[:, 2], Lj)
    k, tri, kinds = k[~flat], tri[~flat], kinds[~flat]
    bad = np.zeros(k.shape[0], dtype=bool)
    isorig = kinds == ORIGINAL
    no = isorig.sum(axis=1)
    # the vertices of each kind in triangle order
    ordo = np.argsort(~isorig, axis=1, kind="stable")
    ordc = np.argsort(isorig, axis=1, kind="stable")
    O = np.take_along_axis(tri, ordo, axis=1)
    Cn = np.take_along_axis(tri, ordc, axis=1)
    P = lambda v: xy[v]
    E0 = m.prim_v[np.where(m.kind[Cn[:, 0]] == CONSTRAINED, m.line[Cn[:, 0]], 0)]
    A, B = xy[E0[:, 0]], xy[E0[:, 1]]
    s3 = no == 3
    bad[s3] = _near_collinear_v(P(O[s3, 0]), P(O[s3, 1]), P(O[s3, 2]))
    s2 = no == 2
    if s2.any():
        a2, b2 = A[s2], B[s2]
        mid = np.stack([(a2[:, 0] + b2[:, 0]) * 0.5, (a2[:, 1] + b2[:, 1]) * 0.5], axis=1)
        o1, o2 = P(O[s2, 0]), P(O[s2, 1])
        bad[s2] = (_near_collinear_v(o1, o2, a2) & _near_collinear_v(o1, o2, b2) &
                   _near_collinear_v(o1, o2, mid))
    s1 = no <= 1
    if s1.any():
        lines = np.ones(k.shape[0], dtype=bool)
        for j in (1, 2):
            has = s1 & (3 - no > j)
            Ej = m.prim_v[m.line[Cn[has, j]]]
            lines[has] &= (_near_collinear_v(A[has], B[has], xy[Ej[:, 0]]) &
                           _near_collinear_v(A[has], B[has], xy[Ej[:, 1]]))
        one = s1 & (no == 1)
        bad[one] = lines[one] & _near_collinear_v(A[one], B[one], P(O[one, 0]))
        zero = s1 & (no == 0)
        bad[zero] = lines[zero]
    ok[cand[np.unique(k[bad])]] = False
    return ok


def contractible(m: Mesh, xy, eps) -> np.ndarray:
    """Sec. 2.2.2: the original-geometry, conditioning, 1-hop and flat-triangle restrictions."""
    xy = np.asarray(xy, dtype=np.float64)
    ok = direct_contractible(m) & one_hop_contractible(m, xy, eps) & \
        conditioning_contractible(m, xy)
    # the flat-triangle rule can only restrict an edge (F FREE, C not) where a triangle of F
    # without C has its other two vertices on an original edge through C; the rest is flat_ok
    a, b = m.edge_v[:, 0], m.edge_v[:, 1]
    fa, fb = m.kind[a] == FREE, m.kind[b] == FREE
    cand = np.nonzero(ok & (fa != fb))[0]
    if cand.size and m.prim_v.shape[0]:
        F = np.where(fa[cand], a[cand], b[cand])
        C = np.where(fa[cand], b[cand], a[cand])
        k, t = _star_pairs(m, cand, F, C)
        tv = m.tri_v[t]
        isF = tv == F[k][:, None]
        XY = tv[~isF].reshape(-1, 2)
        cx = m.kind[XY[:, 0]] == CONSTRAINED
        cy = m.kind[XY[:, 1]] == CONSTRAINED
        L = np.where(cx, m.line[XY[:, 0]], np.where(cy, m.line[XY[:, 1]], 0))
        hit = (cx | cy) & _on_line_v(m, XY[:, 0], L) & _on_line_v(m, XY[:, 1], L) & \
            _on_line_v(m, C[k], L)
        for j in np.unique(k[hit]):
            e = cand[j]
            if not flat_ok(m, xy, int(a[e]), int(b[e]), eps):
                ok[e] = False
    return ok


def edge_values(m: Mesh, xy, p: Params, edges):
    """(contractible, c, w) of the given edges only, from the same definitions applied one edge at
    a time (for sampling meshes too large to evaluate whole)."""
    xy = np.asarray(xy, dtype=np.float64)

    def contr_one(e):
        a, b = m.edge_v[e]
        ka, kb = m.kind[a], m.kind[b]
        if ka == ORIGINAL and kb == ORIGINAL:
            return False
        for o, c in ((a, b), (b, a)):
            if m.kind[o] == ORIGINAL and m.kind[c] == CONSTRAINED:
                if o not in m.prim_v[m.line[c]]:
                    return False
        if ka == CONSTRAINED and kb == CONSTRAINED and m.line[a] != m.line[b]:
            return False
        na = set(m.nbr[m.nbr_off[a]:m.nbr_off[a + 1]].tolist())
        nb = set(m.nbr[m.nbr_off[b]:m.nbr_off[b + 1]].tolist())
        opp = [x for x in m.edge_opp[e] if x >= 0]
        for h in sorted((na & nb) - set(opp)):
            if not any(lengths(xy, np.array([h]), np.array([o]))[0] < p.eps for o in opp):
                return False
        return conditioning_ok(m, xy, int(a), int(b)) and flat_ok(m, xy, int(a), int(b), p.eps)

    def c_one(e):
        ln = lengths(xy, m.edge_v[e:e + 1, 0], m.edge_v[e:e + 1, 1])
        return c_eps(ln, np.array([contr_one(e)]), p.eps)[0]

    out_c, out_k, out_w = [], [], []
    for e in edges:
        e = int(e)
        k = contr_one(e)
        out_k.append(k)
        out_c.append(c_one(e))
        if p.polish:
            out_w.append(1.0)
            continue
        n = m.edge_nbr[e]
        x = c_one(n[0]) * c_one(n[1])
        if n[2] >= 0:
            x = x * c_one(n[2])
            x = x * c_one(n[3])
        out_w.append(float(x * merge_correction(np.array(x))))
    return np.array(out_k), np.array(out_c), np.array(out_w)


def c_eps(length, contr, eps):
    """Contraction weight (Sec. 2.2.1)."""
    return np.where(contr, 0.5 + 0.5 * np.minimum(1.0, length / eps), 1.0)


def merge_correction(x):
    """M (Sec. 2.2.1): 0 below 1/4, 4x - 1 on [1/4, 1/2], 1 above."""
    return np.where(x < 0.25, 0.0, np.where(x <= 0.5, 4.0 * x - 1.0, 1.0))


def edge_weight(m: Mesh, c):
    x = c[m.edge_nbr[:, 0]] * c[m.edge_nbr[:, 1]]
    two = m.edge_nbr[:, 2] >= 0
    x[two] = x[two] * c[m.edge_nbr[two, 2]]
    x[two] = x[two] * c[m.edge_nbr[two, 3]]
    return x * merge_correction(x)


def angle_terms(m: Mesh, xy, p: Params):
    """(T, 3) penalty of corner i (at v[i]) of every triangle (Sec. 2.2.3)."""
    out = np.zeros(m.tri_v.shape, dtype=np.float64)
    for i in range(3):
        o, u, w = m.tri_v[:, i], m.tri_v[:, (i + 1) % 3], m.tri_v[:, (i + 2) % 3]
        ux, uy = xy[u, 0] - xy[o, 0], xy[u, 1] - xy[o, 1]
        wx, wy = xy[w, 0] - xy[o, 0], xy[w, 1] - xy[o, 1]
        lu = np.sqrt(ux * ux + uy * uy)
        lw = np.sqrt(wx * wx + wy * wy)
        den = lu * lw
        ok = den > 0
        cos = np.zeros_like(den)
        cos[ok] = (ux[ok] * wx[ok] + uy[ok] * wy[ok]) / den[ok]
        if p.polish:
            t = np.maximum(0.0, cos - (1.0 - p.delta)) / p.delta
        else:
            t = np.maximum(0.0, (-1.0 + p.delta) - cos) / p.delta
        out[:, i] = np.where(ok, t, 0.0)
    return out


def terms(m: Mesh, xy, p: Params) -> dict:
    """Every term of f, separately."""
    xy = np.asarray(xy, dtype=np.float64)
    ln = lengths(xy, m.edge_v[:, 0], m.edge_v[:, 1])
    contr = contractible(m, xy, p.eps)
    c = c_eps(ln, contr, p.eps)
    w = np.ones(m.n_edges) if p.polish else edge_weight(m, c)
    return {"length": ln, "contractible": contr, "c": c, "w": w, "edge": w * ln,
            "angle": angle_terms(m, xy, p), "short": np.maximum(0.0, p.eps0 - ln) / p.eps0}


def objective(m: Mesh, xy, p: Params) -> dict:
    """f and its parts (Sec. 2.2.4), with the per-edge values."""
    t = terms(m, xy, p)
    wc, pa, pl = t["edge"].sum(), t["angle"].sum(), t["short"].sum()
    t.update(wcontr=wc, pangle=pa, plen=pl, f=wc + p.mu_angle * pa + p.mu_len * pl)
    return t


MOVED, FOLDED, FIXED, BAD = 1, 0, -1, -2


def move_status(m: Mesh, xy, v, q) -> int:
    """1: valid move; 0: some triangle of v would not stay strictly counter-clockwise (exact);
    -1: v is an original vertex (not movable); -2: v out of range or q not finite."""
    if not (0 <= v < m.nv) or not np.isfinite(q).all():
        return BAD
    if m.kind[v] == ORIGINAL:
        return FIXED
    moved = xy.copy()
    moved[v] = q
    for t in np.nonzero((m.tri_v == v).any(axis=1))[0]:
        a, b, c = (moved[k] for k in m.tri_v[t])
        if orient(a, b, c) <= 0:
            return FOLDED
    return MOVED


def delta_f(m: Mesh, xy, p: Params, v, q, base: dict | None = None) -> tuple[int, float, float]:
    """(status, delta_f, bound) of moving vertex v to q. delta_f is +inf unless the move is valid;
    bound is the sum of the absolute term differences (the scale of delta_f's rounding). base may
    hold terms(m, xy, p), computed once for several moves from the same positions."""
    xy = np.asarray(xy, dtype=np.float64)
    st = move_status(m, xy, int(v), np.asarray(q, dtype=np.float64))
    if st != MOVED:
        return st, float("inf"), 0.0
    moved = xy.copy()
    moved[v] = q
    t0 = base if base is not None else terms(m, xy, p)
    t1 = terms(m, moved, p)
    de = t1["edge"] - t0["edge"]
    da = (t1["angle"] - t0["angle"]).ravel()
    ds = t1["short"] - t0["short"]
    df = de.sum() + p.mu_angle * da.sum() + p.mu_len * ds.sum()
    bound = np.abs(de).sum() + p.mu_angle * np.abs(da).sum() + p.mu_len * np.abs(ds).sum()
    return st, float(df), float(bound)


ACCEPTED, REJECTED = 1, 2


def project(m: Mesh, xy, v, d):
    """A constrained vertex's displacement projected on its original edge (a, b): s * e with
    e = b - a and s = (d.e)/(e.e); other kinds keep d."""
    d = np.asarray(d, dtype=np.float64)
    if m.kind[v] != CONSTRAINED:
        return d
    a, b = m.prim_v[m.line[v]]
    ex, ey = xy[b, 0] - xy[a, 0], xy[b, 1] - xy[a, 1]
    s = (d[0] * ex + d[1] * ey) / (ex * ex + ey * ey)
    return np.array([s * ex, s * ey])


def metropolis_chain(m: Mesh, xy, p: Params, temperature, vid, disp, u):
    """Single-vertex Metropolis steps (Sec. 3.1, acceptance min(1, exp(-delta f / T)); moves of
    Sec. 3.2.2), applied one after another in the given order. Returns the final positions and,
    per move, the status (ACCEPTED, REJECTED or the move_status codes), delta f and the decision
    margin |delta f + T ln u| (a decision within rounding of 0 may differ between implementations)."""
    xy = np.array(xy, dtype=np.float64)
    st = np.zeros(len(vid), dtype=np.int64)
    df = np.full(len(vid), np.inf)
    margin = np.full(len(vid), np.inf)
    for i, v in enumerate(vid):
        v = int(v)
        if not (0 <= v < m.nv):
            st[i] = BAD
            continue
        q = xy[v] + project(m, xy, v, disp[i])
        s, d, bound = delta_f(m, xy, p, v, q)
        df[i] = d
        if s != MOVED:
            st[i] = s
            continue
        with np.errstate(divide="ignore", over="ignore"):
            accept = d <= 0.0 or u[i] < np.exp(-np.float64(d) / np.float64(temperature))
        if accept:
            st[i] = ACCEPTED
            xy[v] = q
        else:
            st[i] = REJECTED
        margin[i] = abs(d + temperature * np.log(u[i])) if u[i] > 0 else np.inf
    return xy, st, df, margin


def joint_move(m: Mesh, xy, p: Params, temperature, lam, vid, xi, u):
    """The second variant of Sec. 3.2.2: the distinct movable vertices vid move together, vertex
    vid[i] by (lam * sqrt(star area of vid[i])) * xi[i] at the positions before the move,
    projected for constrained vertices; one Metropolis decision (Sec. 3.1) with u on the change of
    f, taken as the sum over edges and triangles of every term's new minus old value. Returns
    (status, delta, bound, positions after, margin): status ACCEPTED, REJECTED, FOLDED (a triangle
    of a moved vertex not strictly counter-clockwise) or BAD (an id out of range, original or
    repeated, or a draw not finite); bound is the reordering bound of delta's sums; margin as in
    metropolis_chain."""
    xy = np.array(xy, dtype=np.float64)
    vid = [int(v) for v in vid]
    xi = np.asarray(xi, dtype=np.float64).reshape(-1, 2)
    if (len(set(vid)) != len(vid) or not np.isfinite(xi).all()
            or any(not (0 <= v < m.nv) or m.kind[v] == ORIGINAL for v in vid)):
        return BAD, np.inf, 0.0, xy, np.inf
    new = xy.copy()
    for i, v in enumerate(vid):
        k = lam * np.sqrt(star_area(m, xy, v))
        new[v] = xy[v] + project(m, xy, v, np.array([k * xi[i, 0], k * xi[i, 1]]))
    return _joint_decide(m, xy, new, vid, p, temperature, u)


def _joint_decide(m: Mesh, xy, new, vid, p: Params, temperature, u):
    """Validity, change of f and Metropolis decision of a joint move from xy to new, which differ
    at the vertices vid (see joint_move)."""
    moved = np.zeros(m.nv, dtype=bool)
    moved[vid] = True
    for t in np.nonzero(moved[m.tri_v].any(axis=1))[0]:
        a, b, c = (new[k] for k in m.tri_v[t])
        if orient(a, b, c) <= 0:
            return FOLDED, np.inf, 0.0, xy, np.inf
    t0, t1 = terms(m, xy, p), terms(m, new, p)
    de, da, dl = t1["edge"] - t0["edge"], t1["angle"] - t0["angle"], t1["short"] - t0["short"]
    d = de.sum() + p.mu_angle * da.sum() + p.mu_len * dl.sum()
    u53 = 2.0 ** -53
    bound = 2 * (de.size + da.size) * u53 * (np.abs(de).sum() + p.mu_angle * np.abs(da).sum()
                                            + p.mu_len * np.abs(dl).sum()) + 4 * u53 * abs(d)
    with np.errstate(divide="ignore", over="ignore"):
        accept = d <= 0.0 or u < np.exp(-np.float64(d) / np.float64(temperature))
        margin = abs(d + temperature * np.log(u)) if u > 0 else np.inf
    if accept:
        return ACCEPTED, d, bound, new, margin
    return REJECTED, d, bound, xy, margin


def joint_groups(m: Mesh, xy, p: Params, temperature, lam, centres, xi, rd, u):
    """The second variant of Sec. 3.2.3: the groups of several centres (group_members with
    d = (0.5 + 4.5 rd[i]) eps, at the positions before the move) move together, each by
    (lam * sqrt(group area)) * xi[i] projected per member, a vertex held by several groups with
    the displacement of the first of them in centre order (the paper leaves overlaps open); one
    decision as in joint_move. BAD when a centre is out of range or original, or a draw is not
    finite. Returns what joint_move returns."""
    xy = np.array(xy, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64).reshape(-1, 2)
    rd = np.asarray(rd, dtype=np.float64)
    cs = [int(c) for c in centres]
    if (not np.isfinite(xi).all() or not np.isfinite(rd).all()
            or any(not (0 <= c < m.nv) or m.kind[c] == ORIGINAL for c in cs)):
        return BAD, np.inf, 0.0, xy, np.inf
    new, owned = xy.copy(), {}
    for i, c in enumerate(cs):
        members = group_members(m, xy, c, (0.5 + 4.5 * rd[i]) * p.eps)
        k = lam * math.sqrt(group_area(m, xy, members))
        D = np.array([k * xi[i, 0], k * xi[i, 1]])
        for v in members:
            if v not in owned:
                owned[v] = i
                new[v] = xy[v] + project(m, xy, v, D)
    return _joint_decide(m, xy, new, sorted(owned), p, temperature, u)


def star_area(m: Mesh, xy, v):
    """Area of the triangles of vertex v, summed in increasing triangle id, each as
    0.5 * ((b - a) x (c - a)) on its vertices in their stored order."""
    s = 0.0
    for t in np.nonzero((m.tri_v == v).any(axis=1))[0]:
        a, b, c = (xy[k] for k in m.tri_v[t])
        s = s + 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
    return s


def annealing_schedule(m: Mesh, xy, p: Params, temperatures, eps, lambda0, target, order, xi, u):
    """Simulated annealing (Sec. 3.1) with temperature and contraction length lowered together
    (Sec. 3.3.1) and an adaptive step scale (Sec. 3.2): sweep k visits the vertices of `order`
    one after another; the move of vertex v is (lambda_k * sqrt(star area of v)) * xi[k][i] (Sec.
    3.2.2), projected for constrained vertices and accepted by the Metropolis rule with u[k][i].
    After a sweep, with a its accepted fraction, lambda is scaled by 1 + (a - target) limited to
    [1/2, 2] (the paper targets an acceptance rate without giving the rule). Returns the final
    positions, the step scale of every sweep, its accepted moves and the smallest decision margin."""
    xy = np.array(xy, dtype=np.float64)
    lam = float(lambda0)
    lams, accs, margin_min = [], [], np.inf
    for k in range(len(temperatures)):
        pk = Params(eps[k], p.delta, p.eps0, p.mu_angle, p.mu_len, p.polish)
        acc = 0
        for i, v in enumerate(order):
            v = int(v)
            sc = lam * np.sqrt(star_area(m, xy, v))
            d = np.array([sc * xi[k][i][0], sc * xi[k][i][1]])
            _, st, _, margin = metropolis_chain(m, xy, pk, temperatures[k], [v], [d], [u[k][i]])
            if st[0] == ACCEPTED:
                xy[v] = xy[v] + project(m, xy, v, d)
                acc += 1
            margin_min = min(margin_min, margin[0])
        lams.append(lam)
        accs.append(acc)
        a = acc / len(order)
        lam = lam * min(2.0, max(0.5, 1.0 + (a - target)))
    return xy, np.array(lams), np.array(accs), margin_min


# Proposal kinds of proposal_chain and the status of a vertex the perturbation does not apply to.
RESAMPLE, SWAP, CONTRACT = 1, 2, 3
SKIPPED = 3


def _tri_area(xy, tv):
    a, b, c = (xy[k] for k in tv)
    return 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))


def resample_in_star(m: Mesh, xy, v, r0, r1, r2):
    """Sec. 3.2.4: a position uniform by area over the triangles around vertex v (its star).
    With r0, r1, r2 uniform on [0, 1): the triangle is the first, in increasing id, at which the
    running sum of the star's areas (each as in star_area) exceeds r0 times their total; the point
    is (1 - s) a + s (1 - r2) b + s r2 c on its vertices in stored order, s = sqrt(r1), which is
    uniform on the triangle (Osada, Funkhouser, Chazelle and Dobkin, 2002)."""
    tris = np.nonzero((m.tri_v == v).any(axis=1))[0]
    areas = [_tri_area(xy, m.tri_v[t]) for t in tris]
    total = 0.0
    for a in areas:
        total = total + a
    target = r0 * total
    run, pick = 0.0, tris[-1]
    for t, a in zip(tris, areas):
        run = run + a
        if target < run:
            pick = t
            break
    a, b, c = (xy[k] for k in m.tri_v[pick])
    s = math.sqrt(r1)
    ka, kb, kc = 1.0 - s, s * (1.0 - r2), s * r2
    return np.array([ka * a[0] + kb * b[0] + kc * c[0], ka * a[1] + kb * b[1] + kc * c[1]])


def incident_lengths(m: Mesh, xy, v, q=None):
    """Lengths of the edges at v (neighbours in increasing id), with v at q when given."""
    nb = m.nbr[m.nbr_off[v]:m.nbr_off[v + 1]]
    P = xy[v] if q is None else q
    dx = xy[nb, 0] - P[0]
    dy = xy[nb, 1] - P[1]
    return np.sqrt(dx * dx + dy * dy)


def propose(m: Mesh, xy, p: Params, v, kind, r):
    """The position proposed for vertex v by one perturbation, or None when it does not apply.
    r holds four numbers: r[0], r[1], r[2] uniform on [0, 1) and, for SWAP, (r[2], r[3]) a point of
    the unit disk.
    - RESAMPLE (Sec. 3.2.4): resample_in_star with r[0], r[1], r[2].
    - SWAP (Sec. 3.2.5): l = (0.2 + 1.8 r[0]) eps, uniform on [0.2 eps, 2 eps); v must have an edge
      shorter than l; its neighbour w of rank floor(r[1] deg) (increasing id) is chosen and the
      position is w + l (r[2], r[3]), uniform on the disk of radius l around w.
    - CONTRACT (Sec. 3.2.6): the RESAMPLE position, kept only when v is contracted (has an edge
      shorter than eps) at exactly one of its old and new positions: one try, no repetition.
    A constrained vertex's move q - o is projected on its original edge first (Sec. 3.2.1)."""
    o = xy[v]
    if kind in (RESAMPLE, CONTRACT):
        q = resample_in_star(m, xy, v, r[0], r[1], r[2])
    elif kind == SWAP:
        ln = (0.2 + 1.8 * r[0]) * p.eps
        if not (incident_lengths(m, xy, v) < ln).any():
            return None
        nb = m.nbr[m.nbr_off[v]:m.nbr_off[v + 1]]
        w = nb[min(int(r[1] * nb.shape[0]), nb.shape[0] - 1)]
        q = np.array([xy[w, 0] + ln * r[2], xy[w, 1] + ln * r[3]])
    else:
        raise ValueError(f"unknown proposal kind {kind}")
    q = o + project(m, xy, v, q - o)
    if kind == CONTRACT:
        before = bool((incident_lengths(m, xy, v) < p.eps).any())
        after = bool((incident_lengths(m, xy, v, q) < p.eps).any())
        if before == after:
            return None
    return q


def proposal_chain(m: Mesh, xy, p: Params, temperature, kind, vid, r, u):
    """Metropolis steps (Sec. 3.1) with the proposals of one kind (see propose), for the vertices
    of vid one after another, each proposal drawn from the positions its predecessors left.
    Returns the final positions and, per vertex, the status (ACCEPTED, REJECTED, SKIPPED or the
    move_status codes), delta f and the decision margin, as metropolis_chain."""
    xy = np.array(xy, dtype=np.float64)
    n = len(vid)
    st = np.zeros(n, dtype=np.int64)
    df = np.full(n, np.inf)
    margin = np.full(n, np.inf)
    for i, v in enumerate(vid):
        v = int(v)
        q = propose(m, xy, p, v, kind, r[i])
        if q is None:
            st[i] = SKIPPED
            continue
        s, d, _ = delta_f(m, xy, p, v, q)
        df[i] = d
        if s != MOVED:
            st[i] = s
            continue
        with np.errstate(divide="ignore", over="ignore"):
            accept = d <= 0.0 or u[i] < np.exp(-np.float64(d) / np.float64(temperature))
        st[i] = ACCEPTED if accept else REJECTED
        if accept:
            xy[v] = q
        margin[i] = abs(d + temperature * np.log(u[i])) if u[i] > 0 else np.inf
    return xy, st, df, margin


def group_members(m: Mesh, xy, c, d):
    """Sec. 3.2.3: the group of centre c is every movable (not ORIGINAL) vertex whose distance to
    c is at most d, whether or not an edge joins it to c, with no limit on its size: c first,
    then the others in increasing id. The distance is sqrt(dx*dx + dy*dy) of the coordinate
    differences, as for edge lengths. (The paper finds these vertices with a uniform grid; a scan
    over all vertices finds the same ones.)"""
    v = np.arange(m.nv)
    dx = xy[:, 0] - xy[c, 0]
    dy = xy[:, 1] - xy[c, 1]
    dist = np.sqrt(dx * dx + dy * dy)
    near = (dist <= d) & (m.kind != ORIGINAL) & (v != c)
    return [int(c)] + [int(w) for w in v[near]]


def group_area(m: Mesh, xy, members):
    """Area of the triangles holding any member, each once: members in order, each member's
    triangles in increasing id, a triangle counted at the first member it holds; areas as in
    star_area, summed in that order."""
    s = 0.0
    for j, v in enumerate(members):
        for t in np.nonzero((m.tri_v == v).any(axis=1))[0]:
            if any(w in members[:j] for w in m.tri_v[t]):
                continue
            s = s + _tri_area(xy, m.tri_v[t])
    return s


def group_move(m: Mesh, xy, p: Params, c, lam, xi, rd):
    """The group move of centre c (Sec. 3.2.3): d = (0.5 + 4.5 rd) eps, uniform on [eps/2, 5 eps);
    every member moves by (lam * sqrt(group area)) * xi, projected on its original edge when
    constrained. Returns (members, new positions)."""
    d = (0.5 + 4.5 * rd) * p.eps
    members = group_members(m, xy, c, d)
    k = lam * math.sqrt(group_area(m, xy, members))
    D = np.array([k * xi[0], k * xi[1]])
    return members, [xy[v] + project(m, xy, v, D) for v in members]


def group_chain(m: Mesh, xy, p: Params, temperature, lam, centres, xi, rd, u):
    """Metropolis steps (Sec. 3.1) with group moves, the centres one after another, each group
    taken at the positions its predecessors left. A move is
    valid when every triangle holding a member is strictly counter-clockwise afterwards (exact);
    its delta f is f(moved) - f(current) over every term. Returns the final positions and, per
    centre, the status (ACCEPTED, REJECTED, FOLDED), delta f, the decision margin and the
    number of members."""
    xy = np.array(xy, dtype=np.float64)
    n = len(centres)
    st = np.zeros(n, dtype=np.int64)
    df = np.full(n, np.inf)
    margin = np.full(n, np.inf)
    size = np.zeros(n, dtype=np.int64)
    for i, c in enumerate(centres):
        members, qs = group_move(m, xy, p, int(c), lam, xi[i], rd[i])
        size[i] = len(members)
        moved = xy.copy()
        for v, q in zip(members, qs):
            moved[v] = q
        tris = np.nonzero(np.isin(m.tri_v, members).any(axis=1))[0]
        if any(orient(*moved[m.tri_v[t]]) <= 0 for t in tris):
            st[i] = FOLDED
            continue
        t0, t1 = terms(m, xy, p), terms(m, moved, p)
        d = float((t1["edge"] - t0["edge"]).sum() + p.mu_angle * (t1["angle"] - t0["angle"]).sum()
                  + p.mu_len * (t1["short"] - t0["short"]).sum())
        df[i] = d
        with np.errstate(divide="ignore", over="ignore"):
            accept = d <= 0.0 or u[i] < np.exp(-np.float64(d) / np.float64(temperature))
        st[i] = ACCEPTED if accept else REJECTED
        if accept:
            xy = moved
        margin[i] = abs(d + temperature * np.log(u[i])) if u[i] > 0 else np.inf
    return xy, st, df, margin, size
