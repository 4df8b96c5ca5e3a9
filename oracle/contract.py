"""Contraction of short edges (fuzzy topology to true topology): TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU leg may import this module. The
library never does and shares no code with it.

What is computed (paper Sec. 3.4.1, with the readings stated here):
- Contraction works in passes. A pass lists every edge shorter than eps at the start of the pass,
  in increasing (length, lower vertex id, higher vertex id), and tries each in turn that is still
  an edge and still shorter than eps. Passes repeat until one contracts nothing (the paper
  re-tries edges that failed, as neighbouring contractions can lift their restrictions).
- An edge (a, b) is tried only if the original geometry allows it (Sec. 2.2.2): not two original
  vertices; not an original vertex with a constrained one whose original edge does not end at it;
  not two constrained vertices on different original edges.
- The survivor and its position follow the degrees of freedom (Sec. 3.4.1): an original vertex
  survives where it is; a constrained vertex survives a free one where it is; two vertices of the
  same kind (free, or constrained to one original edge) merge into the lower id at a point of the
  edge, tried at a + t (b - a) for t = 1/2, 1/4, 3/4, 0, 1 in that order.
- A contraction is kept only if the topology stays a triangulation: the common neighbours of a and
  b are exactly the vertices opposite the edge (the link condition); an interior edge whose two
  ends both lie on the hull is not contracted; no remaining triangle of the merged vertex has all
  three vertices on one original edge (its ends or vertices constrained to it: a triangle of zero
  area in intent, whatever rounding makes of it, as the paper's strict convexity for flips also
  excludes); and every remaining triangle of the merged vertex is strictly counter-clockwise at
  the chosen position (exact orientation). The edge's one or two
  triangles disappear and the other vertex is replaced by the survivor everywhere.
- At the end, surviving vertices are renumbered in increasing old id and surviving triangles kept
  in increasing old id, each with its vertex order (the removed vertex replaced by the survivor).

Edge lengths are sqrt(dx*dx + dy*dy) in binary64.
"""
from __future__ import annotations

import math

import numpy as np

from . import orient
from .objective import CONSTRAINED, FREE, ORIGINAL

TRIES = (0.5, 0.25, 0.75, 0.0, 1.0)


def _len(xy, a, b):
    dx = xy[b][0] - xy[a][0]
    dy = xy[b][1] - xy[a][1]
    return math.sqrt(dx * dx + dy * dy)


def kinds_allow(kind, line, prim_v, a, b):
    """The original-geometry restriction of Sec. 2.2.2 for the edge (a, b)."""
    ka, kb = kind[a], kind[b]
    if ka == ORIGINAL and kb == ORIGINAL:
        return False
    if ka == ORIGINAL and kb == CONSTRAINED:
        return a in prim_v[line[b]]
    if kb == ORIGINAL and ka == CONSTRAINED:
        return b in prim_v[line[a]]
    if ka == CONSTRAINED and kb == CONSTRAINED:
        return line[a] == line[b]
    return True


def contract(tri_v, kind, line, prim_v, xy, eps):
    """Contract the edges shorter than eps. Returns (tri_v, kind, line, xy, old_to_new) of the
    contracted triangulation (old_to_new[v] = the new id of v's survivor) and the number of
    contractions made."""
    tris = [list(map(int, t)) for t in np.asarray(tri_v).reshape(-1, 3)]
    alive_t = [True] * len(tris)
    kind = [int(k) for k in kind]
    line = [int(k) for k in line]
    prim_v = [tuple(map(int, p)) for p in np.asarray(prim_v).reshape(-1, 2)]
    xy = [tuple(map(float, p)) for p in np.asarray(xy, dtype=np.float64)]
    nv = len(xy)
    star = [set() for _ in range(nv)]
    for t, tv in enumerate(tris):
        for v in tv:
            star[v].add(t)
    merged_into = list(range(nv))

    def edges_of(v):
        """Neighbours of v with the number of triangles on each edge."""
        cnt = {}
        for t in star[v]:
            for w in tris[t]:
                if w != v:
                    cnt[w] = cnt.get(w, 0) + 1
        return cnt

    def on_hull(v):
        return any(c == 1 for c in edges_of(v).values())

    def try_edge(a, b):
        if not kinds_allow(kind, line, prim_v, a, b):
            return False
        shared = sorted(star[a] & star[b])
        opp = set()
        for t in shared:
            opp.update(w for w in tris[t] if w != a and w != b)
        if set(edges_of(a)) & set(edges_of(b)) != opp:
            return False  # link condition
        if len(shared) == 2 and on_hull(a) and on_hull(b):
            return False
        if kind[a] == ORIGINAL or (kind[a] == CONSTRAINED and kind[b] == FREE):
            s, r, cands = a, b, [xy[a]]
        elif kind[b] == ORIGINAL or (kind[b] == CONSTRAINED and kind[a] == FREE):
            s, r, cands = b, a, [xy[b]]
        else:
            s, r = a, b
            ax, ay = xy[a]
            dx, dy = xy[b][0] - ax, xy[b][1] - ay
            cands = [(ax + t * dx, ay + t * dy) for t in TRIES]
        rest = sorted((star[a] | star[b]) - set(shared))

        def on_edge(v, k):
            return (kind[v] == CONSTRAINED and line[v] == k) or (kind[v] == ORIGINAL
                                                               and v in prim_v[k])
        for t in rest:
            tv = [s if w in (a, b) else w for w in tris[t]]
            ks = {line[w] for w in tv if kind[w] == CONSTRAINED}
            if any(all(on_edge(w, k) for w in tv) for k in ks):
                return False
        for P in cands:
            ok = True
            for t in rest:
                pts = [P if w in (a, b) else xy[w] for w in tris[t]]
                if orient(np.array(pts[0]), np.array(pts[1]), np.array(pts[2])) <= 0:
                    ok = False
                    break
            if not ok:
                continue
            for t in shared:
                alive_t[t] = False
                for w in tris[t]:
                    star[w].discard(t)
            for t in sorted(star[r]):
                tris[t] = [s if w == r else w for w in tris[t]]
                star[s].add(t)
            star[r] = set()
            xy[s] = P
            merged_into[r] = s
            return True
        return False

    n_contracted = 0
    while True:
        cand = set()
        for t, tv in enumerate(tris):
            if alive_t[t]:
                for i in range(3):
                    a, b = tv[i], tv[(i + 1) % 3]
                    cand.add((min(a, b), max(a, b)))
        order = sorted((_len(xy, a, b), a, b) for a, b in cand if _len(xy, a, b) < eps)
        done = 0
        for _, a, b in order:
            if not star[a] or not star[b] or not (star[a] & star[b]):
                continue  # no longer an edge
            if _len(xy, a, b) >= eps:
                continue
            if try_edge(a, b):
                done += 1
        n_contracted += done
        if done == 0:
            break

    alive_v = [v for v in range(nv) if star[v]]
    new_id = {v: i for i, v in enumerate(alive_v)}

    def root(v):
        while merged_into[v] != v:
            v = merged_into[v]
        return v

    old_to_new = np.array([new_id.get(root(v), -1) for v in range(nv)], dtype=np.int64)
    out_t = np.array([[new_id[w] for w in tris[t]] for t in range(len(tris)) if alive_t[t]],
                     dtype=np.int64).reshape(-1, 3)
    return (out_t, np.array([kind[v] for v in alive_v], dtype=np.int64),
            np.array([line[v] for v in alive_v], dtype=np.int64),
            np.array([xy[v] for v in alive_v], dtype=np.float64).reshape(-1, 2),
            old_to_new, n_contracted)
