"""Subdivision of a triangulation (paper Sec. 3.5.2): TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU leg may import this module. The
library never does and shares no code with it.

Every triangle is split into four by the midpoints of its three edges (the paper's figure of the
subdivision). Readings of what the paper leaves open:
- a midpoint is ((xa + xb) * 0.5, (ya + yb) * 0.5) in binary64;
- it is CONSTRAINED to an original edge when both ends of its edge lie on that edge (a vertex
  CONSTRAINED to it, or one of its two ORIGINAL ends), else FREE;
- numbering: old vertices keep their ids; the midpoint of the e-th edge in increasing
  (lower id, higher id) order gets id V + e; triangle t = (v0, v1, v2), whose edge i lies opposite
  v_i with midpoint m_i, gives triangles t, T + t, 2T + t, 3T + t = (v0, m2, m1), (v1, m0, m2),
  (v2, m1, m0), (m0, m1, m2).
"""
from __future__ import annotations

import numpy as np

from . import orient

ORIGINAL, CONSTRAINED, FREE = 0, 1, 2


class Subdivided:
    """The subdivided mesh: positions, triangles, kinds, lines (-1 unless CONSTRAINED) and the
    original edges (unchanged)."""

    def __init__(self, xy, tri_v, kind, line, prim_v, name=""):
        self.xy, self.tri_v, self.kind, self.line, self.prim_v = xy, tri_v, kind, line, prim_v
        self.name = name

    @property
    def n_vertices(self):
        return int(self.xy.shape[0])

    @property
    def n_triangles(self):
        return int(self.tri_v.shape[0])


def _on_line(kind, line, prim_v, v, L):
    """Whether vertices v lie on original edges L (arrays; L >= 0)."""
    Ls = np.maximum(L, 0)
    return (((kind[v] == CONSTRAINED) & (line[v] == L)) |
            ((kind[v] == ORIGINAL) & ((prim_v[Ls, 0] == v) | (prim_v[Ls, 1] == v))))


def _ccw(P, tri):
    """Strict counter-clockwise orientation of every triangle: a binary64 filter whose bound
    (3 + 16u) u of |l| + |r| is below 2^-51, then exact orientation where it cannot decide."""
    a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
    l = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1])
    r = (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    det, mag = l - r, np.abs(l) + np.abs(r)
    sure = (np.abs(det) > 2.0 ** -51 * mag) & (mag > 2.0 ** -900)
    ok = sure & (det > 0)
    for k in np.nonzero(~sure)[0]:
        ok[k] = orient(a[k], b[k], c[k]) > 0
    return ok


def subdivide(xy, tri_v, kind, line, prim_v, name="") -> Subdivided:
    """Split every triangle into four (see the module notes). Raises ValueError if a sub-triangle
    is not strictly counter-clockwise (exact orientation)."""
    xy = np.asarray(xy, dtype=np.float64)
    tv = np.asarray(tri_v, dtype=np.int64).reshape(-1, 3)
    kind = np.asarray(kind, dtype=np.int64)
    line = np.asarray(line, dtype=np.int64)
    prim_v = np.asarray(prim_v, dtype=np.int64).reshape(-1, 2)
    V, T = kind.shape[0], tv.shape[0]
    # edge i of a triangle joins v[i+1] and v[i+2]; edges numbered by (lower, higher) end
    ea, eb = tv[:, [1, 2, 0]], tv[:, [2, 0, 1]]
    key = np.minimum(ea, eb) * V + np.maximum(ea, eb)
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    m = V + inv.reshape(T, 3)  # m[:, i]: the midpoint of edge i
    a, b = uniq // V, uniq % V
    mid = np.stack([(xy[a, 0] + xy[b, 0]) * 0.5, (xy[a, 1] + xy[b, 1]) * 0.5], axis=1)
    # the original edge holding both ends, if any
    L = np.full(uniq.shape[0], -1, dtype=np.int64)
    ca, cb = kind[a] == CONSTRAINED, kind[b] == CONSTRAINED
    L[ca] = line[a[ca]]
    L[~ca & cb] = line[b[~ca & cb]]
    oo = (kind[a] == ORIGINAL) & (kind[b] == ORIGINAL)
    if prim_v.shape[0] and oo.any():
        pk = np.minimum(prim_v[:, 0], prim_v[:, 1]) * V + np.maximum(prim_v[:, 0], prim_v[:, 1])
        order = np.argsort(pk, kind="stable")
        pos = np.clip(np.searchsorted(pk[order], uniq[oo]), 0, pk.shape[0] - 1)
        L[oo] = np.where(pk[order][pos] == uniq[oo], order[pos], -1)
    cons = (L >= 0) & _on_line(kind, line, prim_v, a, L) & _on_line(kind, line, prim_v, b, L) \
        if prim_v.shape[0] else np.zeros(uniq.shape[0], dtype=bool)
    out = np.concatenate([np.stack([tv[:, 0], m[:, 2], m[:, 1]], 1),
                          np.stack([tv[:, 1], m[:, 0], m[:, 2]], 1),
                          np.stack([tv[:, 2], m[:, 1], m[:, 0]], 1),
                          np.stack([m[:, 0], m[:, 1], m[:, 2]], 1)]).astype(np.int32)
    P = np.ascontiguousarray(np.concatenate([xy, mid]))
    if not _ccw(P, out).all():
        raise ValueError("a sub-triangle is not strictly counter-clockwise")
    kinds = np.concatenate([kind, np.where(cons, CONSTRAINED, FREE)]).astype(np.int32)
    lines = np.concatenate([line, np.where(cons, L, -1)]).astype(np.int32)
    return Subdivided(P, out, kinds, lines, prim_v.astype(np.int32), name)
