"""Annealing of a constrained triangulation by edge flips: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU leg may import this module. The
GPU library never does and shares no code with it.

What is computed (paper Sec. 3.2.7 for the move, Sec. 3.1 for the acceptance; the energy is the
total edge length, the weight the paper minimises):
- an unconstrained interior edge (b, c) between triangles (a, b, c) and (d, c, b) may flip to
  (a, d) when the quad a, b, d, c is strictly convex (both new triangles strictly
  counter-clockwise, decided exactly); the change of energy is |ad| - |bc|, each length
  sqrt(dx*dx + dy*dy) in binary64;
- a flip is accepted when it improves the weight (change < 0), or, at temperature T > 0, when
  u < exp(-change / T);
- rounds: in round r every candidate edge (unconstrained, interior; named by its slot 3t + i in
  the triangle t of lower id) draws a priority and a uniform u from SplitMix64 (Steele, Lea and
  Flood, 2014) at counters given by (r, slot), from state seed, and is tested against the
  triangulation as the round found it. Among the flips that would be accepted, one is chosen
  when its priority beats every other such flip that would touch one of the triangles its own
  flip touches (its two triangles and their outer neighbours): chosen flips are independent, so
  applying them one after another in any order gives the same triangulation, and a round
  without a chosen flip leaves none that would be accepted.

After a flip of (t, i) with neighbour u: t holds (a, b, d) and u holds (a, d, c), each listed from
a in that order; neighbours and constraint ids follow their edges.

With Steiner vertices on the original edges (line[v] = the original edge of such a vertex, -1 for
the others; prim_v[k] = the two ends of original edge k), a flip is also refused when one of its
new triangles has all three vertices on one original edge: zero area in intent, which the exact
test accepts only because rounding leaves the constrained vertex off its line, and which the
paper's strict convexity excludes.
"""
from __future__ import annotations

import math

import numpy as np

from . import orient

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(z: int) -> int:
    """The SplitMix64 output function applied to z (mod 2^64)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def draws(seed: int, rnd: int, slot: int) -> tuple[int, float]:
    """(priority, u) of a slot in a round: outputs k + 1 and k + 2 of the SplitMix64 sequence from
    state seed (output n mixes seed + n * golden), k = 2 * (rnd * 2^32 + slot);
    u = (second output >> 11) * 2^-53."""
    k = 2 * ((rnd << 32) + slot)
    base = seed & MASK
    p = splitmix64(base + (k + 1) * GOLDEN)
    x = splitmix64(base + (k + 2) * GOLDEN)
    return p, (x >> 11) * 2.0 ** -53


def _len(xy, p, q):
    dx = xy[q, 0] - xy[p, 0]
    dy = xy[q, 1] - xy[p, 1]
    return math.sqrt(dx * dx + dy * dy)


def _back(nbr, w, t):
    for j in range(3):
        if nbr[w, j] == t:
            return j
    raise AssertionError("asymmetric adjacency")


def candidates(tv, nbr, prim):
    """Slots 3t + i of unconstrained interior edges, in the triangle of lower id."""
    out = []
    for t in range(tv.shape[0]):
        for i in range(3):
            u = nbr[t, i]
            if u > t and prim[t, i] < 0:
                out.append(3 * t + i)
    return out


def touched(nbr, s):
    """Triangles a flip of slot s reads or writes: its two and their outer neighbours."""
    t, i = divmod(s, 3)
    u = int(nbr[t, i])
    out = {t, u}
    for w in (t, u):
        for j in range(3):
            x = int(nbr[w, j])
            if x >= 0:
                out.add(x)
    return out


def flat(tri, line, prim_v):
    """Whether the three vertices of tri lie on one original edge (see the module docstring)."""
    if line is None:
        return False
    for w in tri:
        k = line[w]
        if k >= 0 and all(line[x] == k or x in prim_v[k] for x in tri):
            return True
    return False


def test_flip(xy, tv, nbr, s, temperature, u, line=None, prim_v=None):
    """(accepted, change) of the flip of slot s against the current triangulation, not applied."""
    t, i = divmod(s, 3)
    ut = int(nbr[t, i])
    j = _back(nbr, ut, t)
    a, b, c = tv[t, i], tv[t, (i + 1) % 3], tv[t, (i + 2) % 3]
    d = tv[ut, j]
    if orient(xy[a], xy[b], xy[d]) <= 0 or orient(xy[a], xy[d], xy[c]) <= 0:
        return False, 0.0
    if flat((a, b, d), line, prim_v) or flat((a, d, c), line, prim_v):
        return False, 0.0
    change = _len(xy, a, d) - _len(xy, b, c)
    return change < 0.0 or (temperature > 0.0 and u < math.exp(-change / temperature)), change


def chosen(tv, nbr, prim, seed, rnd, xy=None, temperature=None, line=None, prim_v=None):
    """The round's independent flips: candidates (with xy and temperature given: those whose flip
    would be accepted) whose (priority, slot) beats every other such candidate whose touched
    triangles meet theirs."""
    cand = candidates(tv, nbr, prim)
    if xy is not None:
        cand = [s for s in cand
                if test_flip(xy, tv, nbr, s, temperature, draws(seed, rnd, s)[1], line,
                             prim_v)[0]]
    pr = {s: draws(seed, rnd, s)[0] for s in cand}
    tri_of = {}
    for s in cand:
        for x in touched(nbr, s):
            tri_of.setdefault(x, []).append(s)
    out = []
    for s in cand:
        win = True
        for x in touched(nbr, s):
            for s2 in tri_of[x]:
                if s2 != s and (pr[s2], s2) > (pr[s], s):
                    win = False
                    break
            if not win:
                break
        if win:
            out.append(s)
    return out


def try_flip(xy, tv, nbr, prim, s, temperature, u, line=None, prim_v=None):
    """Test and (if accepted) apply the flip of slot s. Returns (accepted, change of weight)."""
    ok, change = test_flip(xy, tv, nbr, s, temperature, u, line, prim_v)
    if not ok:
        return False, change
    t, i = divmod(s, 3)
    ut = int(nbr[t, i])
    j = _back(nbr, ut, t)
    a, b, c = tv[t, i], tv[t, (i + 1) % 3], tv[t, (i + 2) % 3]
    d = tv[ut, j]
    nt1, pt1 = nbr[t, (i + 1) % 3], prim[t, (i + 1) % 3]  # edge (c, a)
    nt2, pt2 = nbr[t, (i + 2) % 3], prim[t, (i + 2) % 3]  # edge (a, b)
    nu1, pu1 = nbr[ut, (j + 1) % 3], prim[ut, (j + 1) % 3]  # edge (b, d)
    nu2, pu2 = nbr[ut, (j + 2) % 3], prim[ut, (j + 2) % 3]  # edge (d, c)
    tv[t] = (a, b, d)
    nbr[t] = (nu1, ut, nt2)
    prim[t] = (pu1, -1, pt2)
    tv[ut] = (a, d, c)
    nbr[ut] = (nu2, nt1, t)
    prim[ut] = (pu2, pt1, -1)
    if nu1 >= 0:
        nbr[nu1, _back(nbr, nu1, ut)] = t
    if nt1 >= 0:
        nbr[nt1, _back(nbr, nt1, t)] = ut
    return True, change


def anneal(xy, tri_v, tri_nbr, tri_prim, temperatures, seed, line=None, prim_v=None):
    """Rounds of flips at the given temperatures, applied one after another. Returns the new
    (tri_v, tri_nbr, tri_prim) and the accepted flips of each round."""
    if line is not None:
        line = [int(k) for k in line]
        prim_v = [tuple(map(int, p)) for p in np.asarray(prim_v).reshape(-1, 2)]
    xy = np.asarray(xy, dtype=np.float64)
    tv = np.array(tri_v, dtype=np.int64).reshape(-1, 3)
    nbr = np.array(tri_nbr, dtype=np.int64).reshape(-1, 3)
    prim = np.array(tri_prim, dtype=np.int64).reshape(-1, 3)
    counts = []
    for r, temp in enumerate(temperatures):
        n = 0
        for s in chosen(tv, nbr, prim, seed, r, xy, float(temp), line, prim_v):
            ok, _ = try_flip(xy, tv, nbr, prim, s, float(temp), draws(seed, r, s)[1], line, prim_v)
            assert ok
            n += 1
        counts.append(n)
    return tv, nbr, prim, counts


def weight(xy, tri_v, tri_nbr):
    """Total edge length, each edge once."""
    xy = np.asarray(xy, dtype=np.float64)
    s = 0.0
    for t in range(tri_v.shape[0]):
        for i in range(3):
            u = tri_nbr[t, i]
            if u < 0 or u > t:
                s += _len(xy, tri_v[t, (i + 1) % 3], tri_v[t, (i + 2) % 3])
    return s
