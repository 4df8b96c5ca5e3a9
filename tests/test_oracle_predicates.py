"""Pins for the checker's exact signs and its hit-distance formula.

Reference values come from Python's ``fractions.Fraction``: exact rational arithmetic on the same
binary64 inputs, an independent implementation from the checker's limb arithmetic. Inputs are
chosen to be hard: points rounded onto the ray line, exactly collinear and cocircular integer
points, nearly cocircular perturbations and direction components spanning 300 orders of magnitude.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle


def side_exact(o, d, v):
    D = F(d[0]) * (F(v[1]) - F(o[1])) - F(d[1]) * (F(v[0]) - F(o[0]))
    return (D > 0) - (D < 0)


def orient_exact(a, b, c):
    D = (F(b[0]) - F(a[0])) * (F(c[1]) - F(a[1])) - (F(b[1]) - F(a[1])) * (F(c[0]) - F(a[0]))
    return (D > 0) - (D < 0)


def incircle_exact(a, b, c, d):
    rows = []
    for p in (a, b, c):
        x, y = F(p[0]) - F(d[0]), F(p[1]) - F(d[1])
        rows.append((x, y, x * x + y * y))
    (a1, a2, a3), (b1, b2, b3), (c1, c2, c3) = rows
    D = a1 * (b2 * c3 - b3 * c2) - a2 * (b1 * c3 - b3 * c1) + a3 * (b1 * c2 - b2 * c1)
    return (D > 0) - (D < 0)


def _side_cases(rng, n):
    out = []
    for k in range(n):
        o = rng.uniform(-1000, 1000, 2)
        th = rng.uniform(0, 2 * np.pi)
        d = np.array([np.cos(th), np.sin(th)])
        mode = k % 5
        if mode == 0:  # a point rounded onto the ray line: the sign is decided by rounding
            v = o + rng.uniform(-50, 50) * d
        elif mode == 1:  # tiny and huge direction components
            d = np.array([10.0 ** rng.integers(-300, 3), -(10.0 ** rng.integers(-300, 3))])
            v = o + rng.uniform(-5, 5) * d + rng.normal(size=2) * 1e-12
        elif mode == 2:  # exact zero: integer data
            o = rng.integers(-100, 100, 2).astype(float)
            d = rng.integers(-9, 9, 2).astype(float)
            v = o + rng.integers(-5, 5) * d
        elif mode == 3:  # one ulp off the line
            v = o + rng.uniform(1, 10) * d
            v = np.nextafter(v, v + rng.choice([-1, 1], 2))
        else:
            v = rng.uniform(-1000, 1000, 2)
        out.append((o, d, v))
    return out


def test_side_sign_matches_rationals():
    rng = np.random.default_rng(1)
    cases = _side_cases(rng, 20000)
    zeros = 0
    for o, d, v in cases:
        e = side_exact(o, d, v)
        zeros += e == 0
        assert oracle.side_sign(o, d, v) == e, (o, d, v)
    assert zeros > 1000  # the integer cases really do hit D = 0


def test_orient_matches_rationals():
    rng = np.random.default_rng(2)
    for k in range(20000):
        a = rng.uniform(-1001, 1001, 2)
        b = rng.uniform(-1001, 1001, 2)
        if k % 3 == 0:
            c = a + rng.uniform(-3, 3) * (b - a)  # rounded onto the line ab
        elif k % 3 == 1:
            a, b = rng.integers(-50, 50, 2).astype(float), rng.integers(-50, 50, 2).astype(float)
            c = a + rng.integers(-4, 4) * (b - a)  # exactly collinear
        else:
            c = rng.uniform(-1001, 1001, 2)
        assert oracle.orient(a, b, c) == orient_exact(a, b, c)
    # the sign flips with operand order (a transposed operand would break this)
    a, b, c = np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0])
    assert oracle.orient(a, b, c) == 1 and oracle.orient(b, a, c) == -1


def test_incircle_matches_rationals():
    rng = np.random.default_rng(3)
    for k in range(6000):
        if k % 3 == 0:  # integer points on a common circle (Pythagorean radius 5)
            pts = [(3, 4), (-4, 3), (-5, 0), (0, -5), (4, -3), (5, 0), (-3, -4)]
            idx = rng.choice(len(pts), 4, replace=False)
            sh = rng.integers(-100, 100, 2)
            a, b, c, d = (np.array(pts[i], float) + sh for i in idx)
            if orient_exact(a, b, c) < 0:
                a, b = b, a
        elif k % 3 == 1:  # nearly cocircular
            cen = rng.uniform(-500, 500, 2)
            r = rng.uniform(0.01, 10)
            th = np.sort(rng.uniform(0, 2 * np.pi, 4))
            a, b, c, d = (cen + r * np.array([np.cos(t), np.sin(t)]) for t in th)
        else:
            a, b, c, d = (rng.uniform(-1000, 1000, 2) for _ in range(4))
            if orient_exact(a, b, c) < 0:
                a, b = b, a
        assert oracle.incircle(a, b, c, d) == incircle_exact(a, b, c, d), (a, b, c, d)
    # centre of the unit circle through three of its points is inside, a far point is outside
    a, b, c = np.array([1.0, 0.0]), np.array([0.0, 1.0]), np.array([-1.0, 0.0])
    assert oracle.incircle(a, b, c, np.array([0.0, 0.0])) == 1
    assert oracle.incircle(a, b, c, np.array([0.0, -1.0])) == 0
    assert oracle.incircle(a, b, c, np.array([3.0, 3.0])) == -1


def test_t_formula_is_the_crossing_parameter():
    """t within a few ulps of the exact rational crossing parameter of the primitive's line."""
    rng = np.random.default_rng(4)
    worst = 0.0
    for _ in range(5000):
        a, b = rng.uniform(0, 1000, 2), rng.uniform(0, 1000, 2)
        o = rng.uniform(0, 1000, 2)
        th = rng.uniform(0, 2 * np.pi)
        d = np.array([np.cos(th), np.sin(th)])
        ex, ey = F(b[0]) - F(a[0]), F(b[1]) - F(a[1])
        num = (F(a[0]) - F(o[0])) * ey - (F(a[1]) - F(o[1])) * ex
        den = F(d[0]) * ey - F(d[1]) * ex
        if den == 0:
            continue
        s = num / den
        t = oracle.t_formula(o, d, np.concatenate([a, b]))
        # conditioning of num and den: relative error <= ~4u * (|terms| / |value|)
        cn = (abs(float(F(a[0]) - F(o[0])) * float(ey)) + abs(float(F(a[1]) - F(o[1])) * float(ex))) / max(abs(float(num)), 1e-300)
        cd = (abs(float(d[0] * ey)) + abs(float(d[1] * ex))) / max(abs(float(den)), 1e-300)
        bound = 6 * 2.0 ** -53 * (cn + cd + 1)
        err = abs(F(t) - s) / abs(s) if s != 0 else abs(F(t))
        assert float(err) <= bound, (a, b, o, d)
        worst = max(worst, float(err) / bound)
    assert worst > 0  # the comparison is not vacuous


def test_t_formula_uses_no_fused_operations():
    """A case where a fused multiply-add in num gives a different last bit (order is fixed)."""
    o = np.array([0.1, 0.7])
    d = np.array([np.cos(1.1), np.sin(1.1)])
    seg = np.array([0.3, 0.2, 0.9, 1.3])
    ex, ey = seg[2] - seg[0], seg[3] - seg[1]
    num = (seg[0] - o[0]) * ey - (seg[1] - o[1]) * ex
    den = d[0] * ey - d[1] * ex
    assert oracle.t_formula(o, d, seg) == num / den  # numpy: plain binary64, unfused
