"""Pins of the oracle's rounding reading R16 (every product of a stencil sum and
both steps of the line elimination is one fused multiply-add): the oracle's
results are recomputed here in exact rational arithmetic, rounding once per
fused multiply-add (Fraction -> float rounds to nearest, ties to even), and
must agree bit for bit; the same computation with the product rounded on its
own must differ somewhere, so the pins can tell the two readings apart."""
import math
from fractions import Fraction

import numpy as np

from oracle import oracle as O


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mul_add(a, b, c):   # the product rounded on its own, then the sum
    return float(Fraction(a * b) + Fraction(c))


def at(x, j, i):
    n = x.shape[0]
    return float(x[j, i]) if 0 <= j < n and 0 <= i < n else 0.0


def stencil_sums(s, x, madd):
    n = x.shape[0]
    y = np.zeros_like(x)
    for j in range(n):
        for i in range(n):
            acc = 0.0
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    acc = madd(float(s[b + 1, a + 1]), at(x, j + b, i + a), acc)
            y[j, i] = acc
    return y


def test_stencil_sums_are_fused():
    rng = np.random.default_rng(16)
    s = rng.uniform(-1, 1, (3, 3))
    x = rng.uniform(-1, 1, (9, 9))
    got = O.apply_stencil(s, x)
    assert np.array_equal(got, stencil_sums(s, x, fma))
    assert not np.array_equal(got, stencil_sums(s, x, mul_add))


def zebra_reference(H, v, f, direction, madd):
    """One zebra relaxation of the fine level, lines of even index first, each
    solved with its neighbours' current values: d_q = f - (the six off-line
    products accumulated) h^-2, forward (d_q - lo y_{q-1}) r_q, backward
    y_q - u_q x_{q+1}; the (r, u) tables are the oracle's own (setup data)."""
    n = v.shape[0]
    hi = float((n + 1) ** 2)
    s = H.stencils[0]
    r, u = H.zebra_tables(1, direction)
    lo = float(s[1, 0] if direction == 0 else s[0, 1]) * hi
    v = v.copy()
    for colour in (0, 1):
        for line in range(colour, n, 2):
            def pos(q):
                return (line, q) if direction == 0 else (q, line)
            prev = 0.0
            for q in range(n):
                j, i = pos(q)
                acc = 0.0
                if direction == 0:
                    for b in (-1, 1):
                        for a in (-1, 0, 1):
                            acc = madd(float(s[b + 1, a + 1]), at(v, j + b, i + a), acc)
                else:
                    for a in (-1, 1):
                        for b in (-1, 0, 1):
                            acc = madd(float(s[b + 1, a + 1]), at(v, j + b, i + a), acc)
                d = float(f[j, i]) - acc * hi
                y = d * r[0] if q == 0 else madd(-lo, prev, d) * r[q]
                v[j, i] = y
                prev = y
            for q in range(n - 2, -1, -1):
                j, i = pos(q)
                jn, i_n = pos(q + 1)
                v[j, i] = madd(-u[q], float(v[jn, i_n]), float(v[j, i]))
    return v


def test_line_elimination_is_fused():
    n = 7
    H = O.Hierarchy(n, math.pi / 5, 2e-3, smoother="zebra")
    rng = np.random.default_rng(17)
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n)) * 50
    for direction in (0, 1):
        got = H.zebra_relax(v0, f, direction)
        assert np.array_equal(got, zebra_reference(H, v0, f, direction, fma)), direction
        assert not np.array_equal(got, zebra_reference(H, v0, f, direction, mul_add)), direction
