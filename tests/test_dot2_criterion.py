"""The compensated dot-product test can tell Dot2 from a broken Dot2.

Host-only: binary32 emulations (numpy float32 arithmetic; fma as the exact
product plus the addend, rounded once) of Dot2 as written, of Dot2 with the
first product's fma contracted into the two-sum that follows (the compiler
mistake that FP contraction can make), and of the plain fma chain, judged by
the criterion of the GPU test: the correct form stays within Dot2's bound,
the contracted one does not, and the plain form's errors grow with the
condition number.
"""
from fractions import Fraction

import numpy as np

from tests.dot2_check import U, cancelling_triples, against_bound

f = np.float32


def fma(a, b, c):
    return f(float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))))


def two_sum(a, b):
    s = f(a + b)
    bb = f(s - a)
    return s, f(f(a - f(s - bb)) + f(b - bb))


def dot2(k0, x0, k1, x1, k2, x2, contract=False):
    p = f(k0 * x0)
    s = fma(k0, x0, -p)
    h = f(k1 * x1)
    r = fma(k1, x1, -h)
    if contract:  # q = k0 x0 + h with the unrounded product, then the two-sum's error term
        q = fma(k0, x0, h)
        bb = f(q - p)
        e = f(f(p - f(q - bb)) + f(h - bb))
    else:
        q, e = two_sum(p, h)
    s = f(s + f(r + e))
    p = q
    h = f(k2 * x2)
    r = fma(k2, x2, -h)
    q, e = two_sum(p, h)
    s = f(s + f(r + e))
    return f(q + s)


def plain(k0, x0, k1, x1, k2, x2):
    return fma(k0, x0, fma(k1, x1, f(k2 * x2)))


def test_criterion_separates_dot2_from_contracted_dot2():
    trip = cancelling_triples(512, 3)
    good = np.array([dot2(*t) for t in trip])
    bad = np.array([dot2(*t, contract=True) for t in trip])
    pl = np.array([plain(*t) for t in trip])
    worst_good, conds, plain_rel = against_bound(trip, good, pl)
    worst_bad, _, _ = against_bound(trip, bad, pl)
    hi = conds > 1e4
    assert worst_good <= 1.0
    assert worst_bad > 100.0
    assert hi.sum() > len(trip) // 4 and np.median(plain_rel[hi]) > 30 * U
