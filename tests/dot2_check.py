"""Inputs and the pass criterion of the compensated dot-product test.

The spectral multiply's compensated form evaluates each three-term dot
product with Dot2 (Ogita, Rump and Oishi, "Accurate sum and dot product",
SIAM J. Sci. Comput. 26 (2005)), whose result res satisfies
|res - s| <= u |s| + gamma_n^2 sum |k_i x_i| for the exact value s of the same
float inputs (u = 2^-24 for binary32, gamma_n = n u / (1 - n u), n = 3 here).
`against_bound` measures results against that bound with exact rational arithmetic.
"""
from fractions import Fraction

import numpy as np

U = 2.0 ** -24
G3 = 3 * U / (1 - 3 * U)


def cancelling_triples(n, seed):
    """n float32 triples (k0, x0, k1, x1, k2, x2), one per row, whose dot
    product cancels: x2 undoes k0 x0 + k1 x1 up to a relative 1e-7 ... 1e-2,
    i.e. condition numbers from about 1e2 to beyond 1/u."""
    rng = np.random.default_rng(seed)

    def sgn(size):
        return rng.choice([-1.0, 1.0], size)

    k = (rng.uniform(0.1, 10.0, (n, 3)) * sgn((n, 3))).astype(np.float32)
    x = (rng.uniform(0.1, 10.0, (n, 3)) * sgn((n, 3))).astype(np.float32)
    delta = 10.0 ** rng.uniform(-7, -2, n) * sgn(n)
    part = k[:, 0].astype(np.float64) * x[:, 0] + k[:, 1].astype(np.float64) * x[:, 1]
    x[:, 2] = (-part / k[:, 2] * (1.0 + delta)).astype(np.float32)
    return np.stack([k[:, 0], x[:, 0], k[:, 1], x[:, 1], k[:, 2], x[:, 2]], axis=1)


def against_bound(trip, comp, plain):
    """Largest ratio of the compensated results' error to Dot2's bound, and,
    over the triples whose exact value is not zero, the condition numbers
    sum |k_i x_i| / |s| and the plain results' relative errors."""
    worst, conds, plain_rel = 0.0, [], []
    for i in range(len(trip)):
        a = [Fraction(float(v)) for v in trip[i]]
        s = a[0] * a[1] + a[2] * a[3] + a[4] * a[5]
        absum = abs(a[0] * a[1]) + abs(a[2] * a[3]) + abs(a[4] * a[5])
        err = abs(Fraction(float(comp[i])) - s)
        bound = U * abs(s) + G3 * G3 * absum
        worst = max(worst, float(err / bound) if bound else float(err > 0))
        if s != 0:
            conds.append(float(absum / abs(s)))
            plain_rel.append(float(abs(Fraction(float(plain[i])) - s) / abs(s)))
    return worst, np.array(conds), np.array(plain_rel)
