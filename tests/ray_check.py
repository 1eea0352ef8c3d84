"""Rays certifying dual infeasibility (an improving direction of the LP),
checked from their definition in exact rational arithmetic on the returned
floats, and the unbounded toy LPs the tests use."""
from fractions import Fraction

import numpy as np

from paper_2512_06715_amd import ucgen

INF = np.inf


def ray_violation(lp, d):
    """(c'd, largest violation) of d as an improving ray of lp: (A d)_i = 0
    on = rows and >= 0 on >= rows, d_j = 0 where l_j and u_j are finite,
    >= 0 where only l_j is, <= 0 where only u_j is.  Exact arithmetic on the
    float values of d and of the LP, independent of any solver's sums."""
    dd = [Fraction(float(v)) for v in d]
    cd = sum((Fraction(float(lp.c[j])) * dd[j] for j in range(lp.n)), Fraction(0))
    worst = Fraction(0)
    for i in range(lp.m):
        s = sum((Fraction(float(lp.val[k])) * dd[int(lp.col_idx[k])]
                 for k in range(int(lp.row_ptr[i]), int(lp.row_ptr[i + 1]))), Fraction(0))
        worst = max(worst, abs(s) if lp.row_kind[i] == 0 else max(Fraction(0), -s))
    for j in range(lp.n):
        fl, fu = bool(np.isfinite(lp.l[j])), bool(np.isfinite(lp.u[j]))
        if fl and fu:
            v = abs(dd[j])
        elif fl:
            v = max(Fraction(0), -dd[j])
        elif fu:
            v = max(Fraction(0), dd[j])
        else:
            v = Fraction(0)
        worst = max(worst, v)
    return cd, worst


def is_ray(lp, d, eps=1e-8):
    cd, worst = ray_violation(lp, d)
    return cd < 0 and worst <= Fraction(eps) * -cd


def unbounded_toys():
    """Four LPs with a closed-form cone of improving rays:
    - min -x1, x1 - x2 = 0, x >= 0: rays t (1, 1);
    - min x, x free, one empty row: rays t (-1);
    - min -x2, x1 - x2 >= 0, x1 >= 0, x2 free: d1 >= d2 > 0;
    - min x1 - 2 x2, x1 + x2 >= 1, x >= 0: d >= 0 with d1 < 2 d2."""
    return [
        ucgen.dense_to_lp(np.array([[1.0, -1.0]]), np.array([0], np.uint8), np.array([0.0]),
                          np.array([-1.0, 0.0]), np.array([0.0, 0.0]), np.array([INF, INF])),
        ucgen.dense_to_lp(np.zeros((1, 1)), np.array([0], np.uint8), np.array([0.0]),
                          np.array([1.0]), np.array([-INF]), np.array([INF])),
        ucgen.dense_to_lp(np.array([[1.0, -1.0]]), np.array([1], np.uint8), np.array([0.0]),
                          np.array([0.0, -1.0]), np.array([0.0, -INF]), np.array([INF, INF])),
        ucgen.dense_to_lp(np.array([[1.0, 1.0]]), np.array([1], np.uint8), np.array([1.0]),
                          np.array([1.0, -2.0]), np.array([0.0, 0.0]), np.array([INF, INF])),
    ]


def random_unbounded_toys(count, seed=7):
    """The first `count` random toys that HiGHS calls unbounded."""
    from oracle import exact
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        m, n = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        lp = ucgen.dense_to_lp(*ucgen.random_toy_lp(rng, m, n))
        if exact.highs(lp)[0] == exact.UNBOUNDED:
            out.append(lp)
    return out
