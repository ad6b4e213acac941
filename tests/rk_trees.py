"""Rooted trees and Runge--Kutta order conditions (Butcher theory).

A method (A, b) has order p iff for every rooted tree t with |t| <= p the
elementary weight b . Phi(t) equals 1 / gamma(t).  Trees are nested tuples of
their subtrees; the counts 1, 1, 2, 4, 9, 20, 48, 115 for orders 1..8 are
checked by the tests.
"""
from functools import lru_cache

import mpmath as mp


@lru_cache(maxsize=None)
def trees(n):
    if n == 1:
        return ((),)
    out = set()

    def parts(rem, maxsize, maxtree):
        if rem == 0:
            yield ()
            return
        for sz in range(min(rem, maxsize), 0, -1):
            for t in trees(sz):
                if sz == maxsize and maxtree is not None and t > maxtree:
                    continue
                for rest in parts(rem - sz, sz, t):
                    yield (t,) + rest

    for p in parts(n - 1, n - 1, None):
        out.add(tuple(sorted(p, reverse=True)))
    return tuple(sorted(out))


def order(t):
    return 1 + sum(order(c) for c in t)


def gamma(t):
    g = order(t)
    for c in t:
        g *= gamma(c)
    return g


def phi(t, A):
    """Internal elementary weights: vector over stages."""
    s = len(A)
    v = [mp.mpf(1)] * s
    for c in t:
        gc = phi(c, A)
        Ag = [mp.fsum(A[i][j] * gc[j] for j in range(s)) for i in range(s)]
        v = [v[i] * Ag[i] for i in range(s)]
    return v


def residuals(A, b, p, scale=lambda t: mp.mpf(1)):
    """Max |b.Phi(t) - scale(t)/gamma(t)| over all trees of order <= p."""
    worst = mp.mpf(0)
    for n in range(1, p + 1):
        for t in trees(n):
            g = phi(t, A)
            val = mp.fsum(b[i] * g[i] for i in range(len(b)))
            worst = max(worst, abs(val - scale(t) / gamma(t)))
    return worst


def residual_at(A, b, p):
    """Max residual over the trees of exactly order p."""
    worst = mp.mpf(0)
    for t in trees(p):
        g = phi(t, A)
        val = mp.fsum(b[i] * g[i] for i in range(len(b)))
        worst = max(worst, abs(val - mp.mpf(1) / gamma(t)))
    return worst
