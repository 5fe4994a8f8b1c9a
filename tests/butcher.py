"""Rooted trees and elementary weights for the Runge-Kutta order conditions
(Butcher; Hairer, Norsett & Wanner, "Solving ODEs I", Sec. II.2): a method
(A, b) has order p when sum_i b_i Phi_i(t) = 1/gamma(t) for every rooted tree
t with at most p vertices.  Test helpers only; they share nothing with the
integrators they check."""
from fractions import Fraction

import numpy as np

_memo = {}


def trees(n):
    """Rooted trees with n vertices, each a sorted tuple of child trees."""
    if n in _memo:
        return _memo[n]
    if n == 1:
        _memo[1] = [()]
        return _memo[1]
    out = set()

    def forests(m, smallest):
        if m == 0:
            yield ()
            return
        for k in range(1, m + 1):
            for t in trees(k):
                key = (k, t)
                if smallest is not None and key < smallest:
                    continue
                for rest in forests(m - k, key):
                    yield (t,) + rest

    for f in forests(n - 1, None):
        out.add(tuple(sorted(f)))
    _memo[n] = sorted(out)
    return _memo[n]


def order(t):
    return 1 + sum(order(x) for x in t)


def gamma(t):
    g = order(t)
    for x in t:
        g *= gamma(x)
    return g


def phi(t, A):
    """Stage vector of the elementary weight of tree t (floating point)."""
    v = np.ones(A.shape[0])
    for ch in t:
        v = v * (A @ phi(ch, A))
    return v


def defects(w, A, p, theta=1.0):
    """max |sum_i w_i Phi_i(t) - theta^rho / gamma(t)| over trees of order <= p."""
    return max(abs(w @ phi(t, A) - theta ** order(t) / gamma(t))
               for n in range(1, p + 1) for t in trees(n))


def exact_failures(w, A, p):
    """Orders n <= p at which some tree's condition fails, in exact rational
    arithmetic (w, A lists of Fractions)."""
    s = len(w)
    memo = {}

    def ph(t):
        if t not in memo:
            v = [Fraction(1)] * s
            for ch in t:
                u = ph(ch)
                v = [v[i] * sum((A[i][j] * u[j] for j in range(s)), Fraction(0))
                     for i in range(s)]
            memo[t] = v
        return memo[t]

    bad = set()
    for n in range(1, p + 1):
        for t in trees(n):
            if sum((w[i] * ph(t)[i] for i in range(s)), Fraction(0)) != Fraction(1, gamma(t)):
                bad.add(n)
    return sorted(bad)
