"""Quadrature rules used by the oracle (the paper gives none; see the readings
recorded for the method: degree-2 product rules on well-separated elements,
degree-5 outer rules with closed-form inner integrals on touching elements).

All rules are returned in barycentric form (lam [n, k], w [n]) with weights
summing to 1; physical weights are w * measure.

Pins: exactness on monomials up to the stated degree (tests).
"""
import functools

import numpy as np


def tet_deg2():
    """4-point symmetric rule, exact to degree 2."""
    al = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
    be = (5.0 - np.sqrt(5.0)) / 20.0
    lam = np.full((4, 4), be)
    np.fill_diagonal(lam, al)
    return lam, np.full(4, 0.25)


def _s31(a):
    """Orbit of barycentric (a, a, a, 1 - 3a) under vertex permutations."""
    return [[1 - 3 * a if j == k else a for j in range(4)] for k in range(4)]


def _s22(b):
    """Orbit of barycentric (b, b, 1/2 - b, 1/2 - b) under vertex permutations."""
    c = 0.5 - b
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    return [[b if j in p else c for j in range(4)] for p in pairs]


def _tet14(params):
    a1, w1, a2, w2, b, w3 = params
    lam = np.array(_s31(a1) + _s31(a2) + _s22(b))
    w = np.array([w1] * 4 + [w2] * 4 + [w3] * 6)
    return lam, w


@functools.lru_cache(maxsize=1)
def _tet14_params():
    return tuple(_solve_tet14())


def tet_deg5():
    lam, w = _tet14(_tet14_params())
    return lam.copy(), w.copy()


def _solve_tet14():
    """Fully symmetric 14-point rule exact to degree 5: two S31 orbits and one
    S22 orbit, with the six orbit parameters fixed by the moment equations
    (solved here by least squares from a nearby start and checked to machine
    precision).  A symmetric rule keeps the discretisation invariant under
    vertex relabelling, so mirror symmetries of a mesh carry over exactly."""
    import itertools
    from math import factorial
    from scipy.optimize import least_squares

    exps = [e for e in itertools.product(range(6), repeat=4) if sum(e) <= 5]
    ref = np.array([6.0 * np.prod([factorial(x) for x in e]) / factorial(3 + sum(e)) for e in exps])
    E = np.array(exps)

    def resid(p):
        lam, w = _tet14(p)
        return (w[:, None] * np.prod(lam[:, None, :] ** E[None, :, :], axis=2)).sum(0) - ref

    p0 = [0.0927, 0.0735, 0.3109, 0.1127, 0.0455, 0.0425]
    sol = least_squares(resid, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15)
    if np.max(np.abs(resid(sol.x))) > 1e-14:
        raise RuntimeError("14-point rule did not converge")
    return sol.x


def tri_deg2():
    """3-point rule at barycentric (2/3, 1/6, 1/6) and permutations, degree 2."""
    lam = np.full((3, 3), 1.0 / 6.0)
    np.fill_diagonal(lam, 2.0 / 3.0)
    return lam, np.full(3, 1.0 / 3.0)


def tri_deg5():
    """Radon 7-point rule, exact to degree 5."""
    s15 = np.sqrt(15.0)
    b1 = (6.0 - s15) / 21.0
    b2 = (6.0 + s15) / 21.0
    w1 = (155.0 - s15) / 1200.0
    w2 = (155.0 + s15) / 1200.0
    lam = [[1 / 3, 1 / 3, 1 / 3]]
    w = [9.0 / 40.0]
    for b, wb in ((b1, w1), (b2, w2)):
        for k in range(3):
            l = [b, b, b]
            l[k] = 1.0 - 2.0 * b
            lam.append(l)
            w.append(wb)
    return np.array(lam), np.array(w)
