"""Clebsch-Gordan coefficients (Condon-Shortley phase) from the Racah formula.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper groups the 2T+1 components of every pseudospin multiplet into one
reduced element by the Wigner-Eckart theorem (main text, Symmetry paragraph of
the GPU section; supplementary section S2.1, Eq. for the bond-space
decomposition).  The coupling coefficients themselves are the textbook ones;
this module evaluates Racah's closed formula in exact rational arithmetic and
takes a single square root at the end, so every value is correct to the last
bit of a double.

All angular momenta are passed doubled (``tj = 2j``, ``tm = 2m``) so that
half-integers stay integers.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, sqrt

import numpy as np


def _f(n2):
    """factorial of a doubled argument that must be even (i.e. an integer)."""
    assert n2 % 2 == 0 and n2 >= 0, n2
    return factorial(n2 // 2)


@lru_cache(maxsize=None)
def cg2(tj1, tm1, tj2, tm2, tJ, tM):
    """<j1 m1; j2 m2 | J M> with all arguments doubled.  Returns a float."""
    if tm1 + tm2 != tM:
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    if tJ > tj1 + tj2 or tJ < abs(tj1 - tj2) or (tj1 + tj2 + tJ) % 2:
        return 0.0
    pref = Fraction((tJ + 1) * _f(tJ + tj1 - tj2) * _f(tJ - tj1 + tj2) * _f(tj1 + tj2 - tJ),
                    _f(tj1 + tj2 + tJ + 2))
    pref *= (_f(tJ + tM) * _f(tJ - tM) * _f(tj1 - tm1) * _f(tj1 + tm1)
             * _f(tj2 - tm2) * _f(tj2 + tm2))
    s = Fraction(0)
    k = 0
    while True:
        args = [tj1 + tj2 - tJ - 2 * k, tj1 - tm1 - 2 * k, tj2 + tm2 - 2 * k,
                tJ - tj2 + tm1 + 2 * k, tJ - tj1 - tm2 + 2 * k]
        if args[0] < 0 or args[1] < 0 or args[2] < 0:
            break
        if args[3] >= 0 and args[4] >= 0:
            den = factorial(k)
            for a in args:
                den *= _f(a)
            s += Fraction((-1) ** k, den)
        k += 1
    if s == 0:
        return 0.0
    val2 = pref * s * s
    return (1.0 if s > 0 else -1.0) * sqrt(float(val2))


def mvals(tj):
    """Doubled magnetic quantum numbers of a multiplet, in DESCENDING order
    (m = j, j-1, ..., -j).  This is the component order used by every full
    (expanded) tensor in the oracle."""
    return list(range(tj, -tj - 1, -2))


@lru_cache(maxsize=None)
def cg_tensor(tj1, tj2, tJ):
    """Dense array C[m1, m2, M] = <j1 m1; j2 m2 | J M>, components in
    descending-m order along every axis."""
    out = np.zeros((tj1 + 1, tj2 + 1, tJ + 1))
    for i1, m1 in enumerate(mvals(tj1)):
        for i2, m2 in enumerate(mvals(tj2)):
            for iJ, M in enumerate(mvals(tJ)):
                out[i1, i2, iJ] = cg2(tj1, m1, tj2, m2, tJ, M)
    out.setflags(write=False)
    return out
