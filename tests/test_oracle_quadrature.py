"""Pins for the oracle's quadrature rules: exactness on monomials up to the
stated degree, against closed-form simplex moments
int_T l0^a l1^b l2^c l3^d dV / V = 3! a! b! c! d! / (3 + a + b + c + d)!."""
import itertools
from math import factorial

import numpy as np
import pytest

from oracle import quadrature as Q


def simplex_moment(exps, dim):
    num = factorial(dim) * np.prod([factorial(e) for e in exps])
    return num / factorial(dim + sum(exps))


@pytest.mark.parametrize("rule,deg,dim", [(Q.tet_deg2, 2, 3), (Q.tet_deg5, 5, 3),
                                          (Q.tri_deg2, 2, 2), (Q.tri_deg5, 5, 2)])
def test_exact_on_monomials(rule, deg, dim):
    lam, w = rule()
    assert abs(w.sum() - 1) < 1e-15
    assert np.all(w > 0)
    assert np.allclose(lam.sum(1), 1.0)
    for exps in itertools.product(range(deg + 1), repeat=dim + 1):
        if sum(exps) > deg:
            continue
        val = np.sum(w * np.prod(lam ** np.array(exps), axis=1))
        assert abs(val - simplex_moment(exps, dim)) < 1e-14, exps


@pytest.mark.parametrize("rule,deg,dim", [(Q.tet_deg2, 2, 3), (Q.tet_deg5, 5, 3),
                                          (Q.tri_deg5, 5, 2)])
def test_not_exact_beyond_degree(rule, deg, dim):
    # a plausible mistake (wrong constant) could still pass low degrees; the
    # first degree beyond must fail for at least one monomial
    lam, w = rule()
    errs = []
    for exps in itertools.product(range(deg + 2), repeat=dim + 1):
        if sum(exps) != deg + 1:
            continue
        val = np.sum(w * np.prod(lam ** np.array(exps), axis=1))
        errs.append(abs(val - simplex_moment(exps, dim)))
    assert max(errs) > 1e-8
