"""Pins for the oracle's quadrature (Sec. 2.3, Eq. 10): exactness on
polynomials, checked against the closed form of the monomial integrals over
a triangle, and the Gauss-Legendre nodes against numpy's table."""
import itertools
import math

import numpy as np
import pytest


def exact_bary_monomial(a, b, c):
    # int_T l0^a l1^b l2^c dA / area  =  2 a! b! c! / (a+b+c+2)!
    return 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


def rule_error(bary, w, deg):
    worst = 0.0
    for a, b in itertools.product(range(deg + 1), repeat=2):
        c = deg - a - b
        if c < 0:
            continue
        q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
        worst = max(worst, abs(q - exact_bary_monomial(a, b, c)))
    return worst


def test_gauss_legendre_matches_numpy(orc):
    for n in (1, 2, 5, 8, 16, 32):
        x, w = orc.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 1e-15
        assert np.max(np.abs(w - wr)) < 2e-15


def test_far_rule_degree_three(orc):
    b, w = orc.far_rule()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(b.sum(axis=1), 1.0, atol=1e-15)
    for deg in range(4):
        assert rule_error(b, w, deg) < 1e-15, deg
    assert rule_error(b, w, 4) > 1e-4  # degree 3 exactly, not 4


def test_near_rule_degree_eight(orc):
    b, w = orc.near_rule(5)
    assert b.shape == (25, 3)
    assert abs(w.sum() - 1.0) < 1e-14
    assert (w > 0).all()
    assert (b >= 0).all() and np.allclose(b.sum(axis=1), 1.0, atol=1e-15)
    for deg in range(9):
        assert rule_error(b, w, deg) < 1e-15, deg
    assert rule_error(b, w, 9) > 1e-10


@pytest.mark.parametrize("n1d", [2, 3, 7])
def test_near_rule_other_orders(orc, n1d):
    b, w = orc.near_rule(n1d)
    for deg in range(2 * n1d - 1):
        assert rule_error(b, w, deg) < 1e-14, deg
