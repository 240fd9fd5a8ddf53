"""Pins for the oracle's quadrature weights (appendix "Integral and derivative approximations").

The paper prints no weight values, so the pins are textbook tables, two
independent derivations, polynomial exactness checked in exact arithmetic, and
closed invariants.
"""
import os
from fractions import Fraction as Fr

import pytest

from oracle import weights as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(x) for x in line.split()]
                rows.append((v[0], [Fr(x, v[1]) for x in v[2:]]))
    return rows


@pytest.mark.parametrize("k", range(1, 6))
def test_adams_moulton_two_derivations_agree(k):
    assert W.adams_moulton(k) == W.adams_moulton_by_moments(k)


def test_adams_moulton_matches_textbook_table():
    # golden file lists s-step AM from newest to oldest; ours b_0 (oldest) .. b_{k+1} (newest)
    for s, coeffs in _table("adams_moulton.txt"):
        if s < 2:
            continue
        k = s - 1
        assert list(W.adams_moulton(k))[::-1] == coeffs


def test_newton_cotes_textbook():
    for L, w in _table("newton_cotes.txt"):
        assert list(W.newton_cotes(L)) == w


def test_bdf_textbook():
    for k, a in _table("bdf.txt"):
        assert list(W.bdf_weights(k)) == a


@pytest.mark.parametrize("k", range(1, 6))
def test_gregory_sum_invariant(k):
    # unit function: the Riemann sum over L+1 points exceeds L by 1, shared by the two ends
    assert sum(o - 1 for o in W.gregory(k)) == Fr(-1, 2)


def test_gregory_first_order_is_partial_sum_of_am2():
    assert W.gregory(1) == (Fr(5, 12), Fr(13, 12))


EXPECTED_DEGREE = {1: 1, 2: 3, 3: 3, 4: 5, 5: 5}


@pytest.mark.parametrize("k", range(1, 6))
def test_interval_weights_polynomial_exactness(k):
    for L in range(1, 2 * k + 8):
        deg = W.exactness_degree(W.interval_weights(k, L))
        if L < k:
            assert deg == (L if L % 2 == 1 else L + 1)          # closed Newton-Cotes
        else:
            assert deg == EXPECTED_DEGREE[k]


@pytest.mark.parametrize("k", range(1, 6))
def test_interval_weights_special_cases(k):
    assert W.interval_weights(k, 0) == (Fr(0),)
    assert W.interval_weights(k, 1) == (Fr(1, 2), Fr(1, 2))             # trapezoid
    if k >= 2:
        assert W.interval_weights(k, 2) == (Fr(1, 3), Fr(4, 3), Fr(1, 3))  # Simpson
        assert W.interval_weights(k, 3) == tuple(Fr(x, 8) for x in (3, 9, 9, 3))
    if k >= 4:
        assert W.interval_weights(k, 4) == tuple(Fr(x, 45) for x in (14, 64, 24, 64, 14))
    if k == 1:
        assert W.interval_weights(1, 2) == (Fr(5, 12), Fr(14, 12), Fr(5, 12))


@pytest.mark.parametrize("k", range(1, 6))
def test_interval_weights_unit_inside(k):
    L = 3 * k + 4
    w = W.interval_weights(k, L)
    assert all(x == 1 for x in w[k + 1:L - k])
    assert w == w[::-1]
