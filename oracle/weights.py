"""Exact-rational quadrature weights (appendix "Integral and derivative approximations").

Everything here is computed in `fractions.Fraction`, then rounded once to float64
where a float table is asked for.

Readings of the paper taken here (it is garbled or silent at these points):
  * The Gregory end weights are the partial sums omega_i = sum_{j=0..i} b_{k+1-j},
    i = 0..k, of the (k+1)-step Adams-Moulton coefficients b_0..b_{k+1}
    (b_{k+1} multiplies the newest point).  The printed sum has a summand that
    does not depend on j; the appendix also says the correction touches k+1
    points at each end, which needs k+2 coefficients, i.e. the (k+1)-step rule.
  * Interval weights for an interval of L steps: for L >= k the two end
    corrections are added to the unit Riemann weights, overlapping when L <= 2k;
    for 1 <= L < k the closed Newton-Cotes rule on the L+1 points of the interval
    (the polynomial integration weights of degree L); L = 0 is the empty interval.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from functools import lru_cache


def _solve_exact(a, b):
    """Solve a x = b exactly (Gauss-Jordan over Fractions).  a: list of rows."""
    n = len(a)
    m = [list(map(Fr, row)) + [Fr(v)] for row, v in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        pv = m[col][col]
        m[col] = [v / pv for v in m[col]]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col]
                m[r] = [vr - f * vc for vr, vc in zip(m[r], m[col])]
    return [m[r][n] for r in range(n)]


@lru_cache(maxsize=None)
def interpolation_matrix(deg: int):
    """P = M^{-1} with M_{ja} = j^a, 0 <= j, a <= deg (polynomial interpolant coefficients)."""
    n = deg + 1
    cols = []
    for l in range(n):                      # column l of M^{-1} solves M x = e_l
        e = [Fr(int(i == l)) for i in range(n)]
        cols.append(_solve_exact([[Fr(j) ** a for a in range(n)] for j in range(n)], e))
    # P[a][l] = cols[l][a]
    return tuple(tuple(cols[l][a] for l in range(n)) for a in range(n))


def poly_integration_weights(deg: int, m, n):
    """I_{m n l} = sum_a P_{al} (n^{a+1} - m^{a+1}) / (a+1), l = 0..deg."""
    P = interpolation_matrix(deg)
    m, n = Fr(m), Fr(n)
    return tuple(sum(P[a][l] * (n ** (a + 1) - m ** (a + 1)) / (a + 1) for a in range(deg + 1))
                 for l in range(deg + 1))


def poly_differentiation_weights(deg: int, m):
    """D_{m l} = sum_{a>=1} P_{al} a m^{a-1}, l = 0..deg."""
    P = interpolation_matrix(deg)
    m = Fr(m)
    return tuple(sum(P[a][l] * a * m ** (a - 1) for a in range(1, deg + 1))
                 for l in range(deg + 1))


def bdf_weights(k: int):
    """Backward-differentiation weights a_j = -D_{0j}, j = 0..k."""
    return tuple(-d for d in poly_differentiation_weights(k, 0))


def adams_moulton(k: int):
    """(k+1)-step Adams-Moulton coefficients b_0..b_{k+1}: I_{k,k+1,l} at degree k+1."""
    return poly_integration_weights(k + 1, k, k + 1)


def adams_moulton_by_moments(k: int):
    """Same coefficients from the moment conditions sum_l b_l l^d = int_k^{k+1} t^d dt."""
    n = k + 2
    a = [[Fr(l) ** d for l in range(n)] for d in range(n)]
    b = [(Fr(k + 1) ** (d + 1) - Fr(k) ** (d + 1)) / (d + 1) for d in range(n)]
    return tuple(_solve_exact(a, b))


@lru_cache(maxsize=None)
def gregory(k: int):
    """Gregory end weights omega_0..omega_k (partial sums of the AM coefficients)."""
    if not 1 <= k <= 5:
        raise ValueError("Gregory order k must be in 1..5")
    b = adams_moulton(k)
    return tuple(sum(b[k + 1 - j] for j in range(i + 1)) for i in range(k + 1))


def newton_cotes(L: int):
    """Closed Newton-Cotes weights on L+1 points (degree-L polynomial integration)."""
    return poly_integration_weights(L, 0, L)


@lru_cache(maxsize=None)
def interval_weights(k: int, L: int):
    """Weights w^{(L)}_i, i = 0..L, for int over an interval of L steps (h factored out)."""
    if L < 0:
        raise ValueError("negative interval")
    if L == 0:
        return (Fr(0),)
    if L < k:
        return newton_cotes(L)
    om = gregory(k)
    w = [Fr(1)] * (L + 1)
    for i in range(k + 1):
        w[i] += om[i] - 1
        w[L - i] += om[i] - 1
    return tuple(w)


def interval_weights_f64(k: int, L: int):
    import numpy as np
    return np.array([float(x) for x in interval_weights(k, L)], dtype=np.float64)


def exactness_degree(w, dmax: int = 12) -> int:
    """Largest d with sum_i w_i i^e == L^{e+1}/(e+1) exactly for all e <= d (-1 if none)."""
    L = len(w) - 1
    deg = -1
    for d in range(dmax + 1):
        lhs = sum(Fr(wi) * Fr(i) ** d for i, wi in enumerate(w))
        if lhs != Fr(L) ** (d + 1) / (d + 1):
            break
        deg = d
    return deg
