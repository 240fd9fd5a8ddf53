"""Pins for the oracle's dense history sums.

Pinned against: exact polynomial integrals (Gregory/Newton-Cotes exactness),
non-commuting constant matrices (orbital order, conjugations), anti-Hermitian
polynomial lesser kernels (storage orientation and symmetries), and the
closed-form convolution of damped exponentials with its convergence order.
"""
import math

import numpy as np
import pytest

from kbe_inputs import make_config_inputs, ret_row, les_row
from oracle.closed_form import lesser_convolution, retarded_convolution, phi
from oracle.history import (ArrayOperands, GeneratorOperands, history_lesser_entry,
                            history_lesser_row, history_R_entry, history_R_row)

DEG = {1: 1, 2: 3, 3: 3, 4: 5, 5: 5}


def _rand_mat(rng, n):
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def _herm(rng, n):
    a = _rand_mat(rng, n)
    return a + np.conj(a.T)


def _build(N, h, fR, fSR, fL, fSL, norb):
    """Dense operand arrays from functions of (t, t') returning norb x norb."""
    LR = np.zeros((N, N, norb, norb), complex)
    LL = np.zeros_like(LR)
    SR = np.zeros_like(LR)
    SL = np.zeros_like(LR)
    for a in range(N):
        for b in range(a + 1):
            LR[a, b] = fR(a * h, b * h)
            LL[a, b] = fL(b * h, a * h)          # stored lesser: L^<[a][b] = G^<(t_b, t_a)
            SR[a, b] = fSR(a * h, b * h)
            SL[a, b] = fSL(b * h, a * h)         # current slice at step a: Sigma^<(t_b, t_a)
    return ArrayOperands(LR, LL, SR, SL)


@pytest.mark.parametrize("k", range(1, 6))
def test_retarded_polynomial_exact(k):
    h = 0.1
    N = 2 * k + 9
    for d in range(DEG[k] + 1):
        for e in range(DEG[k] + 1 - d):
            ops = _build(N, h,
                         lambda t, tp: np.array([[(t - tp) ** d]], complex),
                         lambda t, tp: np.array([[(t - tp) ** e]], complex),
                         lambda t, tp: np.zeros((1, 1)), lambda t, tp: np.zeros((1, 1)), 1)
            for n in range(k, N):
                for m in range(0, n - k + 1):
                    tau = (n - m) * h
                    exact = tau ** (d + e + 1) * math.factorial(d) * math.factorial(e) \
                        / math.factorial(d + e + 1)
                    got = history_R_entry(ops, n, m, h, k)[0, 0]
                    assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact))


def test_retarded_short_interval_newton_cotes():
    # n - m < k uses Newton-Cotes on the L+1 points; exact to degree L (odd L) / L+1 (even L)
    k, h, N = 5, 0.1, 8
    for d in range(4):
        ops = _build(N, h, lambda t, tp: np.array([[(t - tp) ** d]], complex),
                     lambda t, tp: np.ones((1, 1), complex),
                     lambda t, tp: np.zeros((1, 1)), lambda t, tp: np.zeros((1, 1)), 1)
        for L in range(1, k):
            if d > (L if L % 2 else L + 1):
                continue
            got = history_R_entry(ops, 6, 6 - L, h, k)[0, 0]
            assert abs(got - (L * h) ** (d + 1) / (d + 1)) < 1e-13


def test_retarded_matrix_order():
    rng = np.random.default_rng(0)
    A, C = _rand_mat(rng, 3), _rand_mat(rng, 3)
    assert np.abs(A @ C - C @ A).max() > 1e-3
    h, N, k = 0.05, 14, 3
    ops = _build(N, h, lambda t, tp: C, lambda t, tp: A,
                 lambda t, tp: np.zeros((3, 3)), lambda t, tp: np.zeros((3, 3)), 3)
    for n in range(N):
        for m in range(n + 1):
            np.testing.assert_allclose(history_R_entry(ops, n, m, h, k), (n - m) * h * (A @ C),
                                       atol=1e-13)


@pytest.mark.parametrize("k", range(1, 6))
def test_lesser_polynomial_symmetries(k):
    """G^<(t,t') = i t t' H + (t - t') R (anti-Hermitian), Sigma^R = A, Sigma^< = i K,
    G^R(t,t') = (t - t') C: both integrands are linear in s, so every rule is exact."""
    rng = np.random.default_rng(k)
    no = 2
    A, C = _rand_mat(rng, no), _rand_mat(rng, no)
    H, R, K = _herm(rng, no), _herm(rng, no), _herm(rng, no)
    h, N = 0.1, 2 * k + 6
    ops = _build(N, h,
                 lambda t, tp: (t - tp) * C,
                 lambda t, tp: A,
                 lambda t, tp: 1j * t * tp * H + (t - tp) * R,
                 lambda t, tp: 1j * K, no)
    for n in range(N):
        tn = n * h
        for m in range(n + 1):
            tm = m * h
            # int_0^{t_n} A G^<(s, t_m) ds  and  int_0^{t_m} (iK) (t_m - s) C^dagger ds
            t1 = A @ (1j * tm * H * tn ** 2 / 2 + R * (tn ** 2 / 2 - tm * tn))
            t2 = 1j * K @ np.conj(C.T) * tm ** 2 / 2
            np.testing.assert_allclose(history_lesser_entry(ops, n, m, h, k), t1 + t2,
                                       atol=1e-12)


def test_lesser_second_term_polynomial_exact():
    # Sigma^<(t,s) = i (t - s)^e K-like scalar, G^R = (t - t')^d: exact to degree DEG[k]
    k, h, N = 4, 0.1, 16
    for d in range(3):
        for e in range(3 - d + 1):
            ops = _build(N, h, lambda t, tp: np.array([[(t - tp) ** d]], complex),
                         lambda t, tp: np.zeros((1, 1)),
                         lambda t, tp: np.zeros((1, 1)),
                         lambda t, tp: np.array([[1j * (tp - t) ** e if tp >= t else
                                                  1j * (tp - t) ** e]], complex), 1)
            # Sigma^<(t_n, s) = -conj(slice) = -conj(i (t_n - s)^e) = i (t_n - s)^e
            n = N - 1
            for m in range(k, n + 1):
                tm, tn = m * h, n * h
                # int_0^{tm} i (tn - s)^e (tm - s)^d ds, exact via polynomial expansion
                poly = np.polynomial.polynomial
                pe = poly.polypow([tn, -1.0], e)
                pd = poly.polypow([tm, -1.0], d)
                ip = poly.polyint(poly.polymul(pe, pd))
                exact = 1j * (poly.polyval(tm, ip) - poly.polyval(0.0, ip))
                got = history_lesser_entry(ops, n, m, h, k)[0, 0]
                assert abs(got - exact) < 1e-11, (d, e, m)


@pytest.mark.parametrize("k,order", [(1, 3), (2, 4), (3, 5), (4, 6)])
@pytest.mark.parametrize("key", ["c1", "c2"])
def test_closed_form_convergence_order(key, k, order):
    cfg, G, S = make_config_inputs(key)
    errs = {"R": [], "L": []}
    hs = [0.08, 0.04, 0.02, 0.01]
    for h in hs:
        ops = GeneratorOperands(G, S, h)
        n, m = int(round(2.56 / h)), int(round(0.96 / h))
        errs["R"].append(np.abs(history_R_entry(ops, n, m, h, k)
                                - retarded_convolution(S, G, n * h, m * h)).max())
        errs["L"].append(np.abs(history_lesser_entry(ops, n, m, h, k)
                                - lesser_convolution(S, G, n * h, m * h)).max())
    for comp in "RL":
        # least-squares slope of log(error) against log(h); pre-asymptotic wiggles
        # of a few tenths are normal, a wrong weight or index drops the slope by >= 1
        slope = np.polyfit(np.log(hs), np.log(errs[comp]), 1)[0]
        assert slope > order - 0.75, (comp, slope)


@pytest.mark.parametrize("key", ["c1", "c2"])
def test_closed_form_k5_accuracy(key):
    cfg, G, S = make_config_inputs(key)
    h = 0.01
    ops = GeneratorOperands(G, S, h)
    for n, m in [(300, 0), (300, 137), (300, 290)]:
        exR = retarded_convolution(S, G, n * h, m * h)
        exL = lesser_convolution(S, G, n * h, m * h)
        assert np.abs(history_R_entry(ops, n, m, h, 5) - exR).max() < 1e-9
        assert np.abs(history_lesser_entry(ops, n, m, h, 5) - exL).max() < 1e-9


def test_phi_equal_rates_limit():
    a = 0.3 + 1.1j
    for tau in [0.0, 0.5, 3.0]:
        assert abs(phi(a, a, tau) - tau * np.exp(-a * tau)) < 1e-14
        assert abs(phi(a, a + 1e-9, tau) - tau * np.exp(-a * tau)) < 1e-8


def test_array_and_generator_operands_agree():
    cfg, G, S = make_config_inputs("c2")
    h, N = 0.05, 12
    LR = np.zeros((N, N, 4, 4), complex)
    LL, SR, SL = np.zeros_like(LR), np.zeros_like(LR), np.zeros_like(LR)
    for n in range(N):
        LR[n, :n + 1] = ret_row(G, n, h)
        LL[n, :n + 1] = les_row(G, n, h)
        SR[n, :n + 1] = ret_row(S, n, h)
        SL[n, :n + 1] = les_row(S, n, h)
    a_ops = ArrayOperands(LR, LL, SR, SL)
    g_ops = GeneratorOperands(G, S, h)
    for n in [0, 1, 4, 7, 11]:
        np.testing.assert_allclose(history_R_row(a_ops, n, h, 5), history_R_row(g_ops, n, h, 5),
                                   rtol=0, atol=1e-14)
        np.testing.assert_allclose(history_lesser_row(a_ops, n, h, 5),
                                   history_lesser_row(g_ops, n, h, 5), rtol=0, atol=1e-14)


def test_generated_lesser_is_anti_hermitian():
    cfg, G, S = make_config_inputs("c2")
    from kbe_inputs import lesser
    t = np.array([0.3, 1.7, 5.0])
    tp = np.array([2.2, 0.4, 5.0])
    a = lesser(G, t, tp)
    b = lesser(G, tp, t)
    np.testing.assert_allclose(a, -np.conj(np.swapaxes(b, -1, -2)), atol=1e-15)
