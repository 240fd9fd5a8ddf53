"""Closed-form history integrals for damped-exponential generators (pins only).

With Sigma^R(t,s) = -i sum_p A_p e^{-a_p (t-s)} (a_p = i w_p + g_p) and
G^R(s,t') = -i sum_q C_q e^{-b_q (s-t')} (b_q = i v_q + d_q):

  int_{t'}^{t} Sigma^R(t,s) G^R(s,t') ds = - sum_{p,q} A_p C_q phi(a_p, b_q; t - t'),
  phi(a, b; tau) = (e^{-b tau} - e^{-a tau}) / (a - b)   (= tau e^{-a tau} if a = b).

With the smooth lesser forms of `kbe_inputs` (Hermitian parts K_p of Sigma's and
H_q of G's amplitudes, Fermi weights f):

  int_0^t Sigma^R(t,s) G^<(s,t') ds
      = sum_{p,q} f_q A_p H_q e^{(i v_q - d_q/2) t'} phi(a_p, i v_q + d_q/2; t)
  int_0^{t'} Sigma^<(t,s) G^A(s,t') ds
      = - sum_{p,q} f_p K_p C_q^dagger e^{-(i w_p + g_p/2) t} phi(conj(b_q), -i w_p + g_p/2; t')

Both follow from int_0^T e^{z s} ds = (e^{zT} - 1)/z; phi is evaluated through
expm1 of an argument with non-positive real part, so no cancellation occurs.
"""
from __future__ import annotations

import numpy as np


def _expm1_over(x):
    """expm1(x)/x for complex x, accurate near 0."""
    x = np.asarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-5
    xs = x[small]
    out[small] = 1 + xs / 2 + xs * xs / 6 + xs ** 3 / 24
    xl = x[~small]
    out[~small] = np.expm1(xl) / xl
    return out


def phi(a, b, tau):
    """(e^{-b tau} - e^{-a tau}) / (a - b), broadcasting, cancellation-free."""
    a, b, tau = np.broadcast_arrays(np.asarray(a, np.complex128), np.asarray(b, np.complex128),
                                    np.asarray(tau, np.float64))
    d = a - b
    # e^{-b tau} (1 - e^{-d tau})/d = tau e^{-b tau} * (-(expm1(-d tau))/(d tau))
    use_b = d.real >= 0
    out = np.empty(a.shape, dtype=np.complex128)
    x = -d * tau
    out[use_b] = (tau * np.exp(-b * tau) * _expm1_over(x))[use_b]
    y = d * tau
    out[~use_b] = (tau * np.exp(-a * tau) * _expm1_over(y))[~use_b]
    return out


def retarded_convolution(S, G, t, tp):
    """int_{t'}^{t} Sigma^R(t,s) G^R(s,t') ds for scalar t >= t'."""
    a = 1j * S.omega + S.gamma
    b = 1j * G.omega + G.gamma
    ph = phi(a[:, None], b[None, :], t - tp)                             # (P, Q)
    return -np.einsum("pq,pab,qbc->ac", ph, S.amp, G.amp)


def lesser_convolution(S, G, t, tp):
    """int_0^t Sigma^R(t,s) G^<(s,t') ds + int_0^{t'} Sigma^<(t,s) G^A(s,t') ds."""
    a = 1j * S.omega + S.gamma
    v, d = G.omega, G.gamma
    ph1 = phi(a[:, None], (1j * v + d / 2)[None, :], t) * \
        (G.fermi * np.exp((1j * v - d / 2) * tp))[None, :]
    t1 = np.einsum("pq,pab,qbc->ac", ph1, S.amp, G.herm_amp)
    bq = 1j * G.omega + G.gamma
    w, g = S.omega, S.gamma
    ph2 = phi(np.conj(bq)[None, :], (-1j * w + g / 2)[:, None], tp) * \
        (S.fermi * np.exp(-(1j * w + g / 2) * t))[:, None]
    cdag = np.conj(np.swapaxes(G.amp, -1, -2))
    t2 = -np.einsum("pq,pab,qbc->ac", ph2, S.herm_amp, cdag)
    return t1 + t2
