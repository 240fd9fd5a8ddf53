"""Adjoint of the retarded history sum (test infrastructure, like the rest of
this package).

At step n the retarded history sum is linear in the Sigma^R row (Eq. KBER's
history term with the interval weights of the appendix on integration):
  I^R(n,m) = h sum_{j=m..n} w^{(n-m)}_{j-m} Sigma^R(n,j) @ G^R(j,m),   m = 0..n.
For the real inner product <A, B> = Re sum tr(A^dagger B) its adjoint maps a
cotangent row Ibar(n, m), m = 0..n, to
  Sbar(j) = h sum_{m=0..j} w^{(n-m)}_{j-m} Ibar(n,m) @ G^R(j,m)^dagger,  j = 0..n.
This is the gradient of a real loss of I^R with respect to Sigma^R(n, .) in the
convention dL/dRe + i dL/dIm (torch's for complex tensors); for
L = sum_m c_m |I^R(n,m)|_F^2 the cotangent is Ibar(n,m) = 2 c_m I^R(n,m).
Written from the definition: every term of the forward sum, transposed.
"""
from __future__ import annotations

import numpy as np

from .weights import interval_weights_f64


def _dag(x):
    return np.conj(np.swapaxes(x, -1, -2))


def history_R_adjoint_entry(ops, n: int, j: int, ibar, h: float, k: int):
    """Sbar(j) for a cotangent row ibar (n+1, norb, norb)."""
    m = np.arange(j + 1)
    # weight of the term (j, m) in I^R(n, m); zero for m = n (empty interval)
    w = np.array([interval_weights_f64(k, n - mm)[j - mm] if n > mm else 0.0 for mm in m])
    g = ops.LR(np.full(j + 1, j), m)                      # G^R(t_j, t_m)
    return h * np.einsum("i,iab,icb->ac", w, ibar[:j + 1], np.conj(g))


def history_R_adjoint_row(ops, n: int, ibar, h: float, k: int):
    """Sbar(j) for j = 0..n, shape (n+1, norb, norb)."""
    return np.stack([history_R_adjoint_entry(ops, n, j, ibar, h, k) for j in range(n + 1)])
