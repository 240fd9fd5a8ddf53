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
The same sum is linear in G^R as well; over a sweep n = 0..N-1 the gradient
with respect to the stored entry G^R(t_j, t_m), j >= m, is
  Gbar(j, m) = h sum_{n=j..N-1} w^{(n-m)}_{j-m} Sigma^R(n,j)^dagger Ibar(n,m)
(zero weight for n = m, whose interval is empty).  Through a block's truncated
SVD G = U S V^H (section "Hierarchical decomposition") this gives the factor
gradients dU = Gbar V S, dV = Gbar^dagger U S, dS = Re diag(U^dagger Gbar V).
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


def history_R_G_gradient(ops, ibar, N: int, h: float, k: int, rows, cols):
    """Gbar(j, m) for j in rows, m in cols (entries with m > j are zero), shape
    (len(rows), len(cols), norb, norb), for a sweep of N steps; ibar(ns, m) returns the
    cotangents Ibar(n, m) for an index vector ns, shape (len(ns), norb, norb)."""
    rows, cols = list(rows), list(cols)
    norb = np.asarray(ops.sigR(0, 0)).shape[-1]
    out = np.zeros((len(rows), len(cols), norb, norb), dtype=np.complex128)
    wtab = {}   # interval weights by length, computed once each
    for a, j in enumerate(rows):
        for b, m in enumerate(cols):
            if m > j:
                continue
            ns = np.arange(max(j, m + 1), N)
            if len(ns) == 0:
                continue
            for L in set((ns - m).tolist()) - wtab.keys():
                wtab[L] = interval_weights_f64(k, L)
            w = np.array([wtab[n - m][j - m] for n in ns])
            sig = ops.sigR(ns, np.full(len(ns), j))       # Sigma^R(n, j)
            out[a, b] = h * np.einsum("n,nab,nac->bc", w, np.conj(sig), ibar(ns, m))
    return out


def factor_gradients(Gbar, U, S, V):
    """(dU, dS, dV) of one block and orbital pair from its entry gradient Gbar
    (rows x cols) and factors U (rows x r), S (r), V (cols x r)."""
    dU = Gbar @ V * S[None, :]
    dV = _dag(Gbar) @ U * S[None, :]
    dS = np.real(np.einsum("jr,jm,mr->r", np.conj(U), Gbar, V))
    return dU, dS, dV
