"""Dense FP64 history sums (the definition the compressed method must reproduce).

Notation (paper, sections "Green's functions and Keldysh components" and
"Kadanoff-Baym equations"): t_j = j h; matrices are norb x norb; "@" is the
orbital-space matrix product.

Stored operands (the paper's lower-triangular storage):
  LR(j, m) = G^R(t_j, t_m),          j >= m
  LL(a, b) = G^<(t_b, t_a),          a >= b      (row a is the lesser slice at step a)
  sigR(n, j) = Sigma^R(t_n, t_j),    j <= n      (current retarded row of Sigma)
  sigL(n, s) = Sigma^<(t_s, t_n),    s <= n      (current lesser slice of Sigma, stored orientation)

Symmetries used to reach the other triangle (same section):
  G^<(s, m) = LL(m, s)                for s <= m
            = -LL(s, m)^dagger        for s > m          (anti-Hermitian lesser)
  G^A(s, m) = G^R(m, s)^dagger = LR(m, s)^dagger  for s <= m
  Sigma^<(t_n, t_s) = -sigL(n, s)^dagger

History integrals at step n, for every m <= n (right-hand sides of the
retarded and lesser KBE with t = t_n, t' = t_m; the mixed-branch term of the
lesser equation is not part of this path):
  I^R(n,m) = h sum_{j=m..n} w^{(n-m)}_{j-m} Sigma^R(n,j) @ G^R(j,m)
  I^<(n,m) = h sum_{s=0..n} w^{(n)}_s Sigma^R(n,s) @ G^<(s,m)
           + h sum_{s=0..m} w^{(m)}_s Sigma^<(n,s) @ G^A(s,m)
with the interval weights w^{(L)} of `oracle.weights.interval_weights`.
"""
from __future__ import annotations

import numpy as np

from .weights import interval_weights_f64


def _dag(x):
    return np.conj(np.swapaxes(x, -1, -2))


class ArrayOperands:
    """Operands held as dense arrays (small N).

    LR, LL: (N, N, norb, norb) stored lower triangles (upper parts ignored).
    SR: (N, N, norb, norb) with SR[n, j] = Sigma^R(t_n, t_j) for j <= n.
    SL: (N, N, norb, norb) with SL[n, s] = Sigma^<(t_s, t_n) for s <= n.
    """

    def __init__(self, LR, LL, SR, SL):
        self.LR_, self.LL_, self.SR_, self.SL_ = LR, LL, SR, SL

    def LR(self, j, m):
        return self.LR_[j, m]

    def LL(self, a, b):
        return self.LL_[a, b]

    def sigR(self, n, j):
        return self.SR_[n, j]

    def sigL(self, n, s):
        return self.SL_[n, s]


class GeneratorOperands:
    """Operands evaluated on the fly from damped-exponential generators (large N)."""

    def __init__(self, G, S, h):
        from kbe_inputs import generators as gen
        self.G, self.S, self.h, self.gen = G, S, h, gen

    def LR(self, j, m):
        return self.gen.retarded(self.G, np.asarray(j) * self.h, np.asarray(m) * self.h)

    def LL(self, a, b):
        return self.gen.lesser(self.G, np.asarray(b) * self.h, np.asarray(a) * self.h)

    def sigR(self, n, j):
        return self.gen.retarded(self.S, np.asarray(n) * self.h, np.asarray(j) * self.h)

    def sigL(self, n, s):
        return self.gen.lesser(self.S, np.asarray(s) * self.h, np.asarray(n) * self.h)


def g_lesser(ops, s, m):
    """G^<(t_s, t_m) for an index vector s and scalar m, from the stored triangle."""
    s = np.asarray(s)
    out = np.empty(s.shape + ops.LR(0, 0).shape, dtype=np.complex128)
    lo = s <= m
    if lo.any():
        out[lo] = ops.LL(np.full(lo.sum(), m), s[lo])
    if (~lo).any():
        out[~lo] = -_dag(ops.LL(s[~lo], np.full((~lo).sum(), m)))
    return out


def history_R_entry(ops, n: int, m: int, h: float, k: int):
    """I^R(n, m)."""
    L = n - m
    if L == 0:
        return np.zeros_like(ops.LR(0, 0))
    w = interval_weights_f64(k, L)
    j = np.arange(m, n + 1)
    return h * np.einsum("i,iab,ibc->ac", w, ops.sigR(n, j), ops.LR(j, np.full(L + 1, m)))


def history_lesser_entry(ops, n: int, m: int, h: float, k: int):
    """I^<(n, m)."""
    out = np.zeros_like(ops.LR(0, 0))
    if n > 0:
        s = np.arange(n + 1)
        w = interval_weights_f64(k, n)
        out += h * np.einsum("i,iab,ibc->ac", w, ops.sigR(n, s), g_lesser(ops, s, m))
    if m > 0:
        s = np.arange(m + 1)
        w = interval_weights_f64(k, m)
        sig_les = -_dag(ops.sigL(n, s))                         # Sigma^<(t_n, t_s)
        g_adv = _dag(ops.LR(np.full(m + 1, m), s))              # G^A(t_s, t_m)
        out += h * np.einsum("i,iab,ibc->ac", w, sig_les, g_adv)
    return out


def history_R_row(ops, n: int, h: float, k: int):
    """I^R(n, m) for m = 0..n, shape (n+1, norb, norb)."""
    return np.stack([history_R_entry(ops, n, m, h, k) for m in range(n + 1)])


def history_lesser_row(ops, n: int, h: float, k: int):
    """I^<(n, m) for m = 0..n, shape (n+1, norb, norb)."""
    return np.stack([history_lesser_entry(ops, n, m, h, k) for m in range(n + 1)])
