"""torch.autograd wrapper of the retarded history sums over a whole sweep.

history_R(H, GR, SR, h) returns the packed triangle I^R(n, m) of a sweep
n = 0..N-1 over the retarded rows GR (appended into the HODLR handle H, which
is reset first) and is differentiable with respect to SR (the packed Sigma^R
rows).  Sigma^R(n, .) enters step n only, so the backward pass replays the
appends (recomputing the compressed state of every step instead of storing
it) and calls the library's adjoint kernel at each step:
  dL/dSigma^R(n, j) = h sum_{m<=j} w^{(n-m)}_{j-m} dL/dI^R(n, m) G^R(j, m)^dagger.
Gradients with respect to G^R (the factors) are not produced.  Every step runs
in the HIP library; this module only orders the calls.
"""
from __future__ import annotations

import torch

from ._lib import RET


def _row(t, n):
    a = n * (n + 1) // 2
    return t[a:a + n + 1]


class _HistoryR(torch.autograd.Function):
    @staticmethod
    def forward(ctx, SR, H, GR, h):
        N = H.nt
        IR = torch.empty_like(SR)
        H.reset()
        for n in range(N):
            H.append_row(RET, n, _row(GR, n))
            H.history_R(n, _row(SR, n), h, _row(IR, n))
        ctx.H, ctx.GR, ctx.h = H, GR, h
        return IR

    @staticmethod
    def backward(ctx, gIR):
        H, GR, h = ctx.H, ctx.GR, ctx.h
        gIR = gIR.contiguous()
        gSR = torch.empty_like(gIR)
        H.reset()
        for n in range(H.nt):
            H.append_row(RET, n, _row(GR, n))
            H.history_R_adjoint(n, _row(gIR, n), h, _row(gSR, n))
        return gSR, None, None, None


def history_R(H, GR, SR, h):
    """Packed I^R of a full sweep, differentiable with respect to SR."""
    return _HistoryR.apply(SR, H, GR, h)
