"""torch.autograd wrapper of the retarded history sums over a whole sweep.

history_R(H, GR, SR, h) returns the packed triangle I^R(n, m) of a sweep
n = 0..N-1 over the retarded rows GR and is differentiable with respect to SR
(the packed Sigma^R rows).  H only supplies the parameters: every forward builds
its compressed state in a handle of its own, kept by the autograd graph, so a
later forward cannot change the state a pending backward reads.

The backward evaluates every step over that frozen final state (the compressed
G^R of all rows) instead of replaying the appends and merges: per step the
library recomputes the projected rows x_n U_b and Ibar_n V_b from the stored
factors and returns
  dL/dSigma^R(n, j) = h sum_{m<=j} w^{(n-m)}_{j-m} Ibar(n, m) G^R(j, m)^dagger,
and, with factor_grads=True, accumulates the gradients with respect to the
factors of every block, dU = Gbar V S, dV = Gbar^dagger U S, dS = Re diag(U^dagger
Gbar V), Gbar(j, m) = h sum_n w^{(n-m)}_{j-m} Sigma^R(n, j)^dagger Ibar(n, m).
Pass a dict as `state` to receive the private handle (state["handle"]) whose
factors and factor gradients (Hodlr.factors, Hodlr.factor_grad_get) these are.
The forward of step n uses the factors current at step n, which differ from the
final ones by the truncation of the later merges (below eps_SVD), so the backward
is the exact adjoint of the final compressed operator.  Every step runs in the
HIP library; this module only orders the calls.
"""
from __future__ import annotations

import torch

from ._lib import RET, Hodlr


def _row(t, n):
    a = n * (n + 1) // 2
    return t[a:a + n + 1]


class _HistoryR(torch.autograd.Function):
    @staticmethod
    def forward(ctx, SR, spec, GR, h, factor_grads, state):
        H = Hodlr(**spec)
        N = H.nt
        IR = torch.empty_like(SR)
        for n in range(N):
            H.append_row(RET, n, _row(GR, n))
            H.history_R(n, _row(SR, n), h, _row(IR, n))
        ctx.H, ctx.h, ctx.factor_grads, ctx.state = H, h, factor_grads, state
        ctx.save_for_backward(SR)
        if state is not None:
            state["handle"] = H
        return IR

    @staticmethod
    def backward(ctx, gIR):
        H, h = ctx.H, ctx.h
        (SR,) = ctx.saved_tensors
        gIR = gIR.contiguous()
        gSR = torch.empty_like(gIR)
        if ctx.factor_grads:
            H.factor_grad_reset()
        for n in range(H.nt):
            H.history_R_adjoint(n, _row(gIR, n), h, _row(gSR, n))
            if ctx.factor_grads:
                H.factor_grad(n, _row(SR, n), _row(gIR, n), h)
        if ctx.state is not None:
            ctx.state["factor_grads"] = ctx.factor_grads
        return gSR, None, None, None, None, None


def history_R(H, GR, SR, h, factor_grads=False, state=None):
    """Packed I^R of a full sweep, differentiable with respect to SR; H gives the handle
    parameters (its own state is not used)."""
    return _HistoryR.apply(SR, H.spec(), GR, h, factor_grads, state)
