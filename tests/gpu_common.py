"""Shared helpers of the GPU parity tests (inputs, oracle rows, error metric)."""
from __future__ import annotations

import sys

import numpy as np

from kbe_inputs.packed import packed_numpy
from oracle.history import ArrayOperands, history_lesser_row, history_R_row


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dense_from_packed(pk, N):
    """(N, N, norb, norb) lower-triangle array from a packed triangle."""
    norb = pk.shape[-1]
    out = np.zeros((N, N, norb, norb), dtype=np.complex128)
    for n in range(N):
        a = n * (n + 1) // 2
        out[n, :n + 1] = pk[a:a + n + 1]
    return out


def host_inputs(G, S, N, h):
    """Packed (GR, GL, SR, SL) numpy triangles for a sweep."""
    return (packed_numpy(G, "ret", N, h), packed_numpy(G, "les", N, h),
            packed_numpy(S, "ret", N, h), packed_numpy(S, "les", N, h))


def oracle_rows(GR, GL, SR, SL, N, h, k, rows=None):
    """Oracle I^R and I^< rows (dict n -> array) from packed inputs."""
    ops = ArrayOperands(dense_from_packed(GR, N), dense_from_packed(GL, N),
                        dense_from_packed(SR, N), dense_from_packed(SL, N))
    rows = range(N) if rows is None else rows
    IR = {n: history_R_row(ops, n, h, k) for n in rows}
    IL = {n: history_lesser_row(ops, n, h, k) for n in rows}
    return IR, IL


def row_rel_err(got, ref):
    """max_m |got - ref| / max_m |ref| over one row (complex, any shape)."""
    scale = np.abs(ref).max()
    if scale == 0.0:
        return float(np.abs(got).max())
    return float(np.abs(got - ref).max() / scale)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def row(pk, n):
    a = n * (n + 1) // 2
    return pk[a:a + n + 1]
