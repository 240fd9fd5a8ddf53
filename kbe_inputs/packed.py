"""Packed lower-triangle inputs: rows 0..N-1 of a two-time function, row n at
element offset n(n+1)/2, each element norb x norb complex128.

Two builders with the same closed forms as `generators`: NumPy on the host
(small grids) and torch on a device (the full-size workloads, generated in HBM
so nothing of size N^2 crosses PCIe).  Input construction only.
"""
from __future__ import annotations

import numpy as np

from .generators import DampedExpSum, lesser, retarded


def _rows_cols(n0: int, n1: int):
    rows = np.repeat(np.arange(n0, n1), np.arange(n0, n1) + 1)
    starts = np.repeat(np.arange(n0, n1) * (np.arange(n0, n1) + 1) // 2, np.arange(n0, n1) + 1)
    cols = np.arange(rows.size) + (n0 * (n0 + 1) // 2) - starts
    return rows, cols


def packed_numpy(p: DampedExpSum, kind: str, N: int, h: float) -> np.ndarray:
    """kind 'ret': C^R(t_n, t_j); kind 'les': C^<(t_s, t_n) (stored orientation)."""
    rows, cols = _rows_cols(0, N)
    if kind == "ret":
        return retarded(p, rows * h, cols * h)
    if kind == "les":
        return lesser(p, cols * h, rows * h)
    raise ValueError(kind)


def packed_torch(p: DampedExpSum, kind: str, N: int, h: float, device, chunk_elems: int = 1 << 22):
    """Same as packed_numpy, built on a torch device in chunks of rows."""
    import torch
    norb, P = p.norb, p.nterms
    total = N * (N + 1) // 2
    out = torch.empty((total, norb, norb), dtype=torch.complex128, device=device)
    omega = torch.as_tensor(p.omega, dtype=torch.float64, device=device)
    gamma = torch.as_tensor(p.gamma, dtype=torch.float64, device=device)
    fermi = torch.as_tensor(p.fermi, dtype=torch.float64, device=device)
    amp = torch.as_tensor((p.amp if kind == "ret" else p.herm_amp).reshape(P, norb * norb),
                          dtype=torch.complex128, device=device)
    n0 = 0
    while n0 < N:
        n1 = n0 + 1
        while n1 < N and (n1 * (n1 + 1) - n0 * (n0 + 1)) // 2 + n1 + 1 <= chunk_elems:
            n1 += 1
        a, b = n0 * (n0 + 1) // 2, n1 * (n1 + 1) // 2
        nrow = torch.arange(n0, n1, device=device, dtype=torch.int64)
        rows = torch.repeat_interleave(nrow, nrow + 1)
        idx = torch.arange(a, b, device=device, dtype=torch.int64)
        cols = idx - rows * (rows + 1) // 2
        t_row = rows.to(torch.float64) * h
        t_col = cols.to(torch.float64) * h
        if kind == "ret":
            tau = (t_row - t_col)[:, None]
            ph = torch.exp(torch.complex(-gamma[None, :] * tau, -omega[None, :] * tau))
            blk = (-1j) * (ph @ amp)
        elif kind == "les":
            t1, t2 = t_col[:, None], t_row[:, None]     # C^<(t_s, t_n)
            ph = fermi[None, :] * torch.exp(torch.complex(-0.5 * gamma[None, :] * (t1 + t2),
                                                          -omega[None, :] * (t1 - t2)))
            blk = 1j * (ph @ amp)
        else:
            raise ValueError(kind)
        out[a:b] = blk.reshape(-1, norb, norb)
        n0 = n1
    return out


def row_of(packed, n: int):
    """View of row n of a packed triangle."""
    a = n * (n + 1) // 2
    return packed[a:a + n + 1]


class RowSource:
    """Rows of C^R and C^< generated on a device one step at a time, for grids whose
    packed triangles do not fit in memory (norb = 16, N = 8192: 137 GB per triangle).

    The retarded part depends on t_n - t_j only, so row n is the contiguous slice
    [N-1-n, N) of one reversed table of C^R(d h, 0), d = 0..N-1.  The lesser part
    factorizes per term into a function of t_s times a function of t_n; row n is
    (E[:n+1] * c(n)) @ H with E[s, p] = exp(-(i w_p + g_p / 2) t_s) tabulated once.
    Input construction only.
    """

    def __init__(self, p: DampedExpSum, N: int, h: float, device):
        import torch
        self.N, self.h, self.norb = N, h, p.norb
        P, npair = p.nterms, p.norb * p.norb
        dev = torch.device(device)
        omega = torch.as_tensor(p.omega, dtype=torch.float64, device=dev)
        gamma = torch.as_tensor(p.gamma, dtype=torch.float64, device=dev)
        self.fermi = torch.as_tensor(p.fermi, dtype=torch.float64, device=dev)
        amp = torch.as_tensor(p.amp.reshape(P, npair), dtype=torch.complex128, device=dev)
        self.hamp = torch.as_tensor(p.herm_amp.reshape(P, npair), dtype=torch.complex128, device=dev)
        self.omega, self.gamma = omega, gamma
        t = torch.arange(N, dtype=torch.float64, device=dev) * h
        tau = t.flip(0)[:, None]                                   # (N-1-i) h at index i
        ph = torch.exp(torch.complex(-gamma[None, :] * tau, -omega[None, :] * tau))
        self.ret_rev = ((-1j) * (ph @ amp)).reshape(N, p.norb, p.norb).contiguous()
        self.E = torch.exp(torch.complex(-0.5 * gamma[None, :] * t[:, None], -omega[None, :] * t[:, None]))
        self.buf = torch.empty((N, p.norb, p.norb), dtype=torch.complex128, device=dev)

    def ret(self, n: int):
        """C^R(t_n, t_j), j = 0..n (a view)."""
        return self.ret_rev[self.N - 1 - n:]

    def les(self, n: int, out=None):
        """C^<(t_s, t_n), s = 0..n, written into out (default: an internal buffer)."""
        import torch
        tn = n * self.h
        coef = 1j * self.fermi * torch.exp(torch.complex(-0.5 * self.gamma * tn, self.omega * tn))
        dst = self.buf if out is None else out
        torch.matmul(self.E[:n + 1] * coef[None, :], self.hamp, out=dst[:n + 1].view(n + 1, -1))
        return dst[:n + 1]
