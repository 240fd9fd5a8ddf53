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


def _entry_worker(args):
    G, S, h, k, n, ms = args
    from oracle.history import GeneratorOperands, history_lesser_entry, history_R_entry
    ops = GeneratorOperands(G, S, h)
    return [(history_R_entry(ops, n, m, h, k), history_lesser_entry(ops, n, m, h, k)) for m in ms]


def oracle_entries(G, S, h, k, cols_by_row, workers=8):
    """Oracle I^R(n, m) and I^<(n, m) for {n: [m, ...]}, from the generators, computed by a
    pool of spawned processes (no GPU state is inherited).  Returns {n: (mlist, R, L)}."""
    import multiprocessing as mp
    jobs = []
    for n, ms in cols_by_row.items():
        ms = list(ms)
        for i in range(0, len(ms), 8):
            jobs.append((G, S, h, k, n, ms[i:i + 8]))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        res = pool.map(_entry_worker, jobs)
    out = {}
    for (G_, S_, h_, k_, n, ms), vals in zip(jobs, res):
        o = out.setdefault(n, ([], [], []))
        for m, (r, l) in zip(ms, vals):
            o[0].append(m)
            o[1].append(r)
            o[2].append(l)
    return {n: (np.array(v[0]), np.stack(v[1]), np.stack(v[2])) for n, v in out.items()}


def boundary_columns(n, leaf, nlvl, rng, total=64):
    """At least `total` columns m <= n: 0..2, n-6..n, every level boundary leaf*2^l and its
    neighbours, a few other leaf and block boundaries, the rest uniform."""
    ms = {0, 1, 2} | set(range(max(0, n - 6), n + 1))
    for l in range(nlvl + 1):
        b = leaf * 2 ** l
        ms |= {b - 1, b, b + 1}
        ms |= {3 * b - 1, 3 * b, 3 * b + 1}
    ms |= {n - n % leaf, n - n % leaf - 1}
    ms = {m for m in ms if 0 <= m <= n}
    while len(ms) < min(total, n + 1):
        ms.add(int(rng.integers(0, n + 1)))
    return sorted(ms)


def check_entries(label, got_R, got_L, ref, tol):
    """Per row n: max over the sampled columns of |got - ref| divided by the oracle's
    maximum over the same columns (both components).  Returns the worst ratio."""
    worst = 0.0
    for n, (ms, R, L) in ref.items():
        gR, gL = got_R[n][ms], got_L[n][ms]
        sR, sL = max(np.abs(R).max(), 1e-300), max(np.abs(L).max(), 1e-300)
        eR = np.abs(gR - R).max() / sR
        eL = np.abs(gL - L).max() / sL
        worst = max(worst, eR, eL)
        assert eR <= tol, (label, "R", n, eR)
        assert eL <= tol, (label, "L", n, eL)
    say(label, "worst sampled relative error", worst)
    return worst


def oracle_entries_multi(jobs, workers=16):
    """Oracle I^R(n, m) and I^<(n, m) for a list of (G, S, h, k, n, [m, ...]) jobs of possibly
    different objects, one spawned pool for all; returns one list of (R, L) per job."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return pool.map(_entry_worker, jobs)
