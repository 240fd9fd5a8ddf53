"""End-to-end sweep with the truncation active (GPU against the FP64 oracle, C ABI).

The generator is a sum of 20 damped exponentials with amplitudes spread
geometrically from 1 to 1e-10, so the blocks' singular values decay continuously
through eps_SVD = 1e-8 and every merge drops values near eps.  The dense oracle sums
the uncompressed data, so the difference is the truncation error of the compressed
history plus round-off.  For row n it is bounded a priori (section "Hierarchical
decomposition": each merge drops singular values below eps, so a block that received
M_b panel merges carries an error below M_b * eps in the spectral norm) by

    max_m |dI(n, m)| <= h * w_max * sum over levels l of
                        max over blocks b of level l of |x_n(rows of b)|_2 * M_b * eps

for the retarded sum (one block per level holds a column m), with the three
block products of the lesser sum bounded the same way.  The test asserts the
measured error against that bound and reports both.
"""
import numpy as np
import pytest

from gpu_common import dense_from_packed, host_inputs, oracle_rows, row, say, to_dev
from kbe_inputs import DampedExpSum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _geometric_terms(seed, nterms, lo):
    rng = np.random.default_rng(seed)
    omega = rng.uniform(-4.0, 4.0, nterms)
    gamma = rng.uniform(0.02, 0.2, nterms)
    amp = np.geomspace(1.0, lo, nterms).astype(np.complex128).reshape(nterms, 1, 1)
    fermi = 0.5 * (1.0 - np.tanh(0.5 * omega))
    return DampedExpSum(omega, gamma, amp, fermi, dict(kind="geometric", seed=seed))


def _merges_per_block(blocks, leaves, N, P_rows, n0):
    """Panel merges each block has received once rows [0, n0) are merged."""
    row_leaf = np.zeros(N, dtype=int)
    for i, (s0, s1) in enumerate(leaves):
        row_leaf[s0:s1] = i
    starts, p = [], 0
    while p < N:
        starts.append(p)
        q = p + 1
        while q < N and q - p < P_rows and row_leaf[q] == row_leaf[p]:
            q += 1
        p = q
    starts = np.array(starts)
    return [int(np.count_nonzero((starts >= r0) & (starts < min(r1, n0)))) for (_, r0, r1, _, _) in blocks]


def _check_against_bound(P, H, inp, IR, IL, IRg, ILg, N, h, k, nlvl, panel, eps):
    """Assert every row's error against the a-priori bound; return (worst error / bound,
    worst row relative error)."""
    blocks, leaves = H.blocks(), H.leaves()
    sR = dense_from_packed(inp[2], N)[..., 0, 0]   # Sigma^R(n, j)
    sL = dense_from_packed(inp[3], N)[..., 0, 0]   # Sigma^<(s, n) stored orientation
    w_max = max(abs(w) for L in range(2 * k + 2) for w in P.weights(k, L))
    worst_ratio, rel = 0.0, 0.0
    for n in range(N):
        # merges so far, counting every row up to n as merged (an upper bound)
        M = _merges_per_block(blocks, leaves, N, panel, n + 1)
        bR = bL = 0.0
        for lvl in range(1, nlvl + 1):
            cR = cL = 0.0
            for b, (bl, r0, r1, c0, c1) in enumerate(blocks):
                if bl != lvl or M[b] == 0:
                    continue
                rows_ = np.arange(r0, min(r1, n + 1))
                cols_ = np.arange(c0, min(c1, n + 1))
                x_rows = np.linalg.norm(sR[n, rows_])
                x_cols = np.linalg.norm(sR[n, cols_])
                x2_cols = np.linalg.norm(sL[n, cols_])   # |Sigma^<(n, s)| = |stored slice entry|
                cR = max(cR, x_rows * M[b] * eps)
                cL = max(cL, (x_cols + x_rows) * M[b] * eps + x2_cols * M[b] * eps)
            bR += cR
            bL += cL
        bR *= h * w_max
        bL *= h * w_max
        eR = np.abs(row(IRg, n) - IR[n]).max()
        eL = np.abs(row(ILg, n) - IL[n]).max()
        scale = max(np.abs(IR[n]).max(), np.abs(IL[n]).max(), 1e-300)
        assert eR <= bR + 1e-13 * scale, (panel, n, eR, bR)
        assert eL <= bL + 1e-13 * scale, (panel, n, eL, bL)
        if bR > 0:
            worst_ratio = max(worst_ratio, eR / bR, eL / max(bL, 1e-300))
        rel = max(rel, eR / max(np.abs(IR[n]).max(), 1e-300), eL / max(np.abs(IL[n]).max(), 1e-300))
    return worst_ratio, rel


def test_sweep_with_active_truncation(P):
    N, h, k, nlvl, panel, eps = 256, 0.05, 5, 3, 8, 1e-8
    G, S = _geometric_terms(41, 20, 1e-10), _geometric_terms(42, 20, 1e-10)
    inp = host_inputs(G, S, N, h)
    say("oracle: active truncation sweep")
    IR, IL = oracle_rows(*inp, N, h, k)
    H = P.Hodlr(N, nlvl, 1, k=k, tol=eps, panel=panel, max_rank=24)
    GR, GL, SR, SL = [to_dev(x) for x in inp]
    IRg, ILg = torch.zeros_like(GR), torch.zeros_like(GR)
    say("gpu: active truncation sweep")
    H.sweep(0, N, GR, GL, SR, SL, h, IRg, ILg)
    assert H.status() == 0
    IRg, ILg = IRg.cpu().numpy(), ILg.cpu().numpy()
    rk = H.ranks(P.RET)
    say("ranks (retarded)", rk.ravel().tolist())
    assert rk.max() >= 6          # the truncation is active: values on both sides of eps
    worst_ratio, rel = _check_against_bound(P, H, inp, IR, IL, IRg, ILg, N, h, k, nlvl, panel, eps)
    say(f"active truncation: worst error / a-priori bound {worst_ratio:.3e}; worst row relative error "
        f"{rel:.3e} (eps {eps:g})")


def test_rank_one_updates_against_panels(P):
    """Panel height 1 (the paper's row-by-row TSVD update) against panels of 16 rows on the
    active-truncation workload: both within the a-priori bound of their own merge counts,
    parity with the oracle on exact-rank inputs, and the drift of the per-row truncation
    (error of P = 1 relative to P = 16) reported."""
    N, h, k, nlvl, eps = 256, 0.05, 5, 3, 1e-8
    G, S = _geometric_terms(41, 20, 1e-10), _geometric_terms(42, 20, 1e-10)
    inp = host_inputs(G, S, N, h)
    say("oracle: rank-1 updates")
    IR, IL = oracle_rows(*inp, N, h, k)
    errs = {}
    for panel in (1, 16):
        H = P.Hodlr(N, nlvl, 1, k=k, tol=eps, panel=panel, max_rank=24)
        GR, GL, SR, SL = [to_dev(x) for x in inp]
        IRg, ILg = torch.zeros_like(GR), torch.zeros_like(GR)
        H.sweep(0, N, GR, GL, SR, SL, h, IRg, ILg)
        assert H.status() == 0
        IRg, ILg = IRg.cpu().numpy(), ILg.cpu().numpy()
        ratio, rel = _check_against_bound(P, H, inp, IR, IL, IRg, ILg, N, h, k, nlvl, panel, eps)
        errs[panel] = rel
        say(f"panel {panel}: worst row relative error {rel:.3e}, worst error / a-priori bound {ratio:.3e}, "
            f"max rank {int(H.ranks(P.RET).max())}")
    say(f"drift of row-by-row updates: relative error ratio P=1 / P=16 {errs[1] / max(errs[16], 1e-300):.2f}")
