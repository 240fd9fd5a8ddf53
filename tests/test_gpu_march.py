"""GPU parity of the paper's orientation (hnessi_row_march_R): rows of G^R marched along
the relative time over the compressed Sigma^R history, against the oracle's dense row
march (oracle.step_solve.row_march) on the same Sigma and eps.

Bar: max_m |G_gpu(n,m) - G_oracle(n,m)| / max_m |G_oracle(n,m)| <= 1e-10 per row (FP64,
Sigma compressed at 1e-12 on the small grids and at 1e-10 on the norb-4 N_t = 8192 grid,
where the generator's Sigma is exactly low-rank per block).  The small grids end in the
dense tail (rows above the merged front) and span several leaves and levels.
"""
import numpy as np
import pytest

from gpu_common import say, to_dev
from kbe_inputs import hermitian_drive, hermitian_terms, retarded, scalar_terms
from oracle.step_solve import row_march

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _sigma(pS, N, h):
    t = np.arange(N) * h
    norb = pS.norb
    S = np.zeros((N, N, norb, norb), dtype=np.complex128)
    for n in range(N):
        S[n, :n + 1] = retarded(pS, t[n], t[:n + 1])
    return S


@pytest.mark.parametrize("norb,k,N,nlvl", [(1, 5, 150, 2), (2, 3, 140, 2), (4, 5, 128, 1), (4, 4, 141, 2),
                                           (2, 1, 130, 2), (4, 2, 128, 1)])
def test_row_march_against_oracle(P, norb, k, N, nlvl):
    h = 0.02
    pS = scalar_terms(80 + k, 8) if norb == 1 else hermitian_terms(80 + k, 8, norb)
    S = _sigma(pS, N, h)
    eps = hermitian_drive(81 + k, norb, N, h)
    H = P.Hodlr(N, nlvl, norb, k=k, tol=1e-12, panel=16, max_rank=16)
    for n in range(N):
        H.append_row(P.RET, n, to_dev(S[n, :n + 1]))
    npair = norb * norb
    out = torch.zeros((N - k, N * npair), dtype=torch.complex128, device="cuda")
    H.row_march_R(k, N - 1, to_dev(eps), h, out, N * npair)
    torch.cuda.synchronize()
    H.status()
    G = out.cpu().numpy().reshape(N - k, N, norb, norb)
    worst = 0.0
    for n in list(range(k, N, 7)) + list(range(N - 8, N)):
        ref = row_march(S, eps, n, h, k)
        err = np.abs(G[n - k, :n + 1] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= 1e-10, (n, err)
    say(f"  row march norb {norb} k {k} N {N}: worst {worst:.2e}")


@pytest.mark.parametrize("norb,N,nlvl", [(4, 192, 2), (2, 256, 2)])
def test_row_march_rank_above_16(P, norb, N, nlvl):
    """Rank capacity 32 with block ranks above 16: the far field stages the projections of
    16 ranks at a time (two stages here), a lane of the projections holds up to 32 / (64 /
    norb^2) ranks, and the merges run at width 48.  Fast oscillations (|omega| up to 25) give
    the off-diagonal blocks epsilon-ranks of about 16 to 24."""
    h, k = 0.02, 5
    pS = hermitian_terms(97, 24, norb, omega_range=(-25.0, 25.0))
    S = _sigma(pS, N, h)
    eps = hermitian_drive(98, norb, N, h)
    H = P.Hodlr(N, nlvl, norb, k=k, tol=1e-12, panel=16, max_rank=32)
    for n in range(N):
        H.append_row(P.RET, n, to_dev(S[n, :n + 1]))
    assert H.status() == 0
    rmax = int(H.ranks(P.RET).max())
    assert rmax > 16, rmax
    npair = norb * norb
    out = torch.zeros((N - k, N * npair), dtype=torch.complex128, device="cuda")
    H.row_march_R(k, N - 1, to_dev(eps), h, out, N * npair)
    torch.cuda.synchronize()
    assert H.status() == 0
    G = out.cpu().numpy().reshape(N - k, N, norb, norb)
    worst = 0.0
    for n in list(range(k, N, 11)) + list(range(N - 6, N)):
        ref = row_march(S, eps, n, h, k)
        err = np.abs(G[n - k, :n + 1] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= 1e-10, (n, err)
    say(f"  row march norb {norb} N {N} max rank {rmax}: worst {worst:.2e}")


def test_row_march_argument_errors(P):
    N, norb, k = 64, 2, 5
    H = P.Hodlr(N, 1, norb, k=k, tol=1e-12, panel=16, max_rank=16)
    eps = torch.zeros((N, norb, norb), dtype=torch.complex128, device="cuda")
    out = torch.zeros((N, N * norb * norb), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.HnessiError):   # Sigma rows not appended
        H.row_march_R(k, 10, eps, 0.02, out, N * norb * norb)
    for n in range(12):
        H.append_row(P.RET, n, torch.zeros((n + 1, norb, norb), dtype=torch.complex128, device="cuda"))
    for lo, hi, stride in ((k - 1, 10, N * 4), (k, 11, 4), (7, 6, N * 4)):
        with pytest.raises(P.HnessiError):
            H.row_march_R(lo, hi, eps, 0.02, out, stride)
    H8 = P.Hodlr(N, 1, 8, k=k, tol=1e-12, panel=16, max_rank=16)
    with pytest.raises(P.HnessiError):   # norb 8 is not taken
        H8.row_march_R(k, 10, torch.zeros((N, 8, 8), dtype=torch.complex128, device="cuda"), 0.02,
                       torch.zeros((N, N * 64), dtype=torch.complex128, device="cuda"), N * 64)


def test_row_march_full_size_norb4(P):
    """The norb-4 N_t = 8192 grid (leaf 64, 7 levels, tolerance 1e-10) with the workload's
    Sigma generator, every Sigma row appended; rows k..8191 marched in one call (one launch,
    the longest rows first); rows 5, 100, 1023, 1024, 2047 and 2048 against the oracle (1024
    and 2048 are the first rows of a level-2 and a level-1 block's row range)."""
    from kbe_inputs import make_config_inputs
    from kbe_inputs.packed import RowSource
    cfg, _, pS = make_config_inputs("c2")
    N, norb, h, k, tol = cfg["nt"], cfg["norb"], cfg["h"], cfg["k"], cfg["tol"]
    npair = norb * norb
    nlvl = int(round(np.log2(N // cfg["leaf"])))
    eps = hermitian_drive(cfg["seed_s"] + 100, norb, N, h)
    src = RowSource(pS, N, h, "cuda")
    H = P.Hodlr(N, nlvl, norb, k=k, tol=tol, panel=16, max_rank=16)
    for n in range(N):
        H.append_row(P.RET, n, src.ret(n))
    checks = [5, 100, 1023, 1024, 2047, 2048]
    nmax = max(checks)
    out = torch.zeros((N - k, N * npair), dtype=torch.complex128, device="cuda")
    say(f"row march: rows {k}..{N - 1} of the N_t = {N} grid")
    H.row_march_R(k, N - 1, to_dev(eps), h, out, N * npair)
    torch.cuda.synchronize()
    H.status()
    last = out[N - 1 - k, :N * npair].cpu().numpy()
    assert np.all(np.isfinite(last))
    S = _sigma(pS, nmax + 1, h)
    worst = 0.0
    for n in checks:
        got = out[n - k, :(n + 1) * npair].cpu().numpy().reshape(n + 1, norb, norb)
        ref = row_march(S, eps, n, h, k)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        say(f"  row {n}: relative error {err:.2e}")
        assert err <= 1e-10, (n, err)
    say(f"  worst {worst:.2e}")
