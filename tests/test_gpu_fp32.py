"""GPU parity of the FP32-factor form (U and V stored as complex float, everything
else FP64) against the FP64 oracle, called through the C ABI.

Bar: relative error <= max(1e-5, eps_SVD) per row (small grid) or per sampled
entry scaled by its row's maximum (full C4 grid, norb = 16, N_t = 8192,
eps_SVD = 1e-6, whose packed inputs do not fit in memory: rows are generated on
the device step by step).
"""
import time

import numpy as np
import pytest

from gpu_common import host_inputs, oracle_rows, row, row_rel_err, say, to_dev
from kbe_inputs import hermitian_terms, make_config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _sweep(obj, inp, N, h, norb):
    GR, GL, SR, SL = [to_dev(x) for x in inp]
    IR = torch.zeros((N * (N + 1) // 2, norb, norb), dtype=torch.complex128, device="cuda")
    IL = torch.zeros_like(IR)
    obj.sweep(0, N, GR, GL, SR, SL, h, IR, IL)
    torch.cuda.synchronize()
    return IR.cpu().numpy(), IL.cpu().numpy()


# norb 16 runs the matrix-core projections; with leaves starting at multiples of 16
# (N = 192, two levels: 48-row leaves) the matrix-core expansions of the combine too,
# whose 16-column tiles end ragged at every step n not of the form 16 i + 15
@pytest.mark.parametrize("norb,N,nlvl", [(4, 160, 3), (16, 160, 3), (16, 192, 2)])
def test_fp32_factors_small(P, norb, N, nlvl):
    h, k, tol = 0.03, 5, 1e-6
    G, S = hermitian_terms(41 + norb, 6, norb), hermitian_terms(51 + norb, 6, norb)
    inp = host_inputs(G, S, N, h)
    rows = sorted({0, 1, 2, 5, 15, 16, 17, 19, 20, 39, 40, 79, 80, 81, 100, 139, N // 2, N - 2, N - 1} |
                  set(range(N - 20, N, 3)))
    IR, IL = oracle_rows(*inp, N, h, k, rows=rows)
    H32 = P.Hodlr(N, nlvl, norb, k=k, tol=tol, panel=8, max_rank=16, flags=P.FLAG_FP32_FACTORS)
    IRg, ILg = _sweep(H32, inp, N, h, norb)
    assert H32.status() == 0
    H64 = P.Hodlr(N, nlvl, norb, k=k, tol=tol, panel=8, max_rank=16)
    assert H32.nbytes() > H64.nbytes()      # FP64 factors plus their complex-float mirrors
    worst = 0.0
    for n in rows:
        eR, eL = row_rel_err(row(IRg, n), IR[n]), row_rel_err(row(ILg, n), IL[n])
        worst = max(worst, eR, eL)
        assert eR <= 1e-5 and eL <= 1e-5, (n, eR, eL)
    say(f"fp32 factors norb={norb} worst row relative error", worst)
    # factor reconstruction in FP32 storage: close to the stored rows
    g = H32.get(P.RET, N - 10, 3)
    a = (N - 10) * (N - 9) // 2
    assert np.abs(g - inp[0][a + 3]).max() <= 1e-5 * np.abs(inp[0]).max()


def test_c4_full_size_sampled(P):
    from kbe_inputs.packed import RowSource
    from oracle.history import GeneratorOperands, history_lesser_entry, history_R_entry
    cfg, G, S = make_config_inputs("c4")
    N, h, k, norb, tol = cfg["nt"], cfg["h"], cfg["k"], cfg["norb"], cfg["tol"]
    nlvl = int(round(np.log2(N // cfg["leaf"])))
    dev = torch.device("cuda:0")
    gsrc, ssrc = RowSource(G, N, h, dev), RowSource(S, N, h, dev)
    gl = torch.empty((N, norb, norb), dtype=torch.complex128, device=dev)
    sl = torch.empty_like(gl)
    outR, outL = torch.empty_like(gl), torch.empty_like(gl)
    rng = np.random.default_rng(404)
    rows = sorted(set([0, 5, 63, 64, 4095, 4096, N - 1] + list(rng.integers(0, N, 2))))
    got = {}
    H = P.Hodlr(N, nlvl, norb, k=k, tol=tol, panel=16, max_rank=16, flags=P.FLAG_FP32_FACTORS)
    say("gpu: c4 sweep with device-generated rows", N, norb)
    t0 = time.perf_counter()
    # the history step reads the stored rows and factors without changing them, so it
    # is evaluated at the sampled rows only; every row is appended and every panel merged
    for n in range(N):
        H.append_row(P.RET, n, gsrc.ret(n))
        H.append_row(P.LES, n, gsrc.les(n, gl))
        if n in rows:
            H.history_step(n, ssrc.ret(n), ssrc.les(n, sl), h, outR[:n + 1], outL[:n + 1])
            got[n] = (outR[:n + 1].cpu().numpy(), outL[:n + 1].cpu().numpy())
        if n % 256 == 255:
            torch.cuda.synchronize()
            say("  step", n, f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    assert H.status() == 0
    say("max rank", max(int(H.ranks(c).max()) for c in (0, 1)), "device GiB", H.nbytes() / 2**30)
    ops = GeneratorOperands(G, S, h)
    worst = 0.0
    for n in rows:
        gR, gL = got[n]
        sR, sL = np.abs(gR).max(), np.abs(gL).max()
        for m in sorted(set(x for x in [0, n - 3, n] + list(rng.integers(0, n + 1, 2)) if 0 <= x <= n)):
            eR = np.abs(gR[m] - history_R_entry(ops, n, m, h, k)).max() / max(sR, 1e-300)
            eL = np.abs(gL[m] - history_lesser_entry(ops, n, m, h, k)).max() / max(sL, 1e-300)
            worst = max(worst, eR, eL)
            assert eR <= 1e-5 and eL <= 1e-5, (n, m, eR, eL)
    say("c4 fp32 worst sampled relative error", worst)
