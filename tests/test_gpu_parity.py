"""GPU parity: the HIP library against the FP64 oracle, called through the C ABI.

Bar (FP64 form): per row n, max_m |I_gpu(n,m) - I_oracle(n,m)| / max_m |I_oracle(n,m)|
<= 1e-10, for I^R and I^<.
"""
import numpy as np
import pytest

from gpu_common import host_inputs, oracle_rows, row, row_rel_err, say, to_dev
from kbe_inputs import make_config_inputs, hermitian_terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


_C1 = {}


def c1_data():
    if not _C1:
        cfg, G, S = make_config_inputs("c1")
        N, h, k = cfg["nt"], cfg["h"], cfg["k"]
        inp = host_inputs(G, S, N, h)
        say("oracle: c1 full sweep", N)
        IR, IL = oracle_rows(*inp, N, h, k)
        _C1.update(cfg=cfg, inp=inp, IR=IR, IL=IL)
    return _C1


def _sweep(obj, inp, N, h, norb):
    GR, GL, SR, SL = [to_dev(x) for x in inp]
    tot = N * (N + 1) // 2
    IR = torch.zeros((tot, norb, norb), dtype=torch.complex128, device="cuda")
    IL = torch.zeros_like(IR)
    obj.sweep(0, N, GR, GL, SR, SL, h, IR, IL)
    torch.cuda.synchronize()
    return IR.cpu().numpy(), IL.cpu().numpy()


def _check_rows(IRg, ILg, IR, IL, label):
    worst = 0.0
    for n in IR:
        eR = row_rel_err(row(IRg, n), IR[n])
        eL = row_rel_err(row(ILg, n), IL[n])
        worst = max(worst, eR, eL)
        assert eR <= TOL, (label, "R", n, eR)
        assert eL <= TOL, (label, "L", n, eL)
    say(label, "worst row relative error", worst)


def test_c1_full_sweep_hodlr(P):
    d = c1_data()
    cfg = d["cfg"]
    say("gpu: hodlr c1 sweep")
    H = P.Hodlr(cfg["nt"], 4, 1, k=cfg["k"], tol=cfg["tol"], panel=16, max_rank=16)
    IRg, ILg = _sweep(H, d["inp"], cfg["nt"], cfg["h"], 1)
    assert H.status() == 0
    _check_rows(IRg, ILg, d["IR"], d["IL"], "hodlr c1")


def test_c1_full_sweep_dense(P):
    d = c1_data()
    cfg = d["cfg"]
    say("gpu: dense c1 sweep")
    D = P.Dense(cfg["nt"], 1, k=cfg["k"])
    IRg, ILg = _sweep(D, d["inp"], cfg["nt"], cfg["h"], 1)
    _check_rows(IRg, ILg, d["IR"], d["IL"], "dense c1")


@pytest.mark.parametrize("norb,k,panel", [(2, 5, 8), (4, 3, 16), (4, 1, 4), (8, 5, 8), (16, 5, 8)])
def test_multiorbital_sweep(P, norb, k, panel):
    N, h, nlvl = 160, 0.03, 3   # leaves of 20 rows: ragged panels, several blocks per level
    G = hermitian_terms(11 + norb, 6, norb)
    S = hermitian_terms(21 + norb, 6, norb)
    inp = host_inputs(G, S, N, h)
    rows = list(range(0, 24)) + [39, 40, 41, 59, 60, 79, 80, 81, 100, 119, 120, 140, 159]
    say("oracle: multiorbital", norb, k, panel)
    IR, IL = oracle_rows(*inp, N, h, k, rows=rows)
    say("gpu: hodlr multiorbital", norb, k, panel)
    H = P.Hodlr(N, nlvl, norb, k=k, tol=1e-12, panel=panel, max_rank=16)
    IRg, ILg = _sweep(H, inp, N, h, norb)
    assert H.status() == 0
    _check_rows(IRg, ILg, IR, IL, f"hodlr norb={norb} k={k}")
    if norb <= 4:
        say("gpu: dense multiorbital", norb, k)
        D = P.Dense(N, norb, k=k)
        IRg, ILg = _sweep(D, inp, N, h, norb)
        _check_rows(IRg, ILg, IR, IL, f"dense norb={norb} k={k}")


@pytest.mark.parametrize("norb,rows", [(4, 256), (4, 1024), (1, 256), (16, 128)])
def test_tile_shapes(P, norb, rows):
    """Handles created with another projection chunk height (the autotuner's knob) give the
    oracle's rows (ragged chunks: blocks of 20 to 80 rows against 128..1024-row chunks)."""
    N, h, nlvl, k = 160, 0.03, 3, 5
    G = hermitian_terms(31 + norb, 6, norb)
    S = hermitian_terms(41 + norb, 6, norb)
    inp = host_inputs(G, S, N, h)
    rows_ = [0, 1, 19, 20, 39, 40, 79, 80, 100, 159]
    IR, IL = oracle_rows(*inp, N, h, k, rows=rows_)
    P.set_tile_shape(norb, rows)
    try:
        H = P.Hodlr(N, nlvl, norb, k=k, tol=1e-12, panel=8, max_rank=16)
    finally:
        P.set_tile_shape(norb, 0)
    assert H.tile_shape() == rows
    IRg, ILg = _sweep(H, inp, N, h, norb)
    assert H.status() == 0
    _check_rows(IRg, ILg, IR, IL, f"tile shape norb={norb} rows={rows}")


def test_ranks_above_sixteen(P):
    """Blocks whose rank exceeds 16 (a projection pass covers 16 ranks)."""
    from kbe_inputs import scalar_terms
    N, h, nlvl, k = 256, 0.15, 2, 5
    G, S = scalar_terms(31, 22), scalar_terms(32, 22)
    inp = host_inputs(G, S, N, h)
    rows = [0, 1, 5, 63, 64, 65, 127, 128, 129, 191, 192, 200, 255]
    say("oracle: ranks above 16")
    IR, IL = oracle_rows(*inp, N, h, k, rows=rows)
    say("gpu: hodlr ranks above 16")
    H = P.Hodlr(N, nlvl, 1, k=k, tol=1e-12, panel=8, max_rank=24)
    IRg, ILg = _sweep(H, inp, N, h, 1)
    assert H.status() == 0
    rmax = max(int(H.ranks(c).max()) for c in (0, 1))
    say("max rank", rmax)
    assert 16 < rmax <= 24
    _check_rows(IRg, ILg, IR, IL, "hodlr ranks above 16")


def test_ranks_above_sixteen_at_panel_sixteen(P):
    """Rank capacity 32 with 16-row panels: merges of width up to 48 (the wide merge kernels)."""
    from kbe_inputs import scalar_terms
    N, h, nlvl, k = 256, 0.15, 2, 5
    G, S = scalar_terms(33, 26), scalar_terms(34, 26)
    inp = host_inputs(G, S, N, h)
    rows = [0, 1, 5, 15, 16, 17, 63, 64, 65, 127, 128, 129, 191, 192, 200, 255]
    say("oracle: ranks above 16 at panel 16")
    IR, IL = oracle_rows(*inp, N, h, k, rows=rows)
    say("gpu: hodlr ranks above 16 at panel 16")
    H = P.Hodlr(N, nlvl, 1, k=k, tol=1e-12, panel=16, max_rank=32)
    IRg, ILg = _sweep(H, inp, N, h, 1)
    assert H.status() == 0
    rmax = max(int(H.ranks(c).max()) for c in (0, 1))
    say("max rank", rmax)
    assert 16 < rmax <= 32
    _check_rows(IRg, ILg, IR, IL, "hodlr ranks above 16, panel 16")


def test_separate_calls_match_fused(P):
    cfg, G, S = make_config_inputs("c2")
    N, h, norb = 96, 0.02, 4
    inp = host_inputs(G, S, N, h)
    GR, GL, SR, SL = [to_dev(x) for x in inp]
    say("gpu: separate vs fused calls")
    H1 = P.Hodlr(N, 3, norb, k=5, tol=1e-10, panel=8, max_rank=16)
    H2 = P.Hodlr(N, 3, norb, k=5, tol=1e-10, panel=8, max_rank=16)
    for n in range(N):
        a = n * (n + 1) // 2
        sl = slice(a, a + n + 1)
        for Hx in (H1, H2):
            Hx.append_row(P.RET, n, GR[sl])
            Hx.append_row(P.LES, n, GL[sl])
        oR = torch.zeros((n + 1, norb, norb), dtype=torch.complex128, device="cuda")
        oL = torch.zeros_like(oR)
        fR, fL = torch.zeros_like(oR), torch.zeros_like(oR)
        H1.history_R(n, SR[sl], h, oR)
        H1.history_lesser(n, SR[sl], SL[sl], h, oL)
        H2.history_step(n, SR[sl], SL[sl], h, fR, fL)
        assert torch.equal(oR, fR)
        assert torch.equal(oL, fL)


def test_order_and_range_errors(P):
    H = P.Hodlr(64, 2, 1, k=5, tol=1e-10, panel=8, max_rank=8)
    r = torch.zeros((2, 1, 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.HnessiError) as e:
        H.append_row(P.RET, 1, r)            # row 0 missing
    assert e.value.code == -2
    with pytest.raises(P.HnessiError) as e:
        H.history_R(0, r, 0.1, r)             # row 0 not appended
    assert e.value.code == -2
    with pytest.raises(P.HnessiError) as e:
        H.append_row(P.RET, 64, r)
    assert e.value.code == -3
    with pytest.raises(P.HnessiError) as e:
        P.Hodlr(64, 2, 3)                     # unsupported norb
    assert e.value.code == -1
    with pytest.raises(P.HnessiError):
        P.Hodlr(64, 2, 1, panel=16, max_rank=33)  # rank + panel beyond the widest SVD (48)
    with pytest.raises(P.HnessiError) as e:
        P.Hodlr(64, 2, 1, flags=4)            # unknown flag
    assert e.value.code == -1
    with pytest.raises(P.HnessiError) as e:
        P.HodlrBatch(0, 64, 2, 1)             # empty batch
    assert e.value.code == -1
    with pytest.raises(P.HnessiError) as e:
        H.history_R_adjoint(0, r, 0.1, r)     # row 0 not appended
    assert e.value.code == -2


def test_reconstruction_exact_rank(P):
    """Brute force: every stored (t1, t2) of both components is reproduced."""
    N, h, norb = 64, 0.05, 2
    G = hermitian_terms(31, 5, norb)
    S = hermitian_terms(32, 5, norb)
    inp = host_inputs(G, S, N, h)
    H = P.Hodlr(N, 3, norb, k=5, tol=1e-12, panel=8, max_rank=16)
    _sweep(H, inp, N, h, norb)
    say("gpu: reconstruction exact rank")
    for comp, pk in ((P.RET, inp[0]), (P.LES, inp[1])):
        for t1 in range(N):
            for t2 in range(t1 + 1):
                ref = pk[t1 * (t1 + 1) // 2 + t2]
                got = H.get(comp, t1, t2)
                assert np.abs(got - ref).max() <= 1e-11, (comp, t1, t2)
        rk = H.ranks(comp)
        assert rk.max() <= 5                     # five exponentials: rank <= 5 per pair
        assert rk.min() >= 1


def test_reconstruction_full_rank(P):
    """Random (full-rank) data: the merges must keep every singular value >= tol."""
    rng = np.random.default_rng(7)
    N, norb = 48, 1
    tot = N * (N + 1) // 2
    pk = (rng.standard_normal((tot, 1, 1)) + 1j * rng.standard_normal((tot, 1, 1)))
    H = P.Hodlr(N, 2, norb, k=2, tol=1e-13, panel=8, max_rank=24)
    d = to_dev(pk)
    for n in range(N):
        a = n * (n + 1) // 2
        H.append_row(P.RET, n, d[a:a + n + 1])
        H.append_row(P.LES, n, d[a:a + n + 1])
    assert H.status() == 0
    say("gpu: reconstruction full rank")
    for t1 in range(N):
        for t2 in range(t1 + 1):
            ref = pk[t1 * (t1 + 1) // 2 + t2]
            assert np.abs(H.get(P.RET, t1, t2) - ref).max() <= 1e-11, (t1, t2)
    blocks = H.blocks()
    rk = H.ranks(P.RET)
    for b, (lvl, r0, r1, c0, c1) in enumerate(blocks):
        assert rk[b, 0] == min(r1 - r0, c1 - c0)


_C2REF = {}


def c2_reference():
    """Oracle entries of the C2 sweep on the sampled rows and >= 64 columns per row (every
    level boundary 64 * 2^l and its neighbours included), computed once per session."""
    if not _C2REF:
        from gpu_common import boundary_columns, oracle_entries
        cfg, G, S = make_config_inputs("c2")
        N = cfg["nt"]
        rng = np.random.default_rng(2024)
        rows = sorted(set([0, 1, 4, 5, 6, 10, 11, 63, 64, 65, 127, 128, 511, 4095, 4096, N - 1]
                          + [int(x) for x in rng.integers(0, N, 8)]))
        cols = {n: boundary_columns(n, cfg["leaf"], 7, rng) for n in rows}
        say("oracle: c2 sampled entries", sum(len(c) for c in cols.values()))
        _C2REF.update(cfg=cfg, ref=oracle_entries(G, S, cfg["h"], cfg["k"], cols))
    return _C2REF


def _full_size_sweep(P, cls):
    """C2 (N_t=8192, norb=4) in the bench's configuration; returns (cfg, IR, IL, obj) with the
    sampled rows of the outputs on the host."""
    from kbe_inputs.packed import packed_torch
    d = c2_reference()
    cfg, G, S = make_config_inputs("c2")
    N, h = cfg["nt"], cfg["h"]
    dev = torch.device("cuda:0")
    GR, GL = packed_torch(G, "ret", N, h, dev), packed_torch(G, "les", N, h, dev)
    SR, SL = packed_torch(S, "ret", N, h, dev), packed_torch(S, "les", N, h, dev)
    IR, IL = torch.empty_like(GR), torch.empty_like(GR)
    obj = cls(N)
    say("gpu: full-size sweep")
    obj.sweep(0, N, GR, GL, SR, SL, h, IR, IL)
    torch.cuda.synchronize()
    del GR, GL, SR, SL
    gR = {n: row(IR, n).cpu().numpy() for n in d["ref"]}
    gL = {n: row(IL, n).cpu().numpy() for n in d["ref"]}
    return cfg, gR, gL, obj


def test_c2_full_size_hodlr_sampled(P):
    from gpu_common import check_entries
    cfg, gR, gL, H = _full_size_sweep(
        P, lambda N: P.Hodlr(N, 7, 4, k=5, tol=1e-10, panel=16, max_rank=16))
    assert H.status() == 0
    assert H.ranks(P.RET).max() <= 8 and H.ranks(P.LES).max() <= 8   # 8 exponentials per pair
    check_entries("hodlr c2", gR, gL, c2_reference()["ref"], TOL)


def test_c2_full_size_dense_sampled(P):
    from gpu_common import check_entries
    cfg, gR, gL, D = _full_size_sweep(P, lambda N: P.Dense(N, 4, k=5))
    check_entries("dense c2", gR, gL, c2_reference()["ref"], TOL)
