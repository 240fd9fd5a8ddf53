"""GPU parity of the batched form (k-point lattice, one object per momentum k)
against the FP64 oracle, called through the C ABI.

Bar: as for the single-object form, per row (or sampled entry) relative error
<= 1e-10 for I^R and I^<, for every object; a batched object's results equal
those of the same object run alone, bit for bit (same kernels, the object is
the grid's second dimension).
"""
import numpy as np
import pytest

from gpu_common import host_inputs, oracle_rows, row, row_rel_err, say, to_dev
from kbe_inputs import make_config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _zeros(n):
    return torch.zeros((n, 1, 1), dtype=torch.complex128, device="cuda")


def test_batched_matches_oracle_and_single_objects(P):
    cfg, G, S = make_config_inputs("c3")
    sel = [0, 33, 170, 341, 512, 700, 900, 1023]      # momenta spread over the zone
    N, h, k, nlvl = 192, cfg["h"], cfg["k"], 2          # leaves of 48 rows: three panels each
    tot = N * (N + 1) // 2
    inps = [host_inputs(G[i], S[i], N, h) for i in sel]
    stacked = [to_dev(np.concatenate([inp[j] for inp in inps])) for j in range(4)]
    IR, IL = _zeros(len(sel) * tot), _zeros(len(sel) * tot)
    say("gpu: batched sweep", len(sel), N)
    B = P.HodlrBatch(len(sel), N, nlvl, 1, k=k, tol=cfg["tol"], panel=16, max_rank=16)
    B.sweep(0, N, *stacked, h, IR, IL)
    torch.cuda.synchronize()
    assert B.status() == 0
    ranks = B.ranks(P.RET)
    assert ranks.shape == (len(sel), B.blocks().shape[0], 1)
    IRh, ILh = IR.cpu().numpy().reshape(len(sel), tot, 1, 1), IL.cpu().numpy().reshape(len(sel), tot, 1, 1)
    rows = [0, 1, 2, 5, 6, 47, 48, 49, 95, 96, 100, 143, 144, 191]
    worst = 0.0
    for o, inp in enumerate(inps):
        oR, oL = oracle_rows(*inp, N, h, k, rows=rows)
        for n in rows:
            eR, eL = row_rel_err(row(IRh[o], n), oR[n]), row_rel_err(row(ILh[o], n), oL[n])
            worst = max(worst, eR, eL)
            assert eR <= TOL and eL <= TOL, (o, n, eR, eL)
    say("batched worst row relative error", worst)
    # the same objects alone
    for o in (0, 5):
        H = P.Hodlr(N, nlvl, 1, k=k, tol=cfg["tol"], panel=16, max_rank=16)
        sR, sL = _zeros(tot), _zeros(tot)
        H.sweep(0, N, *[to_dev(x) for x in inps[o]], h, sR, sL)
        torch.cuda.synchronize()
        assert np.array_equal(sR.cpu().numpy().reshape(tot, 1, 1), IRh[o]), o
        assert np.array_equal(sL.cpu().numpy().reshape(tot, 1, 1), ILh[o]), o
        assert np.array_equal(H.ranks(P.RET), ranks[o])


def test_batched_fp32_factors(P):
    """Batched objects with complex-float factor mirrors: within 1e-5 of the oracle and within
    1e-5 of the FP64-factor batch."""
    cfg, G, S = make_config_inputs("c3")
    sel = [3, 500, 1000]
    N, h, k, nlvl = 128, cfg["h"], cfg["k"], 1
    tot = N * (N + 1) // 2
    inps = [host_inputs(G[i], S[i], N, h) for i in sel]
    stacked = [to_dev(np.concatenate([inp[j] for inp in inps])) for j in range(4)]
    out = {}
    for flags in (0, P.FLAG_FP32_FACTORS):
        IR, IL = _zeros(len(sel) * tot), _zeros(len(sel) * tot)
        B = P.HodlrBatch(len(sel), N, nlvl, 1, k=k, tol=1e-8, panel=16, max_rank=16, flags=flags)
        B.sweep(0, N, *stacked, h, IR, IL)
        torch.cuda.synchronize()
        assert B.status() == 0
        out[flags] = (IR.cpu().numpy().reshape(len(sel), tot, 1, 1), IL.cpu().numpy().reshape(len(sel), tot, 1, 1))
    rows = [0, 1, 63, 64, 65, 100, 127]
    worst = 0.0
    for o, inp in enumerate(inps):
        oR, oL = oracle_rows(*inp, N, h, k, rows=rows)
        for n in rows:
            eR = row_rel_err(row(out[P.FLAG_FP32_FACTORS][0][o], n), oR[n])
            eL = row_rel_err(row(out[P.FLAG_FP32_FACTORS][1][o], n), oL[n])
            worst = max(worst, eR, eL)
            assert eR <= 1e-5 and eL <= 1e-5, (o, n, eR, eL)
    say("batched fp32 worst row relative error", worst)


def test_batched_argument_errors(P):
    B = P.HodlrBatch(3, 128, 2, 1, k=5, tol=1e-10, panel=16, max_rank=16)
    row = _zeros(3 * 128)
    with pytest.raises(P.HnessiError):       # single-object call on a batch
        P.Hodlr.append_row(B, P.RET, 0, row)
    with pytest.raises(P.HnessiError):       # stride smaller than one row
        B.append_row(P.RET, 0, row, 0)
    with pytest.raises(P.HnessiError):       # out of order
        B.append_row(P.RET, 1, row, 128)
    B.append_row(P.RET, 0, row, 128)


def _graph_stream():
    """Graph sweeps are captured from a stream other than the NULL stream."""
    return torch.cuda.Stream()


GRAPH_SKIP = ("graph sweeps passed this test and the 128-momentum C3 test once, but a graph sweep run "
              "inside the lattice benchmark stopped producing output for 180 s (twice, at 1024 and at 128 "
              "momenta) without a cause found; kept off the GPU until one is")


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_graph_sweep_matches_launches(P):
    """A sweep replayed as graphs (one window per panel, merges forked and joined inside)
    gives the launch-by-launch results bit for bit, twice in a row with eager work and
    synchronizations between the two, and from a partial sweep continued in graph mode."""
    cfg, G, S = make_config_inputs("c3")
    sel = [1, 200, 640, 1000]
    N, h, k, nlvl = 192, cfg["h"], cfg["k"], 2
    tot = N * (N + 1) // 2
    inps = [host_inputs(G[i], S[i], N, h) for i in sel]
    stacked = [to_dev(np.concatenate([inp[j] for inp in inps])) for j in range(4)]
    ref = []
    Be = P.HodlrBatch(len(sel), N, nlvl, 1, k=k, tol=cfg["tol"], panel=16, max_rank=16)
    IR, IL = _zeros(len(sel) * tot), _zeros(len(sel) * tot)
    Be.sweep(0, N, *stacked, h, IR, IL)
    torch.cuda.synchronize()
    ref = (IR.cpu().numpy(), IL.cpu().numpy(), Be.ranks(P.RET))
    s = _graph_stream()
    with torch.cuda.stream(s):
        Bg = P.HodlrBatch(len(sel), N, nlvl, 1, k=k, tol=cfg["tol"], panel=16, max_rank=16, flags=P.FLAG_GRAPHS)
        for rep in range(2):
            IRg, ILg = _zeros(len(sel) * tot), _zeros(len(sel) * tot)
            Bg.reset()
            if rep == 0:
                Bg.sweep(0, N, *stacked, h, IRg, ILg)
            else:   # the first rows launch by launch through the single-step calls, then graphs
                for n in range(40):
                    off = n * (n + 1) // 2
                    Bg.append_row(P.RET, n, stacked[0][off:], tot)
                    Bg.append_row(P.LES, n, stacked[1][off:], tot)
                    Bg.history_step(n, stacked[2][off:], stacked[3][off:], tot, h, IRg[off:], ILg[off:], tot)
                Bg.sweep(40, N, *stacked, h, IRg, ILg)
            s.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum().item()   # eager work between replays
            assert np.isfinite(junk)
            assert np.array_equal(IRg.cpu().numpy(), ref[0]), rep
            assert np.array_equal(ILg.cpu().numpy(), ref[1]), rep
            assert np.array_equal(Bg.ranks(P.RET), ref[2]), rep
        assert Bg.status() == 0
    windows, inst = Bg.graph_stats()
    say("graph windows", windows, "instantiations", inst)
    assert windows >= 2 * (N // 16) - 2 and inst < windows


@pytest.mark.parametrize("graphs", [False, pytest.param(True, marks=pytest.mark.skip(reason=GRAPH_SKIP))])
def test_c3_full_size_sampled(P, graphs):
    """C3 geometry (N_t = 2048, leaf 64, norb = 1) on 128 of the 1024 momenta (every eighth),
    launch by launch or swept as graphs; sampled entries against the oracle, scaled by the
    oracle's largest sampled entry of the row."""
    from kbe_inputs.packed import packed_torch
    from gpu_common import oracle_entries_multi
    cfg, G, S = make_config_inputs("c3")
    N, h, k = cfg["nt"], cfg["h"], cfg["k"]
    nlvl = int(round(np.log2(N // cfg["leaf"])))
    sel = list(range(0, 1024, 8))
    tot = N * (N + 1) // 2
    dev = torch.device("cuda:0")
    arrs = []
    for src, kind in ((G, "ret"), (G, "les"), (S, "ret"), (S, "les")):
        a = torch.empty((len(sel) * tot, 1, 1), dtype=torch.complex128, device=dev)
        for o, i in enumerate(sel):
            a[o * tot:(o + 1) * tot] = packed_torch(src[i], kind, N, h, dev)
        arrs.append(a)
    IR, IL = torch.empty_like(arrs[0]), torch.empty_like(arrs[0])
    torch.cuda.synchronize()
    s = _graph_stream()
    with torch.cuda.stream(s):
        B = P.HodlrBatch(len(sel), N, nlvl, 1, k=k, tol=cfg["tol"], panel=16, max_rank=16,
                         flags=P.FLAG_GRAPHS if graphs else 0)
        say("gpu: c3 batched sweep", len(sel), N, "graphs" if graphs else "launches")
        B.sweep(0, N, *arrs, h, IR, IL)
        s.synchronize()
        assert B.status() == 0
    rng = np.random.default_rng(77)
    jobs, where = [], []
    for o, i in enumerate(sel):
        for n in sorted(set([63, 1024, N - 1] + list(rng.integers(0, N, 1)))):
            ms = sorted(set(x for x in [0, 1, 64, n - 5, n] + list(rng.integers(0, n + 1, 2)) if 0 <= x <= n))
            jobs.append((G[i], S[i], h, k, int(n), ms))
            where.append((o, int(n), ms))
    say("oracle:", len(jobs), "rows of sampled entries")
    res = oracle_entries_multi(jobs)
    worst = 0.0
    for (o, n, ms), vals in zip(where, res):
        a = o * tot + n * (n + 1) // 2
        gR, gL = IR[a:a + n + 1].cpu().numpy(), IL[a:a + n + 1].cpu().numpy()
        oR, oL = np.stack([v[0] for v in vals]), np.stack([v[1] for v in vals])
        sR, sL = np.abs(oR).max(), np.abs(oL).max()
        eR = np.abs(gR[ms] - oR).max() / max(sR, 1e-300)
        eL = np.abs(gL[ms] - oL).max() / max(sL, 1e-300)
        worst = max(worst, eR, eL)
        assert eR <= TOL and eL <= TOL, (sel[o], n, eR, eL)
    say("c3 worst sampled relative error (128 momenta)", worst)
