"""GPU regression tests of the handle's failure reporting, through the C ABI.

Non-finite data met by a panel merge's truncation must be reported as
HNESSI_E_VALUE by hnessi_hodlr_status (the merge drops those directions and every
index stays in range), and the handle must be usable again after a reset.
"""
import numpy as np
import pytest

from gpu_common import host_inputs, oracle_rows, row, row_rel_err, say, to_dev
from kbe_inputs import hermitian_terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def test_nan_row_sets_e_value_and_reset_recovers(P):
    N, h, norb, k = 96, 0.03, 2, 5
    G, S = hermitian_terms(71, 5, norb), hermitian_terms(72, 5, norb)
    inp = host_inputs(G, S, N, h)
    GR, GL, SR, SL = [to_dev(x) for x in inp]
    H = P.Hodlr(N, 3, norb, k=k, tol=1e-12, panel=8, max_rank=12)
    bad = GR.clone()
    a = 40 * 41 // 2
    bad[a + 3, 0, 1] = complex(float("nan"), 0.0)     # row 40, column 3: a block column
    say("gpu: NaN row merged")
    for n in range(N):
        H.append_row(P.RET, n, row(bad, n))
        H.append_row(P.LES, n, row(GL, n))
    with pytest.raises(P.HnessiError) as e:
        H.status()
    assert e.value.code == -7
    say("gpu: sweep after reset")
    H.reset()
    IR, IL = torch.zeros_like(GR), torch.zeros_like(GR)
    H.sweep(0, N, GR, GL, SR, SL, h, IR, IL)
    assert H.status() == 0
    rows = [0, 5, 39, 40, 63, 64, 95]
    ref_R, ref_L = oracle_rows(*inp, N, h, k, rows=rows)
    IRh, ILh = IR.cpu().numpy(), IL.cpu().numpy()
    for n in rows:
        assert row_rel_err(row(IRh, n), ref_R[n]) <= 1e-10
        assert row_rel_err(row(ILh, n), ref_L[n]) <= 1e-10


def test_rank_capacity_reported(P):
    """Full-rank data with a small rank capacity: HNESSI_E_RANK, indices stay in range."""
    rng = np.random.default_rng(5)
    N = 64
    tot = N * (N + 1) // 2
    pk = to_dev(rng.standard_normal((tot, 1, 1)) + 1j * rng.standard_normal((tot, 1, 1)))
    H = P.Hodlr(N, 2, 1, k=3, tol=1e-12, panel=8, max_rank=4)
    for n in range(N):
        H.append_row(P.RET, n, row(pk, n))
        H.append_row(P.LES, n, row(pk, n))
    with pytest.raises(P.HnessiError) as e:
        H.status()
    assert e.value.code == -6
    assert H.ranks(P.RET).max() <= 4
