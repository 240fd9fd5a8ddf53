"""The entry point that allocates nothing (hnessi_compress_block_noalloc), called
through the C ABI, against hnessi_compress_block on the same inputs: two calls in
a row, the second with a smaller block, must give the same rank, singular values
and factors, and both must pass the oracle's truncation check."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import say, to_dev
from oracle.tsvd import singular_values

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _matrix(rng, m, n, s):
    k = len(s)
    U0 = np.linalg.qr(rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k)))[0]
    V0 = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))[0]
    return (U0 * s) @ np.conj(V0.T)


def _call(P, name, A, tol, max_rank):
    rows, cols = A.shape
    U = torch.full((max_rank, rows), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    V = torch.full((max_rank, cols), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    S = torch.full((max_rank,), 7.0, dtype=torch.float64, device="cuda")
    rk = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(P.lib(), name)(p(A), rows, cols, cols, tol, max_rank, p(U), p(S), p(V), p(rk), st)
    assert rc == 0, P.lib().hnessi_last_error()
    torch.cuda.synchronize()
    r = int(rk.item())
    return U[:r].cpu().numpy().T, S[:r].cpu().numpy(), V[:r].cpu().numpy().T, r


def test_noalloc_matches_allocating_entry_point(P):
    rng = np.random.default_rng(77)
    tol = 1e-9
    cases = [(300, 1100, np.geomspace(3.0, 1e-13, 24)), (45, 130, np.geomspace(1.0, 1e-12, 16))]
    for m, n, s in cases:
        A = to_dev(_matrix(rng, m, n, s))
        say("noalloc vs allocating", m, n)
        Ua, Sa, Va, ra = _call(P, "hnessi_compress_block", A, tol, 32)
        Ub, Sb, Vb, rb = _call(P, "hnessi_compress_block_noalloc", A, tol, 32)
        assert ra == rb == int(np.count_nonzero(s >= tol))
        assert np.array_equal(Sa, Sb) and np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
        Ah = A.cpu().numpy()
        err = np.linalg.norm(Ah - (Ub * Sb) @ np.conj(Vb.T), 2)
        assert err < tol, err
        np.testing.assert_allclose(Sb, singular_values(Ah)[:rb], rtol=0, atol=1e-3 * tol + 1e-13 * s[0])


def test_noalloc_rejects_oversized_blocks(P):
    A = torch.zeros((4097, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.HnessiError) as e:
        P.compress_block(A, 1e-10, 4, noalloc=True)
    assert e.value.code == -1
