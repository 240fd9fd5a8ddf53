"""GPU tests of the one-block truncated SVD (hnessi_compress_block) against the
oracle's truncation reference, and of the allocator hook, called through the C ABI.

Bar (section "Hierarchical decomposition", absolute eps rule): the kept rank is the
number of singular values >= tol (a value within 1e-3 * tol of tol may go either way),
the spectral error |A - U S V^dagger|_2 is below tol, U and V are orthonormal, and the
reconstruction agrees with the oracle's TSVD within 2 * tol.
"""
import gc

import numpy as np
import pytest

from gpu_common import say, to_dev
from oracle.tsvd import singular_values, tsvd

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


def _check(P, A, tol, max_rank, label):
    sv = singular_values(A)
    U, S, V, r = P.compress_block(to_dev(A), tol, max_rank)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    n_eps = int(np.count_nonzero(sv >= tol))
    near = int(np.count_nonzero(np.abs(sv - tol) < 1e-3 * tol))
    assert abs(r - min(n_eps, max_rank)) <= near, (label, r, n_eps, near)
    if r:
        assert S[-1] >= tol and np.all(np.diff(S) <= 1e-14 * S[0]), (label, S)
        np.testing.assert_allclose(np.conj(U.T) @ U, np.eye(r), atol=1e-12)
        np.testing.assert_allclose(np.conj(V.T) @ V, np.eye(r), atol=1e-12)
        np.testing.assert_allclose(S, sv[:r], rtol=0, atol=1e-3 * tol + 1e-13 * sv[0])
    rec = (U * S) @ np.conj(V.T) if r else np.zeros_like(A)
    err = np.linalg.norm(A - rec, 2)
    if n_eps <= max_rank and near == 0:
        assert err < tol, (label, err, tol)
    Uo, so, Vo = tsvd(A, tol)
    diff = np.linalg.norm(rec - (Uo * so) @ np.conj(Vo.T), 2)
    if n_eps <= max_rank:
        assert diff < 2 * tol, (label, diff)
    say(label, "rank", r, "eps-rank", n_eps, "spectral error", err, "vs oracle", diff)
    return r, err


def test_compress_block_continuous_spectrum(P):
    """Singular values spread evenly (in log) from 2 to 1e-14 across tol = 1e-9."""
    rng = np.random.default_rng(3)
    s = np.geomspace(2.0, 1e-14, 20)
    A = _matrix(rng, 150, 700, s)
    tol = 1e-9
    gap = np.min(np.abs(s - tol)) / tol
    assert gap > 0.1     # the nearest values are 0.86 and 0.67 of tol away
    r, err = _check(P, A, tol, 24, "continuous spectrum")
    assert r == int(np.count_nonzero(s >= tol))
    assert err < tol


@pytest.mark.parametrize("m,n,seed", [(1, 5, 1), (7, 300, 2), (8, 64, 3), (9, 65, 4), (64, 64, 5),
                                      (200, 90, 6), (37, 129, 7), (300, 1000, 8)])
def test_compress_block_shapes_vs_oracle(P, m, n, seed):
    """Ragged row and column counts (partial merge panels, partial 64-row chunks, rows > cols)."""
    rng = np.random.default_rng(seed)
    k = min(m, n, 30)
    s = np.geomspace(5.0, 1e-13, k) * rng.uniform(0.7, 1.3, k)
    s = np.sort(s)[::-1]
    A = _matrix(rng, m, n, s)
    _check(P, A, 1e-8, 40, f"shape {m}x{n}")


def test_compress_block_exact_rank_and_zero(P):
    rng = np.random.default_rng(11)
    A = _matrix(rng, 100, 333, np.array([3.0, 1.0, 0.5, 1e-3]))
    r, err = _check(P, A, 1e-10, 16, "exact rank 4")
    assert r == 4 and err < 1e-12
    Z = np.zeros((20, 50), dtype=np.complex128)
    U, S, V, r = P.compress_block(to_dev(Z), 1e-10, 8)
    assert r == 0


def test_compress_block_rank_cap(P):
    """More values above tol than max_rank: the largest max_rank are kept."""
    rng = np.random.default_rng(12)
    s = np.geomspace(1.0, 1e-3, 12)
    A = _matrix(rng, 60, 200, s)
    U, S, V, r = P.compress_block(to_dev(A), 1e-6, 5)
    assert r == 5
    np.testing.assert_allclose(S.cpu().numpy(), s[:5], rtol=1e-10)


def test_compress_block_nonfinite_reported(P):
    """A NaN entry: the truncation reports HNESSI_E_VALUE through rank_out."""
    rng = np.random.default_rng(13)
    A = _matrix(rng, 40, 120, np.array([1.0, 0.1]))
    A[17, 33] = np.nan
    with pytest.raises(P.HnessiError) as e:
        P.compress_block(to_dev(A), 1e-10, 8)
    assert e.value.code == -7
    # the library stays usable
    _check(P, _matrix(rng, 40, 120, np.array([1.0, 0.1])), 1e-10, 8, "after non-finite")


def test_compress_block_argument_errors(P):
    import ctypes as C
    L = P.lib()
    A = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    U = torch.zeros((8, 4), dtype=torch.complex128, device="cuda")
    S = torch.zeros(8, dtype=torch.float64, device="cuda")
    rk = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.hnessi_compress_block(None, 4, 4, 4, 1e-10, 8, p(U), p(S), p(U), p(rk), st) == -1
    assert L.hnessi_compress_block(p(A), 4, 4, 3, 1e-10, 8, p(U), p(S), p(U), p(rk), st) == -1   # lda < cols
    assert L.hnessi_compress_block(p(A), 4, 4, 4, 0.0, 8, p(U), p(S), p(U), p(rk), st) == -1
    assert L.hnessi_compress_block(p(A), 4, 4, 4, 1e-10, 41, p(U), p(S), p(U), p(rk), st) == -1
    assert L.hnessi_compress_block(p(A), 0, 4, 4, 1e-10, 8, p(U), p(S), p(U), p(rk), st) == -1


def test_allocator_hook_failure_gives_nomem(P):
    """An allocator that returns NULL: creation and compress_block fail with HNESSI_E_NOMEM."""
    calls = []

    def bad_alloc(nbytes, stream):
        calls.append(nbytes)
        return 0

    def free(ptr, stream):
        raise AssertionError("nothing was allocated")

    P.set_allocator(bad_alloc, free)
    try:
        with pytest.raises(P.HnessiError) as e:
            P.Hodlr(128, 2, 2, k=5, tol=1e-10, panel=8, max_rank=8)
        assert e.value.code == -4
        with pytest.raises(P.HnessiError) as e:
            P.Dense(64, 1, k=5)
        assert e.value.code == -4
        A = torch.ones((8, 16), dtype=torch.complex128, device="cuda")
        with pytest.raises(P.HnessiError) as e:
            P.compress_block(A, 1e-10, 4)
        assert e.value.code == -4
        assert calls
    finally:
        P.set_allocator()


def test_allocator_hook_partial_failure_releases(P):
    """The n-th allocation fails: everything allocated before it is returned through the hook."""
    live, count = {}, [0]

    def alloc(nbytes, stream):
        count[0] += 1
        if count[0] == 9:
            return 0
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, stream):
        del live[ptr]

    P.set_allocator(alloc, free)
    try:
        with pytest.raises(P.HnessiError) as e:
            P.Hodlr(128, 2, 2, k=5, tol=1e-10, panel=8, max_rank=8)
        assert e.value.code == -4
        assert not live, "allocations leaked"
    finally:
        P.set_allocator()


def test_torch_caching_allocator_serves_the_handle(P):
    """A sweep with the handle's memory from PyTorch's caching allocator equals the default."""
    from gpu_common import host_inputs
    from kbe_inputs import hermitian_terms
    N, h, norb = 96, 0.03, 2
    G, S = hermitian_terms(91, 5, norb), hermitian_terms(92, 5, norb)
    GR, GL, SR, SL = [to_dev(x) for x in host_inputs(G, S, N, h)]
    outs = []
    for use_torch in (False, True):
        if use_torch:
            P.use_torch_allocator()
        try:
            # objects of earlier tests that the collector frees later would shift the count
            gc.collect()
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            H = P.Hodlr(N, 3, norb, k=5, tol=1e-12, panel=8, max_rank=12)
            held = torch.cuda.memory_allocated() - before
            IR, IL = torch.zeros_like(GR), torch.zeros_like(GR)
            H.sweep(0, N, GR, GL, SR, SL, h, IR, IL)
            assert H.status() == 0
            if use_torch:
                assert held >= H.nbytes()          # served by torch's allocator
            H.close()
            if use_torch:   # and returned to it: nothing of the handle is still held
                assert torch.cuda.memory_allocated() - before <= 0
            outs.append((IR.cpu(), IL.cpu()))
        finally:
            P.set_allocator()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
