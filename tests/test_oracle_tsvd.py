"""Pins for the truncation reference: matrices built with known singular values."""
import numpy as np

from oracle.tsvd import eps_rank, tsvd


def _orth(rng, m, r):
    z = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    return np.linalg.qr(z)[0]


def test_tsvd_known_spectrum():
    rng = np.random.default_rng(1)
    s = np.array([3.0, 1.0, 1e-3, 2e-10, 1.5e-10, 5e-11, 1e-14])
    U0, V0 = _orth(rng, 40, 7), _orth(rng, 30, 7)
    B = (U0 * s) @ np.conj(V0.T)
    U, ss, V = tsvd(B, 1e-10)
    assert len(ss) == 5                       # sigma >= eps kept
    np.testing.assert_allclose(ss, s[:5], rtol=1e-6, atol=1e-15)
    err = np.linalg.norm(B - (U * ss) @ np.conj(V.T), 2)
    assert abs(err - 5e-11) < 1e-14          # spectral error = first dropped value
    np.testing.assert_allclose(np.conj(U.T) @ U, np.eye(5), atol=1e-12)
    np.testing.assert_allclose(np.conj(V.T) @ V, np.eye(5), atol=1e-12)


def test_eps_rank_of_exponential_kernel():
    # e^{-(i w + g)(t - t')} restricted to t >= t' blocks is rank one per term
    t = np.arange(64, 128) * 0.01
    tp = np.arange(0, 64) * 0.01
    rng = np.random.default_rng(2)
    w, g = rng.uniform(-4, 4, 5), rng.uniform(0.02, 0.2, 5)
    B = sum(np.exp(-(1j * w[p] + g[p]) * (t[:, None] - tp[None, :])) for p in range(5))
    assert eps_rank(B, 1e-10) <= 5
    assert eps_rank(B[:, :1], 1e-10) == 1
