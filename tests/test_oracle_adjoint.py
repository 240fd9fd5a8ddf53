"""Pins of the adjoint oracle: the adjoint identity against the (separately
pinned) forward oracle, and central finite differences of a weighted
|I^R|^2 loss in the convention dL/dRe + i dL/dIm."""
import numpy as np

from oracle.adjoint import history_R_adjoint_row
from oracle.history import ArrayOperands, history_R_row


def _random_ops(rng, N, norb):
    def c(*shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return ArrayOperands(c(N, N, norb, norb), c(N, N, norb, norb), c(N, N, norb, norb), c(N, N, norb, norb))


def _inner(a, b):
    return float(np.real(np.sum(np.conj(a) * b)))


def test_adjoint_identity_against_forward():
    rng = np.random.default_rng(5)
    h = 0.1
    for norb in (1, 3):
        for k in (1, 3, 5):
            for n in (0, 1, 2, 4, 7, 12):
                ops = _random_ops(rng, 13, norb)
                ibar = rng.standard_normal((n + 1, norb, norb)) + 1j * rng.standard_normal((n + 1, norb, norb))
                fwd = history_R_row(ops, n, h, k)
                adj = history_R_adjoint_row(ops, n, ibar, h, k)
                # perturb Sigma^R(n, .) by d: I changes by A(d); <ibar, A d> = <A^T ibar, d>
                d = rng.standard_normal((n + 1, norb, norb)) + 1j * rng.standard_normal((n + 1, norb, norb))
                ops.SR_[n, :n + 1] += d
                Ad = history_R_row(ops, n, h, k) - fwd
                lhs, rhs = _inner(ibar, Ad), _inner(adj, d)
                assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs)), (norb, k, n, lhs, rhs)


def test_adjoint_matches_finite_differences_of_loss():
    rng = np.random.default_rng(6)
    N, norb, h, k, n = 10, 2, 0.2, 5, 9
    ops = _random_ops(rng, N, norb)
    c = rng.uniform(0.1, 1.0, n + 1)

    def loss():
        I = history_R_row(ops, n, h, k)
        return float(np.sum(c[:, None, None] * np.abs(I) ** 2))

    I = history_R_row(ops, n, h, k)
    g = history_R_adjoint_row(ops, n, 2.0 * c[:, None, None] * I, h, k)
    eps = 1e-6
    for (j, a, b) in [(0, 0, 0), (3, 1, 0), (8, 0, 1), (9, 1, 1)]:
        base = ops.SR_[n, j, a, b]
        ops.SR_[n, j, a, b] = base + eps
        lp = loss()
        ops.SR_[n, j, a, b] = base - eps
        lm = loss()
        ops.SR_[n, j, a, b] = base + 1j * eps
        ip = loss()
        ops.SR_[n, j, a, b] = base - 1j * eps
        im = loss()
        ops.SR_[n, j, a, b] = base
        fd = (lp - lm) / (2 * eps) + 1j * (ip - im) / (2 * eps)
        assert abs(fd - g[j, a, b]) <= 1e-6 * max(1.0, abs(fd)), (j, a, b, fd, g[j, a, b])


def test_adjoint_of_last_column_is_zero():
    """I^R(n, n) = 0 for every Sigma, so a cotangent on m = n alone has a zero adjoint."""
    rng = np.random.default_rng(7)
    ops = _random_ops(rng, 8, 2)
    n = 7
    ibar = np.zeros((n + 1, 2, 2), dtype=np.complex128)
    ibar[n] = rng.standard_normal((2, 2))
    assert np.abs(history_R_adjoint_row(ops, n, ibar, 0.1, 5)).max() == 0.0
