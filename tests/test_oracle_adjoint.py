"""Pins of the adjoint oracle: the adjoint identity against the (separately
pinned) forward oracle, and central finite differences of a weighted
|I^R|^2 loss in the convention dL/dRe + i dL/dIm."""
import numpy as np

from oracle.adjoint import factor_gradients, history_R_adjoint_row, history_R_G_gradient
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


def test_G_gradient_adjoint_identity_over_a_sweep():
    """<Ibar, I(G + dG) - I(G)> = <Gbar, dG> summed over all steps of a sweep, with the
    forward oracle recomputing every row (the sum is linear in G^R)."""
    rng = np.random.default_rng(11)
    N, h = 11, 0.1
    for norb in (1, 2):
        for k in (1, 3, 5):
            ops = _random_ops(rng, N, norb)
            ibar = [rng.standard_normal((n + 1, norb, norb)) + 1j * rng.standard_normal((n + 1, norb, norb))
                    for n in range(N)]
            fwd = [history_R_row(ops, n, h, k) for n in range(N)]
            d = rng.standard_normal((N, N, norb, norb)) + 1j * rng.standard_normal((N, N, norb, norb))
            d *= np.tril(np.ones((N, N)))[:, :, None, None]   # stored triangle j >= m only
            ops.LR_ += d
            lhs = sum(_inner(ibar[n], history_R_row(ops, n, h, k) - fwd[n]) for n in range(N))
            gb = history_R_G_gradient(ops, lambda ns, m: np.stack([ibar[n][m] for n in ns]), N, h, k, range(N),
                              range(N))
            rhs = _inner(gb, d)
            assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs)), (norb, k, lhs, rhs)


def test_G_gradient_matches_finite_differences_of_loss():
    """Central differences of L = sum_n sum_m c_m |I^R(n,m)|^2 with respect to stored
    entries of G^R, against Gbar for Ibar = 2 c I."""
    rng = np.random.default_rng(12)
    N, norb, h, k = 9, 2, 0.2, 3
    ops = _random_ops(rng, N, norb)
    c = rng.uniform(0.1, 1.0, N)

    def loss():
        return float(sum(np.sum(c[:n + 1, None, None] * np.abs(history_R_row(ops, n, h, k)) ** 2)
                         for n in range(N)))

    ibar = [2.0 * c[:n + 1, None, None] * history_R_row(ops, n, h, k) for n in range(N)]
    gb = history_R_G_gradient(ops, lambda ns, m: np.stack([ibar[n][m] for n in ns]), N, h, k, range(N),
                              range(N))
    eps = 1e-6
    for (j, m, a, b) in [(0, 0, 0, 0), (4, 1, 1, 0), (7, 7, 0, 1), (8, 2, 1, 1), (5, 4, 0, 0)]:
        base = ops.LR_[j, m, a, b]
        vals = []
        for dd in (eps, -eps, 1j * eps, -1j * eps):
            ops.LR_[j, m, a, b] = base + dd
            vals.append(loss())
        ops.LR_[j, m, a, b] = base
        fd = (vals[0] - vals[1]) / (2 * eps) + 1j * (vals[2] - vals[3]) / (2 * eps)
        assert abs(fd - gb[j, m, a, b]) <= 1e-6 * max(1.0, abs(fd)), (j, m, fd, gb[j, m, a, b])


def test_factor_gradients_match_finite_differences():
    """dU, dS, dV of L(U S V^H) = <Gbar0, U S V^H> + |U S V^H|^2 / 2 by central differences
    (a loss whose entry gradient is Gbar0 + G, so the chain rule is checked on its own)."""
    rng = np.random.default_rng(13)
    R, Cn, r = 7, 5, 3
    U = rng.standard_normal((R, r)) + 1j * rng.standard_normal((R, r))
    V = rng.standard_normal((Cn, r)) + 1j * rng.standard_normal((Cn, r))
    S = rng.uniform(0.5, 2.0, r)
    Gb0 = rng.standard_normal((R, Cn)) + 1j * rng.standard_normal((R, Cn))

    def loss(U, S, V):
        G = U @ np.diag(S) @ np.conj(V.T)
        return _inner(Gb0, G) + 0.5 * float(np.sum(np.abs(G) ** 2))

    G = U @ np.diag(S) @ np.conj(V.T)
    dU, dS, dV = factor_gradients(Gb0 + G, U, S, V)
    eps = 1e-6

    def fd_complex(f):
        vals = [f(dd) for dd in (eps, -eps, 1j * eps, -1j * eps)]
        return (vals[0] - vals[1]) / (2 * eps) + 1j * (vals[2] - vals[3]) / (2 * eps)

    for (i, q) in [(0, 0), (3, 2), (6, 1)]:
        def fU(dd):
            Up = U.copy()
            Up[i, q] += dd
            return loss(Up, S, V)
        fd = fd_complex(fU)
        assert abs(fd - dU[i, q]) <= 1e-6 * max(1.0, abs(fd)), (i, q, fd, dU[i, q])
    for (i, q) in [(0, 1), (4, 2)]:
        def fV(dd):
            Vp = V.copy()
            Vp[i, q] += dd
            return loss(U, S, Vp)
        fd = fd_complex(fV)
        assert abs(fd - dV[i, q]) <= 1e-6 * max(1.0, abs(fd)), (i, q, fd, dV[i, q])
    for q in range(r):
        Sp, Sm = S.copy(), S.copy()
        Sp[q] += eps
        Sm[q] -= eps
        fd = (loss(U, Sp, V) - loss(U, Sm, V)) / (2 * eps)
        assert abs(fd - dS[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, dS[q])
