"""Pins of the FP64 step-solve oracle against closed forms of the retarded equation:
Sigma = 0 with a constant Hermitian eps (G = -i exp(-i eps (t-t'))), and eps = 0 with a
constant scalar Sigma = lam (i G' = lam int_0^tau G, G(0) = -i, so G = -i cosh(kappa tau),
kappa^2 = -i lam); the first k rows are the exact ones (the bootstrap is not part of the
step), and the error must fall at the scheme's order under step halving: k for the free
propagator, min(k, 4) with memory (the near-diagonal start integrates intervals shorter
than k with the closed Newton-Cotes rule of their own length)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle.step_solve import solve


def _free_case(N, h, norb, k, seed=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))
    eps = 0.5 * (A + A.conj().T)
    G = np.zeros((N, N, norb, norb), dtype=np.complex128)
    for n in range(N):
        for m in range(n + 1):
            G[n, m] = -1j * expm(-1j * eps * (n - m) * h)
    return np.broadcast_to(eps, (N, norb, norb)).copy(), np.zeros((N, N, norb, norb), dtype=np.complex128), G


def _memory_case(N, h, lam):
    kap = np.sqrt(-1j * lam)
    G = np.zeros((N, N, 1, 1), dtype=np.complex128)
    S = np.zeros((N, N, 1, 1), dtype=np.complex128)
    for n in range(N):
        for m in range(n + 1):
            G[n, m] = -1j * np.cosh(kap * (n - m) * h)
            S[n, m] = lam
    return np.zeros((N, 1, 1), dtype=np.complex128), S, G


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_free_propagator_order(k):
    T, norb = 1.6, 2
    errs = []
    for N in (65, 129):
        h = T / (N - 1)
        eps, S, G = _free_case(N, h, norb, k)
        Gs = solve(S, eps, G, h, k, N)
        errs.append(max(np.abs(Gs[n, :n + 1] - G[n, :n + 1]).max() for n in range(N)))
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-2 and order > k - 0.3, (k, errs, order)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_constant_memory_kernel_order(k):
    T, lam = 1.6, 0.8
    errs = []
    for N in (65, 129):
        h = T / (N - 1)
        eps, S, G = _memory_case(N, h, lam)
        Gs = solve(S, eps, G, h, k, N)
        errs.append(max(np.abs(Gs[n, :n + 1] - G[n, :n + 1]).max() for n in range(N)))
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-3 and order > min(k, 4) - 0.3, (k, errs, order)


def test_exponential_memory_kernel_order():
    """Sigma(t,s) = lam exp(-gam (t-s)), eps = 0: with F(tau) = int_0^tau exp(-gam (tau-s)) G(s) ds
    the pair (G, F) obeys the linear system G' = -i lam F, F' = G - gam F, G(0) = -i, F(0) = 0,
    solved exactly by the matrix exponential."""
    T, lam, gam, k = 1.6, 0.9, 0.7, 4
    A = np.array([[0.0, -1j * lam], [1.0, -gam]], dtype=np.complex128)
    errs = []
    for N in (65, 129):
        h = T / (N - 1)
        ex = np.array([(expm(A * tau * h) @ np.array([-1j, 0.0]))[0] for tau in range(N)])
        G = np.zeros((N, N, 1, 1), dtype=np.complex128)
        S = np.zeros((N, N, 1, 1), dtype=np.complex128)
        for n in range(N):
            for m in range(n + 1):
                G[n, m] = ex[n - m]
                S[n, m] = lam * np.exp(-gam * (n - m) * h)
        Gs = solve(S, np.zeros((N, 1, 1), dtype=np.complex128), G, h, k, N)
        errs.append(max(np.abs(Gs[n, :n + 1] - G[n, :n + 1]).max() for n in range(N)))
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-4 and order > k - 0.3, (errs, order)


def test_first_rows_and_diagonal_are_kept():
    N, h, k = 12, 0.1, 3
    eps, S, G = _memory_case(N, h, 0.5)
    Gs = solve(S, eps, G, h, k, N)
    assert np.array_equal(Gs[:k], G[:k])
    for n in range(N):
        assert np.allclose(Gs[n, n], -1j)


# ---------------------------------------------------------------------------
# the lesser row (left form of the lesser equation, equal-time entry from the new row)

from oracle.step_solve import solve_lesser  # noqa: E402


def _lesser_errors(make, ks, Ns, T):
    out = {}
    for k in ks:
        errs = []
        for N in Ns:
            h = T / (N - 1)
            SR, SL, eps, GR, GL = make(N, h)
            _, GLs = solve_lesser(SR, SL, eps, GR, GL, h, k, N)
            errs.append(np.abs(GLs - GL).max() / np.abs(GL).max())
        out[k] = errs
    return out


def test_lesser_free_propagation_order():
    """Sigma = 0, constant Hermitian eps: G^<(t,t') = i e^{-i eps t} rho e^{i eps t'} for a
    Hermitian density matrix rho; the march from the exact first rows converges at order k."""
    norb, T = 2, 1.6
    rng = np.random.default_rng(4)
    A = rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))
    eps0 = 0.5 * (A + A.conj().T)
    B = rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))
    rho = 0.25 * (B @ B.conj().T)

    def make(N, h):
        U = [expm(-1j * eps0 * n * h) for n in range(N)]
        GR = np.zeros((N, N, norb, norb), dtype=np.complex128)
        GL = np.zeros((N, N, norb, norb), dtype=np.complex128)
        for n in range(N):
            for m in range(N):
                GL[n, m] = 1j * U[n] @ rho @ U[m].conj().T
                if m <= n:
                    GR[n, m] = -1j * U[n - m]
        z = np.zeros((N, N, norb, norb), dtype=np.complex128)
        return z, z.copy(), np.broadcast_to(eps0, (N, norb, norb)).copy(), GR, GL

    res = _lesser_errors(make, [2, 5], (65, 129), T)
    for k, errs in res.items():
        order = np.log2(errs[0] / errs[1])
        assert errs[1] < 1e-3 and order > k - 0.3, (k, errs, order)


def test_lesser_memory_kernel_closed_form_order():
    """eps = 0, constant scalar Sigma^R = lam, Sigma^< = 0: G^R(t, 0) = -i g(t) with
    g(t) = cosh(kappa t), kappa^2 = -i lam, and G^<(t, t') = G^R(t,0) G^<(0,0) G^A(0,t')
    = i rho0 g(t) conj(g(t')) solves the lesser equation; order min(k, 4)."""
    lam, rho0, T = 0.8, 0.3, 1.6
    kap = np.sqrt(-1j * lam)

    def make(N, h):
        t = np.arange(N) * h
        g = np.cosh(kap * t)
        GR = np.zeros((N, N, 1, 1), dtype=np.complex128)
        SR = np.zeros((N, N, 1, 1), dtype=np.complex128)
        for n in range(N):
            for m in range(n + 1):
                GR[n, m] = -1j * np.cosh(kap * (n - m) * h)
                SR[n, m] = lam
        GL = (1j * rho0 * np.outer(g, np.conj(g))).reshape(N, N, 1, 1)
        return SR, np.zeros_like(SR), np.zeros((N, 1, 1), dtype=np.complex128), GR, GL

    res = _lesser_errors(make, [3, 4, 5], (65, 129), T)
    for k, errs in res.items():
        order = np.log2(errs[0] / errs[1])
        assert errs[1] < 1e-3 and order > min(k, 4) - 0.3, (k, errs, order)


def test_lesser_memory_and_lesser_self_energy_closed_form_order():
    """eps = 0, constant scalar Sigma^R = lam and Sigma^< = mu (mu imaginary, so Sigma^< is
    anti-Hermitian): the lesser solution without initial correlations beyond G^<(0,0) is
    G^<(t,t') = G^R(t,0) G^<(0,0) G^A(0,t') + int_0^t int_0^{t'} G^R(t,s) Sigma^< G^A(s',t'),
    i.e. i rho0 cosh(kappa t) conj(cosh(kappa t')) + mu sinh(kappa t) conj(sinh(kappa t')) / |kappa|^2
    with kappa^2 = -i lam.  Order min(k, 3): the second integral over the short intervals
    [0, t_m], m < k, takes the closed Newton-Cotes rule of the interval's own length, the
    trapezoid at m = 1 with an O(h^3) error that column m carries through all later steps."""
    lam, mu, rho0, T = 0.8, 0.35j, 0.3, 1.6
    kap = np.sqrt(-1j * lam)

    def make(N, h):
        t = np.arange(N) * h
        c, sh = np.cosh(kap * t), np.sinh(kap * t)
        GR = np.zeros((N, N, 1, 1), dtype=np.complex128)
        SR = np.zeros((N, N, 1, 1), dtype=np.complex128)
        for n in range(N):
            for m in range(n + 1):
                GR[n, m] = -1j * np.cosh(kap * (n - m) * h)
                SR[n, m] = lam
        GL = (1j * rho0 * np.outer(c, np.conj(c)) + mu * np.outer(sh, np.conj(sh)) / abs(kap) ** 2)
        SL = np.full((N, N, 1, 1), mu, dtype=np.complex128)
        return SR, SL, np.zeros((N, 1, 1), dtype=np.complex128), GR, GL.reshape(N, N, 1, 1)

    res = _lesser_errors(make, [2, 3, 5], (65, 129), T)
    for k, errs in res.items():
        order = np.log2(errs[0] / errs[1])
        assert errs[1] < 1e-3 and order > min(k, 3) - 0.3, (k, errs, order)


# ---------------------------------------------------------------------------
# the paper's orientation: each row marched along t' in the right form

from oracle.step_solve import row_march  # noqa: E402


@pytest.mark.parametrize("k", [2, 3, 5])
def test_row_march_free_propagator_order(k):
    T, norb = 1.6, 2
    errs = []
    for N in (65, 129):
        h = T / (N - 1)
        eps, S, G = _free_case(N, h, norb, k)
        n = N - 1
        errs.append(np.abs(row_march(S, eps, n, h, k) - G[n, :n + 1]).max())
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-2 and order > k - 0.3, (k, errs, order)


@pytest.mark.parametrize("k", [3, 5])
def test_row_march_memory_kernel_order(k):
    T, lam = 1.6, 0.8
    errs = []
    for N in (65, 129):
        h = T / (N - 1)
        eps, S, G = _memory_case(N, h, lam)
        n = N - 1
        errs.append(np.abs(row_march(S, eps, n, h, k) - G[n, :n + 1]).max())
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-3 and order > min(k, 4) - 0.3, (k, errs, order)


def test_row_march_time_dependent_eps_closed_form():
    """Sigma = 0, scalar eps(t) = e0 + a cos(w t): G^R(t,t') = -i exp(-i int_{t'}^{t} eps) =
    -i exp(-i [e0 (t - t') + (a/w)(sin w t - sin w t')]); the row march takes eps at every
    column t', so this pins its use of eps(t'); order k."""
    e0, amp, om, T = 0.6, 0.8, 3.0, 1.6
    for k in (3, 5):
        errs = []
        for N in (65, 129):
            h = T / (N - 1)
            t = np.arange(N) * h
            eps = (e0 + amp * np.cos(om * t)).astype(np.complex128).reshape(N, 1, 1)
            n = N - 1
            ph = e0 * (t[n] - t[:n + 1]) + (amp / om) * (np.sin(om * t[n]) - np.sin(om * t[:n + 1]))
            exact = (-1j * np.exp(-1j * ph)).reshape(n + 1, 1, 1)
            S = np.zeros((N, N, 1, 1), dtype=np.complex128)
            errs.append(np.abs(row_march(S, eps, n, h, k) - exact).max())
        order = np.log2(errs[0] / errs[1])
        assert errs[1] < 1e-3 and order > k - 0.3, (k, errs, order)
