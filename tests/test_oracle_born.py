"""Pins of the lattice second-Born oracle (real-space route) against what does not use
it: the momentum-space convolution of the same products (brute force, tiny lattices),
the closed form of a momentum-independent (local) Green's function, the anti-Hermitian
relation between the two lesser orientations, and the U^2 scaling."""
import numpy as np
import pytest

from oracle.born import born_momentum_bruteforce, born_step, to_momentum, to_real


def _rand(rng, N, J):
    return rng.standard_normal((N, J)) + 1j * rng.standard_normal((N, J))


@pytest.mark.parametrize("L", [2, 3])
def test_real_space_route_matches_momentum_convolution(L):
    rng = np.random.default_rng(L)
    N, J = L * L, 3
    GR, GLs = _rand(rng, N, J), _rand(rng, N, J)
    SR, SLs = born_step(GR, GLs, L, 0.7)
    bR, bL = born_momentum_bruteforce(GR, GLs, L, 0.7)
    np.testing.assert_allclose(SR, bR, rtol=0, atol=1e-13 * np.abs(bR).max())
    np.testing.assert_allclose(SLs, bL, rtol=0, atol=1e-13 * np.abs(bL).max())


def test_local_green_function_closed_form():
    """G_k independent of k: G_r = delta_{r,0} G, so every Born product is local and
    Sigma_k = U^2 (Gg^2 Gl' - Gl^2 Gg') is the same for every k."""
    rng = np.random.default_rng(5)
    L, J, U = 4, 6, 1.3
    gr = rng.standard_normal(J) + 1j * rng.standard_normal(J)
    gls = rng.standard_normal(J) + 1j * rng.standard_normal(J)
    GR, GLs = np.tile(gr, (L * L, 1)), np.tile(gls, (L * L, 1))
    SR, SLs = born_step(GR, GLs, L, U)
    gl = -np.conj(gls)
    gg = gr + gl
    ggr = gls - np.conj(gr)
    want_R = U * U * (gg ** 2 * gls - gl ** 2 * ggr)
    want_L = U * U * gls ** 2 * gg
    np.testing.assert_allclose(SR, np.tile(want_R, (L * L, 1)), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(SLs, np.tile(want_L, (L * L, 1)), rtol=1e-13, atol=1e-14)


def test_lesser_orientations_anti_hermitian():
    """Sigma^<_k(t_j, t_n) = -conj(Sigma^<_k(t_n, t_j)), the second computed here from its
    own Born product G^<(t_n,t_j)^2 G^>(t_j,t_n) at -r."""
    rng = np.random.default_rng(9)
    L, J, U = 4, 5, 0.9
    GR, GLs = _rand(rng, L * L, J), _rand(rng, L * L, J)
    _, SLs = born_step(GR, GLs, L, U)
    Gl_nj = -np.conj(GLs)
    Gg_jn = GLs - np.conj(GR)
    Sl_nj = to_momentum(U * U * to_real(Gl_nj, L) ** 2 * to_real(Gg_jn, L, -1), L)
    np.testing.assert_allclose(SLs, -np.conj(Sl_nj), rtol=0, atol=1e-13 * np.abs(SLs).max())


def test_u_squared_scaling_and_round_trip():
    rng = np.random.default_rng(2)
    L, J = 4, 3
    GR, GLs = _rand(rng, L * L, J), _rand(rng, L * L, J)
    a = born_step(GR, GLs, L, 1.0)
    b = born_step(GR, GLs, L, 3.0)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, 9.0 * x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(to_momentum(to_real(GR, L), L), GR, rtol=0, atol=1e-13)
