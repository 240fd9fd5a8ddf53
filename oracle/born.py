"""FP64 lattice second-Born self-energy of one time step (test infrastructure, like the
rest of this package; only tests, the smoke entry point and the benchmark's CPU leg may
import it).

Section "Driven 2D Hubbard example", Eq. BornApproxLG, evaluated in real space as the
section "Implementation details" describes (transform G_k -> G_r, product, transform
Sigma_r -> Sigma_k):
    Sigma^>_r(t,t') = U^2 G^>_r(t,t') G^>_r(t,t') G^<_{-r}(t',t)
    Sigma^<_r(t,t') = U^2 G^<_r(t,t') G^<_r(t,t') G^>_{-r}(t',t)
on the L x L square lattice (one band): momenta k = 2 pi (kx, ky) / L, sites
r = (x, y), both enumerated x-major, G_r = (1/N_k) sum_k e^{i k.r} G_k,
Sigma_k = sum_r e^{-i k.r} Sigma_r.

One time step n gives the row t = t_n, t' = t_j, j = 0..n, from what the library stores:
    GR[k, j]  = G^R_k(t_n, t_j)        (retarded row)
    GLs[k, j] = G^<_k(t_j, t_n)        (stored lesser slice)
The other two-time values follow from the definitions of the components (one band,
t_n >= t_j):  G^<_k(t_n,t_j) = -conj(G^<_k(t_j,t_n)),  G^>_k(t_n,t_j) = G^R_k(t_n,t_j) +
G^<_k(t_n,t_j),  G^>_k(t_j,t_n) = G^<_k(t_j,t_n) - conj(G^R_k(t_n,t_j)) (retarded minus
advanced is greater minus lesser).  Outputs in the same orientations:
    SR[k, j]  = Sigma^R_k(t_n, t_j) = Sigma^>_k(t_n,t_j) - Sigma^<_k(t_n,t_j)
    SLs[k, j] = Sigma^<_k(t_j, t_n)    (computed from its own Born product, not by symmetry)
Every transform is an explicit DFT matrix product; every product is the definition's.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(L: int):
    """E[r, k] = exp(i k.r) over x-major sites r and momenta k of the L x L lattice."""
    m = np.arange(L)
    x = np.repeat(m, L)
    y = np.tile(m, L)
    ph = np.outer(x, x) + np.outer(y, y)          # kx x + ky y in units of 2 pi / L
    return np.exp(2j * np.pi * ph / L)


def to_real(A_k, L: int, sign: int = 1):
    """(1/N) sum_k e^{sign i k.r} A_k for A_k of shape (N, ...)."""
    E = dft_matrix(L)
    if sign < 0:
        E = np.conj(E)
    return np.tensordot(E, A_k, axes=(1, 0)) / (L * L)


def to_momentum(A_r, L: int):
    """sum_r e^{-i k.r} A_r for A_r of shape (N, ...)."""
    E = dft_matrix(L)
    return np.tensordot(np.conj(E).T, A_r, axes=(1, 0))


def born_step(GR, GLs, L: int, U: float):
    """(SR, SLs) of one time step from GR[k, j], GLs[k, j] (shape (L*L, n+1))."""
    GR = np.asarray(GR, dtype=np.complex128)
    GLs = np.asarray(GLs, dtype=np.complex128)
    Gl_nj = -np.conj(GLs)                 # G^<(t_n, t_j)
    Gg_nj = GR + Gl_nj                    # G^>(t_n, t_j)
    Gl_jn = GLs                           # G^<(t_j, t_n)
    Gg_jn = GLs - np.conj(GR)             # G^>(t_j, t_n)
    u2 = U * U
    # Sigma^>(t_n, t_j) and Sigma^<(t_n, t_j): G(t_n,t_j) at r, G(t_j,t_n) at -r
    Sg_nj = u2 * to_real(Gg_nj, L) ** 2 * to_real(Gl_jn, L, -1)
    Sl_nj = u2 * to_real(Gl_nj, L) ** 2 * to_real(Gg_jn, L, -1)
    # Sigma^<(t_j, t_n): G^<(t_j,t_n) at r, G^>(t_n,t_j) at -r
    Sl_jn = u2 * to_real(Gl_jn, L) ** 2 * to_real(Gg_nj, L, -1)
    return to_momentum(Sg_nj - Sl_nj, L), to_momentum(Sl_jn, L)


def born_momentum_bruteforce(GR, GLs, L: int, U: float):
    """The same step from the momentum-space convolution (O(N_k^2) per entry): with
    A_k B_k C_k the three factors of a Born product,
        Sigma_k = (U^2 / N_k^2) sum_{k1, k2} A_{k1} B_{k2} C_{k1 + k2 - k}
    (momenta added modulo the lattice).  Only for tiny lattices; pins born_step."""
    GR = np.asarray(GR, dtype=np.complex128)
    GLs = np.asarray(GLs, dtype=np.complex128)
    N = L * L
    Gl_nj = -np.conj(GLs)
    Gg_nj = GR + Gl_nj
    Gl_jn = GLs
    Gg_jn = GLs - np.conj(GR)

    def add(k1, k2, k):   # index of k1 + k2 - k
        x = (k1 // L + k2 // L - k // L) % L
        y = (k1 % L + k2 % L - k % L) % L
        return x * L + y

    def conv(A, B, C):
        out = np.zeros_like(A)
        for k in range(N):
            s = 0
            for k1 in range(N):
                for k2 in range(N):
                    s = s + A[k1] * B[k2] * C[add(k1, k2, k)]
            out[k] = s
        return U * U * out / (N * N)

    SR = conv(Gg_nj, Gg_nj, Gl_jn) - conv(Gl_nj, Gl_nj, Gg_jn)
    SLs = conv(Gl_jn, Gl_jn, Gg_nj)
    return SR, SLs
