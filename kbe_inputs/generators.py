"""Damped-exponential generators (input construction only, no method arithmetic)."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class DampedExpSum:
    """Parameters of one two-time function C (retarded and lesser parts).

    omega, gamma, fermi: shape (P,) float64.  amp: shape (P, norb, norb) complex128.
    """
    omega: np.ndarray
    gamma: np.ndarray
    amp: np.ndarray
    fermi: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def norb(self) -> int:
        return int(self.amp.shape[-1])

    @property
    def nterms(self) -> int:
        return int(self.omega.shape[0])

    @property
    def herm_amp(self) -> np.ndarray:
        """Hermitian part of each amplitude, used by the lesser form."""
        return 0.5 * (self.amp + np.conj(np.swapaxes(self.amp, -1, -2)))


def _fermi(omega: np.ndarray, beta_f: float) -> np.ndarray:
    return 0.5 * (1.0 - np.tanh(0.5 * beta_f * omega))


def scalar_terms(seed: int, nterms: int = 8, beta_f: float = 1.0,
                 omega_range=(-4.0, 4.0), gamma_range=(0.02, 0.2),
                 scale: float = 1.0) -> DampedExpSum:
    """norb = 1: w ~ U[omega_range], g ~ U[gamma_range], a ~ scale * Dirichlet(1)."""
    rng = np.random.default_rng(seed)
    omega = rng.uniform(*omega_range, size=nterms)
    gamma = rng.uniform(*gamma_range, size=nterms)
    a = scale * rng.dirichlet(np.ones(nterms))
    amp = a.astype(np.complex128).reshape(nterms, 1, 1)
    return DampedExpSum(omega, gamma, amp, _fermi(omega, beta_f),
                        dict(kind="scalar", seed=seed, beta_f=beta_f))


def _haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def hermitian_terms(seed: int, nterms: int, norb: int, beta_f: float = 1.0,
                    omega_range=(-4.0, 4.0), gamma_range=(0.02, 0.2),
                    d_range=(0.5, 1.5)) -> DampedExpSum:
    """A_p = a_p U_p diag(d_p) U_p^H with Haar U_p, d_p ~ U[d_range]^norb, a ~ Dirichlet(1)."""
    rng = np.random.default_rng(seed)
    omega = rng.uniform(*omega_range, size=nterms)
    gamma = rng.uniform(*gamma_range, size=nterms)
    a = rng.dirichlet(np.ones(nterms))
    amp = np.empty((nterms, norb, norb), dtype=np.complex128)
    for p in range(nterms):
        u = _haar_unitary(rng, norb)
        d = rng.uniform(*d_range, size=norb)
        amp[p] = a[p] * (u * d[None, :]) @ np.conj(u.T)
    return DampedExpSum(omega, gamma, amp, _fermi(omega, beta_f),
                        dict(kind="hermitian", seed=seed, beta_f=beta_f))


def lattice_terms(seed: int, nk_side: int = 32, beta_f: float = 1.0):
    """Per-k generators on an nk_side x nk_side square lattice, eps_k = -2(cos kx + cos ky).

    G_k^R = -i e^{-(i eps_k + g_k) tau} (1 + 0.3 sum_{p=1..3} c_p e^{-(i nu_p + eta_p) tau}),
    g_k ~ U[0.02, 0.1], nu ~ U[-1, 1], eta ~ U[0.01, 0.1], c complex normal with
    sum |c_p| = 1, drawn per k.  Sigma_k^R: 4 terms, w = eps_k + U[-2, 2],
    g ~ U[0.02, 0.2], amplitudes 0.25 * Dirichlet(1).  Lesser weights f(eps_k).
    Returns two lists (G_k, Sigma_k) of DampedExpSum, k-major (kx slow, ky fast).
    """
    rng = np.random.default_rng(seed)
    gs, ss = [], []
    ks = 2.0 * np.pi * np.arange(nk_side) / nk_side
    for kx in ks:
        for ky in ks:
            eps = -2.0 * (np.cos(kx) + np.cos(ky))
            gk = rng.uniform(0.02, 0.1)
            nu = rng.uniform(-1.0, 1.0, size=3)
            eta = rng.uniform(0.01, 0.1, size=3)
            c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
            c = c / np.sum(np.abs(c))
            omega = np.concatenate([[eps], eps + nu])
            gamma = np.concatenate([[gk], gk + eta])
            amp = np.concatenate([[1.0 + 0j], 0.3 * c]).reshape(4, 1, 1)
            f = np.full(4, _fermi(np.array(eps), beta_f))
            gs.append(DampedExpSum(omega, gamma, amp, f, dict(kind="lattice_G", eps=eps)))
            so = eps + rng.uniform(-2.0, 2.0, size=4)
            sg = rng.uniform(0.02, 0.2, size=4)
            sa = (0.25 * rng.dirichlet(np.ones(4))).astype(np.complex128).reshape(4, 1, 1)
            ss.append(DampedExpSum(so, sg, sa, np.full(4, _fermi(np.array(eps), beta_f)),
                                   dict(kind="lattice_S", eps=eps)))
    return gs, ss


def retarded(p: DampedExpSum, t1, t2) -> np.ndarray:
    """C^R(t1, t2) for t1 >= t2 (broadcast arrays), shape (..., norb, norb)."""
    tau = np.asarray(t1, dtype=np.float64) - np.asarray(t2, dtype=np.float64)
    ph = np.exp(-(1j * p.omega + p.gamma) * tau[..., None])          # (..., P)
    out = ph @ p.amp.reshape(p.nterms, -1)                             # (..., norb^2)
    return (-1j * out).reshape(tau.shape + (p.norb, p.norb))


def lesser(p: DampedExpSum, t1, t2) -> np.ndarray:
    """C^<(t1, t2) for any t1, t2 (broadcast arrays), shape (..., norb, norb)."""
    t1 = np.asarray(t1, dtype=np.float64)
    t2 = np.asarray(t2, dtype=np.float64)
    tau = t1 - t2
    tsum = t1 + t2
    ph = p.fermi * np.exp(-1j * p.omega * tau[..., None] - 0.5 * p.gamma * tsum[..., None])
    out = ph @ p.herm_amp.reshape(p.nterms, -1)
    return (1j * out).reshape(tau.shape + (p.norb, p.norb))


def ret_row(p: DampedExpSum, n: int, h: float) -> np.ndarray:
    """Stored retarded row n: C^R(t_n, t_j), j = 0..n, shape (n+1, norb, norb)."""
    j = np.arange(n + 1)
    return retarded(p, np.full(n + 1, n * h), j * h)


def les_row(p: DampedExpSum, n: int, h: float) -> np.ndarray:
    """Stored lesser row n (paper orientation): C^<(t_s, t_n), s = 0..n."""
    s = np.arange(n + 1)
    return lesser(p, s * h, np.full(n + 1, n * h))


def packed_offset(n: int) -> int:
    """Offset (in elements of norb x norb) of row n in a packed lower triangle."""
    return n * (n + 1) // 2


def hermitian_drive(seed: int, norb: int, nt: int, h: float, scale: float = 1.0,
                    amp: float = 0.5, freq: float = 2.0) -> np.ndarray:
    """One-body term eps(t_n) = E0 + cos(freq t_n) amp E1, n = 0..nt-1, shape
    (nt, norb, norb): E0, E1 Hermitian with N(0, scale^2 / norb) entries (GUE-like),
    seeded."""
    rng = np.random.default_rng(seed)
    es = []
    for _ in range(2):
        z = (rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))) * (scale / np.sqrt(2.0 * norb))
        es.append(0.5 * (z + np.conj(z.T)))
    t = np.arange(nt) * h
    return es[0][None] + (amp * np.cos(freq * t))[:, None, None] * es[1][None]


def channel_terms(seed: int, norb: int, nchan: int, nterms: int = 1, omega_range=(-2.0, 2.0),
                  gamma_range=(0.05, 0.2), e_range=(-1.5, 1.5), d_range=(0.2, 0.6)):
    """A one-body term and a retarded self-energy that share one Haar eigenbasis U:
    eps0 = U diag(e) U^H and Sigma amplitudes A_p = a_p U diag(d_p) U^H, where e and d_p
    take nchan distinct values (each on norb / nchan orbitals).  Every orbital pair then
    couples the same nchan channels, which keeps the solution's block ranks bounded by
    nchan (1 + nterms) on long grids.  Returns (eps0 (norb, norb), DampedExpSum)."""
    rng = np.random.default_rng(seed)
    u = _haar_unitary(rng, norb)
    chan = np.arange(norb) % nchan
    e = rng.uniform(*e_range, size=nchan)[chan]
    omega = rng.uniform(*omega_range, size=nterms)
    gamma = rng.uniform(*gamma_range, size=nterms)
    a = rng.dirichlet(np.ones(nterms))
    amp = np.empty((nterms, norb, norb), dtype=np.complex128)
    for p in range(nterms):
        d = rng.uniform(*d_range, size=nchan)[chan]
        amp[p] = a[p] * (u * d[None, :]) @ np.conj(u.T)
    eps0 = (u * e[None, :]) @ np.conj(u.T)
    return eps0, DampedExpSum(omega, gamma, amp, _fermi(omega, 1.0), dict(kind="channels", seed=seed))
