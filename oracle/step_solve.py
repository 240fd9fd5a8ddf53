"""FP64 time step of the retarded Kadanoff-Baym equation (test infrastructure, like the
rest of this package; only tests may import it).

Equation (section "Kadanoff-Baym equations", retarded component, orbital matrices):
  left form   i d/dt G^R(t,t') - eps(t) G^R(t,t') = int_{t'}^{t} Sigma^R(t,s) G^R(s,t') ds
  right form -i d/dt' G^R(t,t') - G^R(t,t') eps(t') = int_{t'}^{t} G^R(t,s) Sigma^R(s,t') ds
  G^R(t,t) = -i.
The history term of the left form is the sum of Eq. KBER in the current-Sigma-row
orientation.  A time step n >= k, with rows 0..n-1 known (the first k rows come from a
bootstrap, not part of this step):
  * columns m < n-k: the left form at (t_n, t_m), the t-derivative by the backward
    differentiation weights a_j = -D_0j of the appendix, the history sum with the interval
    weights w^{(n-m)}, its newest term (j = n) moved to the left:
      [i a_0/h - eps(n) - h w^{(n-m)}_{n-m} Sigma(n,n)] G(n,m)
          = -(i/h) sum_{l=1..k} a_l G(n-l,m) + h sum_{j=m..n-1} w^{(n-m)}_{j-m} Sigma(n,j) G(j,m)
  * columns n-k <= m < n: the right form at (t_n, t_m), the t'-derivative of the degree-k
    polynomial through row n's points n-k..n (differentiation weights D_ip of the appendix,
    G(n,n) = -i known), the integral over [m, n] with the interval weights w^{(n-m)}: one
    linear system for the k unknown entries (a start of the row that needs no entry from
    the other side of the diagonal), which multiply the known matrices from the left, so
    the rows of G decouple.  With k-1 unknowns and G(n,n-k) taken from the first part the
    march is unstable for even k.
  * m = n: G(n,n) = -i.
Written from the equations; every sum is the definition's.
"""
from __future__ import annotations

import numpy as np

from .weights import bdf_weights, interval_weights_f64, poly_differentiation_weights


def bdf(k: int):
    return np.array([float(x) for x in bdf_weights(k)])


def diff_matrix(k: int):
    """D[i][p]: derivative at point i of the degree-k interpolant through points 0..k."""
    return np.array([[float(x) for x in poly_differentiation_weights(k, i)] for i in range(k + 1)])


def bulk_column(Gcol, Sig_row, eps_n, n: int, m: int, h: float, k: int):
    """G(n, m) for a column m < n-k from the left form: Gcol[j - m] = G(j, m) for
    j = m..n-1, Sig_row[j] = Sigma^R(n, j) for j = 0..n, eps_n = eps(t_n)."""
    norb = eps_n.shape[-1]
    I = np.eye(norb, dtype=np.complex128)
    a = bdf(k)
    L = n - m
    w = interval_weights_f64(k, L)
    M = (1j * a[0] / h) * I - eps_n - h * w[L] * Sig_row[n]
    rhs = -(1j / h) * sum(a[l] * Gcol[n - l - m] for l in range(1, k + 1))
    rhs = rhs + h * sum(w[j - m] * (Sig_row[j] @ Gcol[j - m]) for j in range(m, n))
    return np.linalg.solve(M, rhs)


def near_block(Sig_near, Sig_row, eps, n: int, h: float, k: int):
    """G(n, m) for m = n-k..n-1 (shape (k, norb, norb)) from the right form with
    G(n, n) = -i: Sig_near[u][i] = Sigma^R(t_{n-k+u}, t_{n-k+i}) (i <= u < k),
    Sig_row[j] = Sigma^R(n, j), eps[t] = eps(t) (t = n-k..n-1 read)."""
    norb = Sig_row.shape[-1]
    I = np.eye(norb, dtype=np.complex128)
    Gnn = -1j * I
    D = diff_matrix(k)
    C = np.zeros((k * norb, k * norb), dtype=np.complex128)
    R = np.zeros((norb, k * norb), dtype=np.complex128)
    for i in range(k):       # the equation at column m = n-k+i
        m = n - k + i
        L = n - m
        w = interval_weights_f64(k, L)
        for u in range(k):   # the unknown G(n, n-k+u)
            blk = -(1j / h) * D[i][u] * I
            if u == i:
                blk = blk - eps[m]
            if u >= i:
                blk = blk - h * w[u - i] * Sig_near[u][i]
            C[u * norb:(u + 1) * norb, i * norb:(i + 1) * norb] = blk
        R[:, i * norb:(i + 1) * norb] = (1j / h) * D[i][k] * Gnn + h * w[L] * (Gnn @ Sig_row[m])
    X = np.linalg.solve(C.T, R.T).T          # X C = R, X = [G(n, n-k+u)]_u
    return np.stack([X[:, u * norb:(u + 1) * norb] for u in range(k)])


def step(G, Sig, eps, n: int, h: float, k: int):
    """Row n of G^R, shape (n+1, norb, norb), from rows 0..n-1 of G (dense, G[j, m] for
    m <= j < n), Sigma^R (dense, Sig[s, m] for m <= s <= n) and eps (eps[t], t <= n)."""
    norb = eps.shape[-1]
    row = np.zeros((n + 1, norb, norb), dtype=np.complex128)
    row[n] = -1j * np.eye(norb, dtype=np.complex128)
    for m in range(0, n - k):
        row[m] = bulk_column(G[m:n, m], Sig[n], eps[n], n, m, h, k)
    if k > 0:
        near = [[Sig[n - k + u, n - k + i] for i in range(k)] for u in range(k)]
        row[n - k:n] = near_block(near, Sig[n], eps, n, h, k)
    return row


def step_lesser(GR, GL, SR, SL, eps, n: int, h: float, k: int):
    """Row n of G^<, G^<(t_n, t_m) for m = 0..n (shape (n+1, norb, norb)).  Equation of
    the lesser component (section "Kadanoff-Baym equations", Eq. KBEL, mixed term dropped)
    in its two forms:
      left   i d/dt G^<(t,t') = eps(t) G^<(t,t') + int_0^t Sigma^R(t,s) G^<(s,t') ds
                                + int_0^{t'} Sigma^<(t,s) G^A(s,t') ds
      right -i d/dt' G^<(t,t') = G^<(t,t') eps(t') + int_0^{t'} G^<(t,s) Sigma^A(s,t') ds
                                + int_0^t G^R(t,s) Sigma^<(s,t') ds
    (the right form is the left one's conjugate transpose, by G^<(t,t')^dagger = -G^<(t',t)).
      * columns m <= n-k: the left form at (t_n, t_m), the t-derivative by the backward
        differentiation weights on G^<(n-l, m) (all below the diagonal), the first integral
        over [0, t_n] with w^{(n)}, its newest term (s = n) moved to the left, the second
        over [0, t_m] with w^{(m)}:
          [i a_0/h - eps(n) - h w^{(n)}_n Sigma^R(n,n)] G^<(n,m) = -(i/h) sum_{l>=1} a_l G^<(n-l,m)
              + h sum_{s<n} w^{(n)}_s Sigma^R(n,s) G^<(s,m) + h sum_{s<=m} w^{(m)}_s Sigma^<(n,s) G^A(s,m)
      * columns m = n-k+1..n (the equal-time entry included): the right form at (t_n, t_m),
        its t'-derivative by the differentiation weights D_ip on the points n-k..n of row n
        (G^<(n, n-k) from the first part), the first integral over [0, t_m] with w^{(m)}
        (its terms s > n-k hold unknowns), the second over [0, t_n] with w^{(n)}: one
        system for the k unknown entries, which multiply known matrices from the right.
    A column derivative for every m < n (values above the diagonal taken from the row being
    solved by the lesser symmetry) is unstable near the diagonal (observed on this oracle:
    the error grows by about (a_1/a_0)^2 per step at k = 2).
    GR[t, t'] (t' <= t, rows 0..n, row n the new retarded row), GL[t, t'] (every t, t' < n,
    both triangles), SR[t, t'] (t' <= t <= n), SL[t, t'] (Sigma^<, every t, t' <= n), eps[t]."""
    norb = eps.shape[-1]
    row = np.zeros((n + 1, norb, norb), dtype=np.complex128)
    for m in range(0, n - k + 1):
        row[m] = lesser_bulk_column(lambda s, m=m: GL[s, m], GR[m, :m + 1], SR[n], SL[n], eps[n], n, m, h, k)
    near = [[SL[s, n - k + i] for s in range(n + 1)] for i in range(1, k + 1)]
    row[n - k + 1:] = lesser_near_block(row[:n - k + 1], GR[n], [SR[n - k + i] for i in range(1, k + 1)], near,
                                        eps, n, h, k)
    return row


def lesser_bulk_column(Gcol, GRm, SRn, SLn, eps_n, n: int, m: int, h: float, k: int):
    """G^<(n, m) for a column m <= n-k from the left form: Gcol(s) = G^<(t_s, t_m) for s < n,
    GRm[s] = G^R(t_m, t_s) (s <= m), SRn[s] = Sigma^R(t_n, t_s), SLn[s] = Sigma^<(t_n, t_s)
    (s <= n), eps_n = eps(t_n)."""
    norb = eps_n.shape[-1]
    I = np.eye(norb, dtype=np.complex128)
    a = bdf(k)
    wn = interval_weights_f64(k, n)
    wm = interval_weights_f64(k, m)
    M = (1j * a[0] / h) * I - eps_n - h * wn[n] * SRn[n]
    rhs = -(1j / h) * sum(a[l] * Gcol(n - l) for l in range(1, k + 1))
    rhs = rhs + h * sum(wn[s] * (SRn[s] @ Gcol(s)) for s in range(0, n))
    rhs = rhs + h * sum(wm[s] * (SLn[s] @ GRm[s].conj().T) for s in range(0, m + 1))
    return np.linalg.solve(M, rhs)


def lesser_near_block(row, GRn, SRnear, SLnear, eps, n: int, h: float, k: int):
    """G^<(n, n-k+p), p = 1..k (shape (k, norb, norb)) from the right form: row[s] =
    G^<(t_n, t_s) for s <= n-k (the left-form columns), GRn[s] = G^R(t_n, t_s) (s <= n),
    SRnear[i-1][s] = Sigma^R(t_m, t_s) (s <= m) and SLnear[i-1][s] = Sigma^<(t_s, t_m)
    (s <= n) for m = n-k+i, eps[t] (t = n-k+1..n read)."""
    norb = eps.shape[-1]
    I = np.eye(norb, dtype=np.complex128)
    D = diff_matrix(k)
    wn = interval_weights_f64(k, n)
    C = np.zeros((k * norb, k * norb), dtype=np.complex128)
    R = np.zeros((norb, k * norb), dtype=np.complex128)
    for i in range(1, k + 1):
        m = n - k + i
        wm = interval_weights_f64(k, m)
        SA = lambda s, i=i: SRnear[i - 1][s].conj().T            # Sigma^A(s, m), s <= m
        for p in range(1, k + 1):
            blk = -(1j / h) * D[i][p] * I
            if p == i:
                blk = blk - eps[m]
            s = n - k + p
            if s <= m:
                blk = blk - h * wm[s] * SA(s)
            C[(p - 1) * norb:p * norb, (i - 1) * norb:i * norb] = blk
        r = (1j / h) * D[i][0] * row[n - k]
        r = r + h * sum(wm[s] * (row[s] @ SA(s)) for s in range(0, n - k + 1))
        r = r + h * sum(wn[s] * (GRn[s] @ SLnear[i - 1][s]) for s in range(0, n + 1))
        R[:, (i - 1) * norb:i * norb] = r
    X = np.linalg.solve(C.T, R.T).T                # X C = R over X = [G^<(n, n-k+p)]_p
    return np.stack([X[:, (p - 1) * norb:p * norb] for p in range(1, k + 1)])


def solve_lesser(SR, SL, eps, GR_init, GL_init, h: float, k: int, N: int):
    """G^R and G^< on the whole grid (dense; G^< and Sigma^< on both triangles): rows
    0..k-1 of both from the initial arrays, then per step the retarded row (step) and the
    lesser row (step_lesser), the upper triangle of G^< by G^<(m, n) = -G^<(n, m)^dagger."""
    GR = solve(SR, eps, GR_init, h, k, N)
    norb = eps.shape[-1]
    GL = np.zeros((N, N, norb, norb), dtype=np.complex128)
    GL[:k, :k] = GL_init[:k, :k]
    for n in range(k, N):
        row = step_lesser(GR, GL, SR, SL, eps, n, h, k)
        GL[n, :n + 1] = row
        GL[:n, n] = -np.conj(np.swapaxes(row[:n], -1, -2))
    return GR, GL


def row_march(Sig, eps, n: int, h: float, k: int):
    """Row n of G^R by the paper's orientation (Eq. KBER: the derivative in the relative
    time, the current G row times the Sigma history): the right form
        -i d/dt' G^R(t_n, t') - G^R(t_n, t') eps(t') = int_{t'}^{t_n} G^R(t_n, s) Sigma^R(s, t') ds
    marched along the row from the diagonal, G^R(n, n) = -i, needs no other row.  Columns
    n-k..n-1: the k-unknown start of `step` (polynomial differentiation weights on the
    points n-k..n); columns m < n-k, leftwards: the t'-derivative by the backward
    differentiation weights on the points m, m+1, .., m+k of the row (f'(t_m) h ~
    -sum_l a_l f(t_{m+l})), the integral over [t_m, t_n] with w^{(n-m)}, its term s = m
    taken to the left:
        G(n,m) [i a_0/h - eps(m) - h w^{(n-m)}_0 Sigma(m,m)]
            = -(i/h) sum_{l>=1} a_l G(n, m+l) + h sum_{s=m+1}^{n} w^{(n-m)}_{s-m} G(n,s) Sigma(s,m).
    Sig[s, m] (m <= s <= n), eps[t] (t <= n).  Returns (n+1, norb, norb)."""
    norb = eps.shape[-1]
    I = np.eye(norb, dtype=np.complex128)
    a = bdf(k)
    row = np.zeros((n + 1, norb, norb), dtype=np.complex128)
    row[n] = -1j * I
    if k > 0:
        near = [[Sig[n - k + u, n - k + i] for i in range(k)] for u in range(k)]
        row[n - k:n] = near_block(near, Sig[n], eps, n, h, k)
    for m in range(n - k - 1, -1, -1):
        L = n - m
        w = interval_weights_f64(k, L)
        M = (1j * a[0] / h) * I - eps[m] - h * w[0] * Sig[m, m]
        rhs = -(1j / h) * sum(a[l] * row[m + l] for l in range(1, k + 1))
        rhs = rhs + h * sum(w[s - m] * (row[s] @ Sig[s, m]) for s in range(m + 1, n + 1))
        row[m] = np.linalg.solve(M.T, rhs.T).T        # X M = rhs
    return row


def solve(Sig, eps, G_init, h: float, k: int, N: int):
    """G^R on the whole grid (dense, G[n, m] for m <= n): rows 0..k-1 from G_init, the
    rest by successive steps."""
    norb = eps.shape[-1]
    G = np.zeros((N, N, norb, norb), dtype=np.complex128)
    G[:k] = G_init[:k]
    for n in range(k, N):
        G[n, :n + 1] = step(G, Sig, eps, n, h, k)
    return G
