"""Truncated SVD with the paper's absolute threshold (section "Hierarchical decomposition").

Reading: singular values sigma_i >= eps are kept and sigma_i < eps dropped, so the
spectral-norm error of B ~ U S V^dagger is the largest dropped singular value,
which is below eps.  One truncation per orbital pair (section "Multiorbital
compression").
"""
from __future__ import annotations

import numpy as np


def tsvd(B, eps: float):
    """Return (U, s, V) with B ~ U diag(s) V^dagger and s >= eps."""
    U, s, Vh = np.linalg.svd(np.asarray(B, dtype=np.complex128), full_matrices=False)
    r = int(np.count_nonzero(s >= eps))
    return U[:, :r], s[:r], np.conj(Vh[:r].T)


def eps_rank(B, eps: float) -> int:
    s = np.linalg.svd(np.asarray(B, dtype=np.complex128), compute_uv=False)
    return int(np.count_nonzero(s >= eps))


def singular_values(B):
    return np.linalg.svd(np.asarray(B, dtype=np.complex128), compute_uv=False)
