"""Seeded synthetic two-time inputs for the compressed history integrals.

This module is shared by the FP64 oracle and by the device path.  It holds input
construction only: parameter draws and the evaluation of the generating closed
forms at grid points.  It holds none of the quadrature, history-sum or
compression arithmetic.

Every two-time function here is a sum of damped exponentials with norb x norb
matrix amplitudes A_p (the paper stores each N_o x N_o orbital block as one
matrix element per time pair, section "Multiorbital compression"):

    retarded:  C^R(t,t') = -i sum_p A_p exp(-(i w_p + g_p)(t - t')),    t >= t'
    lesser:    C^<(t,t') =  i sum_p f_p H_p exp(-i w_p (t - t')) exp(-g_p (t + t')/2)

with H_p the Hermitian part of A_p and f_p a Fermi weight.  The lesser form is
anti-Hermitian, C^<(t,t') = -[C^<(t',t)]^dagger, as the paper's symmetry
relation for the lesser component requires, and it is smooth across t = t'.

Grid convention (paper, section "Green's functions and Keldysh components"):
t_j = j h.  Retarded rows are stored as C^R(t_n, t_j), j = 0..n; lesser rows in
the paper's stored orientation C^<(t_s, t_n), s = 0..n.  Orbital indices are
innermost and row-major, so a row is (n+1) x norb x norb complex128.
"""
from .generators import (  # noqa: F401
    DampedExpSum, scalar_terms, hermitian_terms, lattice_terms,
    retarded, lesser, ret_row, les_row, packed_offset, hermitian_drive, channel_terms,
)
from .configs import CONFIGS, make_config_inputs  # noqa: F401
