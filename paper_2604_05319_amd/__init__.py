"""Compressed history integrals of Kadanoff-Baym time stepping on AMD MI355X.

The compute path is the HIP library libhnessi.so (C ABI in include/hnessi.h);
this package only marshals arguments to it.
"""
from ._lib import (RET, LES, FLAG_FP32_FACTORS, FLAG_GRAPHS, Dense, Hodlr, HodlrBatch, HnessiError, compress_block,  # noqa: F401
                   exported_names, lib, weights, step_weights, born_lattice, LIB_PATH, set_allocator, set_tile_shape, use_torch_allocator)
