"""ctypes binding of libhnessi.so (argument marshalling only).

Every call forwards to the C ABI declared in include/hnessi.h; device arrays
are contiguous complex128 torch tensors on the GPU and streams are torch's
current HIP stream.  There is no fallback: if the library or the GPU is
missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhnessi.so")

RET, LES = 0, 1
FLAG_FP32_FACTORS = 1   # U, V stored as complex float
FLAG_GRAPHS = 2         # sweeps replayed as HIP graphs, one per window between panel ends

STATUS = {0: "OK", -1: "E_ARG", -2: "E_ORDER", -3: "E_RANGE", -4: "E_NOMEM", -5: "E_DEVICE",
          -6: "E_RANK", -7: "E_VALUE"}


class HnessiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_SIGS = {
    "hnessi_last_error": ([], C.c_char_p),
    "hnessi_set_allocator": ([ALLOC_FN, FREE_FN, C.c_void_p], C.c_int),
    "hnessi_weights": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "hnessi_step_weights": ([C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_born_lattice": ([C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p,
                             C.c_void_p, C.c_longlong, C.c_void_p], C.c_int),
    "hnessi_hodlr_create": ([C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                             C.c_int, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "hnessi_hodlr_create_batched": ([C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_double, C.c_int, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "hnessi_hodlr_nk": ([C.c_void_p], C.c_int),
    "hnessi_hodlr_append_row_batched": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_longlong, C.c_void_p],
                                        C.c_int),
    "hnessi_history_step_batched": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_longlong, C.c_double,
                                     C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p], C.c_int),
    "hnessi_sweep_batched": ([C.c_void_p, C.c_int, C.c_int] + [C.c_void_p] * 4 + [C.c_longlong, C.c_double]
                             + [C.c_void_p] * 3, C.c_int),
    "hnessi_hodlr_destroy": ([C.c_void_p], C.c_int),
    "hnessi_hodlr_reset": ([C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_hodlr_append_row": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_history_R": ([C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_step_R": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                       C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_row_march_R": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_longlong,
                            C.c_void_p], C.c_int),
    "hnessi_step_lesser": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_double, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_step_R_batched": ([C.c_void_p, C.c_int, C.c_void_p, C.c_longlong, C.c_void_p, C.c_longlong, C.c_void_p,
                               C.c_longlong, C.c_void_p, C.c_longlong, C.c_double, C.c_void_p, C.c_longlong,
                               C.c_void_p], C.c_int),
    "hnessi_history_lesser": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                               C.c_void_p], C.c_int),
    "hnessi_history_R_adjoint": ([C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p],
                                 C.c_int),
    "hnessi_history_R_factor_grad": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p],
                                     C.c_int),
    "hnessi_factor_grad_reset": ([C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_factor_grad_get": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_hodlr_factors": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
                             C.c_int),
    "hnessi_history_step": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_sweep": ([C.c_void_p, C.c_int, C.c_int] + [C.c_void_p] * 4 + [C.c_double]
                     + [C.c_void_p] * 3, C.c_int),
    "hnessi_set_tile_shape": ([C.c_int, C.c_int], C.c_int),
    "hnessi_get_tile_shape": ([C.c_void_p], C.c_int),
    "hnessi_hodlr_graph_stats": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_hodlr_status": ([C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_hodlr_get": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "hnessi_hodlr_ranks": ([C.c_void_p, C.c_int, C.c_void_p, C.c_int], C.c_int),
    "hnessi_hodlr_blocks": ([C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "hnessi_hodlr_leaves": ([C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "hnessi_hodlr_bytes": ([C.c_void_p], C.c_size_t),
    "hnessi_compress_block": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_compress_block_noalloc": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_dense_create": ([C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "hnessi_dense_destroy": ([C.c_void_p], C.c_int),
    "hnessi_dense_reset": ([C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_dense_append_row": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_dense_history_step": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                   C.c_void_p, C.c_void_p], C.c_int),
    "hnessi_dense_sweep": ([C.c_void_p, C.c_int, C.c_int] + [C.c_void_p] * 4 + [C.c_double]
                           + [C.c_void_p] * 3, C.c_int),
    "hnessi_dense_bytes": ([C.c_void_p], C.c_size_t),
    "hnessi_hodlr_profile": ([C.c_void_p, C.c_int], C.c_int),
    "hnessi_hodlr_profile_read": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "hnessi_dense_profile": ([C.c_void_p, C.c_int], C.c_int),
    "hnessi_dense_profile_read": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
}


def lib():
    """Load the library (once) and declare every exported call."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def _check(rc):
    if rc < 0:
        raise HnessiError(rc, lib().hnessi_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("device tensor expected (the library runs on the GPU only)")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if t.dtype not in (torch.complex128, torch.float64, torch.int32):
        raise ValueError(f"unsupported dtype {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _profile_read(fn, h, kind):
    """(steps, ms) arrays of the timed launches of one kernel kind."""
    cnt = _check(fn(h, kind, None, None, 0))
    steps = np.zeros(max(cnt, 1), dtype=np.int32)
    ms = np.zeros(max(cnt, 1), dtype=np.float64)
    _check(fn(h, kind, steps.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p), cnt))
    return steps[:cnt], ms[:cnt]


# ctypes callbacks of every hook ever installed: a handle returns its memory through the
# hook it was created with, so none of them may be collected while the process runs
_hooks = []


def set_allocator(alloc=None, free=None):
    """Route the library's device allocations through Python callables.

    alloc(nbytes, stream_ptr) -> device pointer (int) or 0; free(ptr, stream_ptr).
    With no arguments the library's default (hipMallocAsync / hipFreeAsync) is restored."""
    if alloc is None and free is None:
        _check(lib().hnessi_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0)) or 0) or None
        except Exception:
            return None

    def _f(ptr, stream, ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:
            pass

    hook = (ALLOC_FN(_a), FREE_FN(_f))
    _hooks.append(hook)
    _check(lib().hnessi_set_allocator(hook[0], hook[1], None))


def use_torch_allocator():
    """Serve the library's device memory from PyTorch's caching allocator
    (stream-ordered on the stream of the allocating call)."""
    import torch

    def _alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def _free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(_alloc, _free)


def set_tile_shape(norb, proj_rows):
    """Projection chunk rows of handles created from now on (0: default)."""
    _check(lib().hnessi_set_tile_shape(norb, proj_rows))


def weights(k: int, L: int) -> np.ndarray:
    w = np.zeros(L + 1, dtype=np.float64)
    _check(lib().hnessi_weights(k, L, w.ctypes.data_as(C.c_void_p)))
    return w


def born_lattice(L, n, U, GR, GL, in_stride, SR, SL, out_stride):
    """Lattice second-Born self-energy of step n: Sigma^R_k(t_n, t_j) into SR and
    Sigma^<_k(t_j, t_n) into SL from G^R_k(t_n, t_j) and G^<_k(t_j, t_n) (device tensors,
    object k at k * stride, entries j = 0..n)."""
    _check(lib().hnessi_born_lattice(L, n, U, _ptr(GR), _ptr(GL), in_stride, _ptr(SR), _ptr(SL), out_stride,
                                     _stream()))


def step_weights(k: int):
    """(a, D): backward differentiation weights a_l and the differentiation matrix D[i][p]."""
    n = max(k + 1, 1)
    a = np.zeros(n, dtype=np.float64)
    D = np.zeros((n, n), dtype=np.float64)
    _check(lib().hnessi_step_weights(k, a.ctypes.data_as(C.c_void_p), D.ctypes.data_as(C.c_void_p)))
    return a, D


class Hodlr:
    """HODLR-compressed retarded and lesser components (one handle, one stream)."""

    def __init__(self, nt, nlvl, norb, k=5, tol=1e-10, panel=16, max_rank=16, flags=0):
        h = C.c_void_p()
        _check(lib().hnessi_hodlr_create(C.byref(h), nt, nlvl, norb, k, tol, panel, max_rank, flags,
                                         _stream()))
        self.h = h
        self.nt, self.nlvl, self.norb, self.k = nt, nlvl, norb, k
        self.tol, self.panel, self.max_rank, self.flags = tol, panel, max_rank, flags

    def spec(self):
        """The creation parameters (a handle of the same geometry: Hodlr(**H.spec()))."""
        return dict(nt=self.nt, nlvl=self.nlvl, norb=self.norb, k=self.k, tol=self.tol, panel=self.panel,
                    max_rank=self.max_rank, flags=self.flags)

    def close(self):
        if self.h:
            _check(lib().hnessi_hodlr_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(lib().hnessi_hodlr_reset(self.h, _stream()))

    def append_row(self, comp, n, row):
        _check(lib().hnessi_hodlr_append_row(self.h, comp, n, _ptr(row), _stream()))

    def history_R(self, n, sigR, h, out):
        _check(lib().hnessi_history_R(self.h, n, _ptr(sigR), h, _ptr(out), _stream()))

    def step_R(self, n, eps, sigR, sig_near, prev_rows, h, out):
        """Row n of G^R into out from the stored rows 0..n-1 (the row is not appended):
        eps (k+1, norb, norb) = eps(t_{n-k+i}); sigR (n+1, norb, norb) = Sigma^R(n, j);
        sig_near (k, k, norb, norb) = Sigma^R(t_{n-k+u}, t_{n-k+i}); prev_rows: k device
        rows, prev_rows[l-1] = row n-l of G^R."""
        if len(prev_rows) != self.k:
            raise ValueError(f"prev_rows must hold the k = {self.k} previous rows")
        ptrs = (C.c_void_p * self.k)(*[_ptr(r).value for r in prev_rows])
        _check(lib().hnessi_step_R(self.h, n, _ptr(eps), _ptr(sigR), _ptr(sig_near), ptrs, h, _ptr(out),
                                   _stream()))

    def row_march_R(self, n_lo, n_hi, eps, h, out, row_stride):
        """Rows n_lo..n_hi of G^R in the paper's orientation over the stored Sigma^R (this
        handle's retarded component): row n at out + (n - n_lo) * row_stride entries."""
        _check(lib().hnessi_row_march_R(self.h, n_lo, n_hi, _ptr(eps), h, _ptr(out), row_stride, _stream()))

    def step_lesser(self, n, eps, sigR_rows, sigL_slices, GR_row, prev_slices, h, out):
        """Lesser slice n (G^<(t_s, t_n), s <= n) into out: sigR_rows / sigL_slices the Sigma^R
        rows and Sigma^< slices n-k+1..n, GR_row the retarded row n, prev_slices the lesser
        slices n-1..n-k (all device tensors)."""
        k = self.k
        if len(sigR_rows) != k or len(sigL_slices) != k or len(prev_slices) != k:
            raise ValueError(f"sigR_rows, sigL_slices and prev_slices must each hold k = {k} arrays")
        arr = lambda xs: (C.c_void_p * k)(*[_ptr(x).value for x in xs])
        _check(lib().hnessi_step_lesser(self.h, n, _ptr(eps), arr(sigR_rows), arr(sigL_slices), _ptr(GR_row),
                                        arr(prev_slices), h, _ptr(out), _stream()))

    def history_lesser(self, n, sigR, sigL, h, out):
        _check(lib().hnessi_history_lesser(self.h, n, _ptr(sigR), _ptr(sigL), h, _ptr(out), _stream()))

    def history_step(self, n, sigR, sigL, h, outR, outL):
        _check(lib().hnessi_history_step(self.h, n, _ptr(sigR), _ptr(sigL), h, _ptr(outR), _ptr(outL),
                                         _stream()))

    def history_R_adjoint(self, n, ibar, h, out):
        """out(j) = h sum_{m<=j} w^{(n-m)}_{j-m} ibar(m) G^R(j,m)^dagger, j = 0..n."""
        _check(lib().hnessi_history_R_adjoint(self.h, n, _ptr(ibar), h, _ptr(out), _stream()))

    def factor_grad(self, n, sigR, ibar, h):
        _check(lib().hnessi_history_R_factor_grad(self.h, n, _ptr(sigR), _ptr(ibar), h, _stream()))

    def factor_grad_reset(self):
        _check(lib().hnessi_factor_grad_reset(self.h, _stream()))

    def _block_arrays(self, b, fn, *lead):
        lvl, r0, r1, c0, c1 = (int(x) for x in self.blocks()[b])
        U = np.zeros((self.max_rank, r1 - r0), dtype=np.complex128)
        V = np.zeros((self.max_rank, c1 - c0), dtype=np.complex128)
        S = np.zeros(self.max_rank)
        rk = _check(fn(self.h, *lead, U.ctypes.data_as(C.c_void_p), S.ctypes.data_as(C.c_void_p),
                       V.ctypes.data_as(C.c_void_p)))
        # rank columns, column r of U at U[:, r]
        return U[:rk].T.copy(), S[:rk].copy(), V[:rk].T.copy()

    def factor_grad_get(self, b, q):
        """(dU, dS, dV) of retarded block b, pair q: dU (rows, rank), dS (rank,), dV (cols, rank)."""
        return self._block_arrays(b, lib().hnessi_factor_grad_get, b, q)

    def factors(self, comp, b, q):
        """(U, S, V) of block b, pair q of component comp: U (rows, rank), S (rank,), V (cols, rank)."""
        return self._block_arrays(b, lambda h, b_, q_, *a: lib().hnessi_hodlr_factors(h, comp, b_, q_, *a), b, q)

    def sweep(self, n_begin, n_end, GR, GL, SR, SL, h, IR, IL):
        _check(lib().hnessi_sweep(self.h, n_begin, n_end, _ptr(GR), _ptr(GL), _ptr(SR), _ptr(SL), h,
                                  _ptr(IR), _ptr(IL), _stream()))

    def tile_shape(self):
        """Projection chunk rows of this handle."""
        return _check(lib().hnessi_get_tile_shape(self.h))

    def graph_stats(self):
        """(windows replayed as graphs, instantiations) of this handle's sweeps."""
        w, i = C.c_longlong(0), C.c_longlong(0)
        _check(lib().hnessi_hodlr_graph_stats(self.h, C.byref(w), C.byref(i)))
        return w.value, i.value

    def status(self):
        return _check(lib().hnessi_hodlr_status(self.h, _stream()))

    def get(self, comp, t1, t2):
        out = np.zeros((self.norb, self.norb), dtype=np.complex128)
        _check(lib().hnessi_hodlr_get(self.h, comp, t1, t2, out.ctypes.data_as(C.c_void_p)))
        return out

    def blocks(self):
        cap = 5 * (2 ** self.nlvl)
        tab = np.zeros(cap, dtype=np.int32)
        nb = _check(lib().hnessi_hodlr_blocks(self.h, tab.ctypes.data_as(C.c_void_p), cap))
        return tab[:5 * nb].reshape(nb, 5)

    def leaves(self):
        cap = 2 * (2 ** self.nlvl)
        tab = np.zeros(cap, dtype=np.int32)
        nl = _check(lib().hnessi_hodlr_leaves(self.h, tab.ctypes.data_as(C.c_void_p), cap))
        return tab[:2 * nl].reshape(nl, 2)

    def ranks(self, comp):
        """(nb, norb^2) ranks; (nk, nb, norb^2) for a batch."""
        nb = self.blocks().shape[0]
        nk = getattr(self, "nk", 1)
        cap = max(nk * nb * self.norb ** 2, 1)
        r = np.zeros(cap, dtype=np.int32)
        cnt = _check(lib().hnessi_hodlr_ranks(self.h, comp, r.ctypes.data_as(C.c_void_p), cap))
        r = r[:cnt].reshape(nk, nb, self.norb ** 2)
        return r if nk > 1 else r[0]

    def nbytes(self):
        return int(lib().hnessi_hodlr_bytes(self.h))

    def profile(self, stride):
        _check(lib().hnessi_hodlr_profile(self.h, stride))

    def profile_read(self, kind):
        return _profile_read(lib().hnessi_hodlr_profile_read, self.h, kind)


class HodlrBatch(Hodlr):
    """nk independent objects of one geometry (a k-point lattice), advanced in lockstep.

    Device arrays are object-major: object o's data starts o * stride elements
    (complex128) after the first object's."""

    def __init__(self, nk, nt, nlvl, norb, k=5, tol=1e-10, panel=16, max_rank=16, flags=0):
        h = C.c_void_p()
        _check(lib().hnessi_hodlr_create_batched(C.byref(h), nk, nt, nlvl, norb, k, tol, panel, max_rank,
                                                 flags, _stream()))
        self.h = h
        self.nk = nk
        self.nt, self.nlvl, self.norb, self.k = nt, nlvl, norb, k
        self.tol, self.panel, self.max_rank, self.flags = tol, panel, max_rank, flags

    def append_row(self, comp, n, rows, k_stride):
        _check(lib().hnessi_hodlr_append_row_batched(self.h, comp, n, _ptr(rows), k_stride, _stream()))

    def history_step(self, n, sigR, sigL, in_stride, h, outR, outL, out_stride):
        _check(lib().hnessi_history_step_batched(self.h, n, _ptr(sigR), _ptr(sigL), in_stride, h, _ptr(outR),
                                                 _ptr(outL), out_stride, _stream()))

    def step_R(self, n, eps, eps_stride, sigR, in_stride, sig_near, near_stride, prev_rows, prev_stride, h,
               out, out_stride):
        """Row n of G^R of every object (strides in complex entries between objects)."""
        if len(prev_rows) != self.k:
            raise ValueError(f"prev_rows must hold the k = {self.k} previous rows")
        ptrs = (C.c_void_p * self.k)(*[_ptr(r).value for r in prev_rows])
        _check(lib().hnessi_step_R_batched(self.h, n, _ptr(eps), eps_stride, _ptr(sigR), in_stride, _ptr(sig_near),
                                           near_stride, ptrs, prev_stride, h, _ptr(out), out_stride, _stream()))

    def sweep(self, n_begin, n_end, GR, GL, SR, SL, h, IR, IL, k_stride=None):
        """Packed triangles of every object, object-major (k_stride defaults to one triangle)."""
        if k_stride is None:
            k_stride = self.nt * (self.nt + 1) // 2 * self.norb ** 2
        for t in (GR, GL, SR, SL, IR, IL):
            if t.numel() < self.nk * k_stride:
                raise ValueError("array smaller than nk objects")
        _check(lib().hnessi_sweep_batched(self.h, n_begin, n_end, _ptr(GR), _ptr(GL), _ptr(SR), _ptr(SL),
                                          k_stride, h, _ptr(IR), _ptr(IL), _stream()))


class Dense:
    """Uncompressed storage of both components and direct-summation history integrals."""

    def __init__(self, nt, norb, k=5):
        h = C.c_void_p()
        _check(lib().hnessi_dense_create(C.byref(h), nt, norb, k, _stream()))
        self.h = h
        self.nt, self.norb, self.k = nt, norb, k

    def close(self):
        if self.h:
            _check(lib().hnessi_dense_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(lib().hnessi_dense_reset(self.h, _stream()))

    def append_row(self, comp, n, row):
        _check(lib().hnessi_dense_append_row(self.h, comp, n, _ptr(row), _stream()))

    def history_step(self, n, sigR, sigL, h, outR, outL):
        _check(lib().hnessi_dense_history_step(self.h, n, _ptr(sigR), _ptr(sigL), h, _ptr(outR),
                                               _ptr(outL), _stream()))

    def sweep(self, n_begin, n_end, GR, GL, SR, SL, h, IR, IL):
        _check(lib().hnessi_dense_sweep(self.h, n_begin, n_end, _ptr(GR), _ptr(GL), _ptr(SR), _ptr(SL),
                                        h, _ptr(IR), _ptr(IL), _stream()))

    def nbytes(self):
        return int(lib().hnessi_dense_bytes(self.h))

    def profile(self, stride):
        _check(lib().hnessi_dense_profile(self.h, stride))

    def profile_read(self, kind):
        return _profile_read(lib().hnessi_dense_profile_read, self.h, kind)


def compress_block(A, tol, max_rank, noalloc=False):
    """TSVD of a dense device block A (rows x cols complex128).  Returns (U, S, V, rank).
    noalloc: use the entry point whose scratch is the library's static device array."""
    import torch
    rows, cols = A.shape
    U = torch.zeros((max_rank, rows), dtype=torch.complex128, device=A.device)
    V = torch.zeros((max_rank, cols), dtype=torch.complex128, device=A.device)
    S = torch.zeros(max_rank, dtype=torch.float64, device=A.device)
    rk = torch.zeros(1, dtype=torch.int32, device=A.device)
    fn = lib().hnessi_compress_block_noalloc if noalloc else lib().hnessi_compress_block
    _check(fn(_ptr(A), rows, cols, cols, tol, max_rank, _ptr(U), _ptr(S), _ptr(V), _ptr(rk), _stream()))
    r = int(rk.item())
    if r < 0:
        raise HnessiError(r, "compress_block failed on the device (non-finite data or internal rank overflow)")
    return U[:r].T.contiguous(), S[:r].clone(), V[:r].T.contiguous(), r
