"""CPU-side checks of the C-ABI library: it loads, exports every declared call,
and its host-only weight tables match the oracle's exact rationals."""
import os
import re

import numpy as np
import pytest

import paper_2604_05319_amd as P
from oracle import weights as OW

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hnessi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hnessi_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_call():
    L = P.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.exported_names())


@pytest.mark.parametrize("k", range(1, 6))
def test_host_weights_match_oracle(k):
    for L in range(0, 2 * k + 6):
        w = P.weights(k, L)
        ref = OW.interval_weights_f64(k, L)
        np.testing.assert_array_equal(w, ref)


def test_weights_argument_errors():
    with pytest.raises(P.HnessiError):
        P.weights(0, 3)
    with pytest.raises(P.HnessiError):
        P.weights(6, 3)


def test_no_host_fallback_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    # creating a handle must fail loudly (no CPU path exists)
    with pytest.raises(Exception):
        P.Hodlr(64, 3, 1)


def test_tile_shape_validation():
    """hnessi_set_tile_shape checks norb and the chunk rows before anything else (no GPU)."""
    import paper_2604_05319_amd as P
    for norb, rows in ((3, 256), (4, 300), (4, 128), (16, 512), (8, 1024)):
        with pytest.raises(P.HnessiError):
            P.set_tile_shape(norb, rows)
    for norb, rows in ((1, 1024), (4, 256), (16, 128), (8, 0)):
        P.set_tile_shape(norb, rows)
        P.set_tile_shape(norb, 0)


@pytest.mark.parametrize("k", range(1, 6))
def test_host_step_weights_match_oracle(k):
    """The step solve's backward differentiation and differentiation-matrix tables
    (host, exact rationals rounded once) against the oracle's exact rationals."""
    a, D = P.step_weights(k)
    np.testing.assert_array_equal(a, [float(x) for x in OW.bdf_weights(k)])
    for i in range(k + 1):
        np.testing.assert_array_equal(D[i], [float(x) for x in OW.poly_differentiation_weights(k, i)])


def test_step_weights_argument_errors():
    for k in (0, 6):
        with pytest.raises(P.HnessiError):
            P.step_weights(k)
