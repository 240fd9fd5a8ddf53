"""GPU parity of the lattice second-Born self-energy (hnessi_born_lattice) against the FP64
oracle (real-space route with explicit DFT matrices), element by element.

Bar: max |gpu - oracle| / max |oracle| <= 1e-12 per output array (FP64 transforms of at
most 1024 points; the oracle's DFT sums and the kernel's radix-2 stages differ only in
rounding order).  Cases: every lattice size, rows whose length is not a multiple of the
kernel's column tile, padded object strides, outputs aliasing the inputs, and the
32 x 32 lattice workload (N_t = 2048) at its first, middle and last steps with the
lattice generator's Green's functions.
"""
import numpy as np
import pytest

from gpu_common import say
from oracle.born import born_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05319_amd as P
    return P


def _dev(x, stride):
    N, J = x.shape
    buf = np.zeros((N, stride), dtype=np.complex128)
    buf[:, :J] = x
    return torch.from_numpy(buf).to("cuda")


def _run(P, GR, GL, L, U, n, in_stride, out_stride, alias=False):
    gR, gL = _dev(GR, in_stride), _dev(GL, in_stride)
    if alias:
        sR, sL, out_stride = gR, gL, in_stride
    else:
        sR = torch.full((L * L, out_stride), complex("nan"), dtype=torch.complex128, device="cuda")
        sL = torch.full_like(sR, complex("nan"))
    P.born_lattice(L, n, U, gR, gL, in_stride, sR, sL, out_stride)
    torch.cuda.synchronize()
    return sR.cpu().numpy(), sL.cpu().numpy()


def _check(got, ref, label):
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  {label}: relative error {err:.2e}")
    assert err <= 1e-12, (label, err)


@pytest.mark.parametrize("L", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("n", [0, 1, 6, 37])
def test_born_random_against_oracle(P, L, n):
    rng = np.random.default_rng(100 * L + n)
    N, J = L * L, n + 1
    GR = rng.standard_normal((N, J)) + 1j * rng.standard_normal((N, J))
    GL = rng.standard_normal((N, J)) + 1j * rng.standard_normal((N, J))
    U = 0.75
    refR, refL = born_step(GR, GL, L, U)
    sR, sL = _run(P, GR, GL, L, U, n, J + 3, J + 5)
    _check(sR[:, :J], refR, f"L {L} n {n} Sigma^R")
    _check(sL[:, :J], refL, f"L {L} n {n} Sigma^<")
    # entries beyond the row are not written
    assert np.isnan(sR[:, J:]).all() and np.isnan(sL[:, J:]).all()


def test_born_outputs_alias_inputs(P):
    rng = np.random.default_rng(3)
    L, n = 16, 29
    N, J = L * L, n + 1
    GR = rng.standard_normal((N, J)) + 1j * rng.standard_normal((N, J))
    GL = rng.standard_normal((N, J)) + 1j * rng.standard_normal((N, J))
    refR, refL = born_step(GR, GL, L, 1.1)
    sR, sL = _run(P, GR, GL, L, 1.1, n, J, J, alias=True)
    _check(sR, refR, "aliased Sigma^R")
    _check(sL, refL, "aliased Sigma^<")


def test_born_argument_errors(P):
    x = torch.zeros((16, 8), dtype=torch.complex128, device="cuda")
    for L, n, ins, outs in ((3, 2, 8, 8), (4, -1, 8, 8), (4, 7, 7, 8), (4, 7, 8, 7)):
        with pytest.raises(P.HnessiError):
            P.born_lattice(L, n, 0.5, x, x, ins, x.clone(), x.clone(), outs)


def test_born_lattice_workload(P):
    """32 x 32 lattice, N_t = 2048, h = 0.02: the lattice generator's G^R_k rows and G^<_k
    slices at steps 0, 1, 1023 and 2047, every output entry against the oracle."""
    from kbe_inputs import make_config_inputs
    from kbe_inputs.generators import les_row, ret_row
    cfg, G, _ = make_config_inputs("c3")
    L, h = cfg["nk_side"], cfg["h"]
    for n in (0, 1, 1023, cfg["nt"] - 1):
        GR = np.stack([ret_row(g, n, h)[:, 0, 0] for g in G])
        GL = np.stack([les_row(g, n, h)[:, 0, 0] for g in G])
        refR, refL = born_step(GR, GL, L, 0.5)
        sR, sL = _run(P, GR, GL, L, 0.5, n, n + 1, n + 1)
        _check(sR, refR, f"lattice step {n} Sigma^R")
        _check(sL, refL, f"lattice step {n} Sigma^<")
