"""k-space filter on the GPU (one DFT pass per axis and direction) against
the FP64 oracle's FFT filter, both parity measures at 1e-4."""
import numpy as np
import pytest
import torch

import synth
from oracle import postproc as PP

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available()
    return mod


@pytest.mark.parametrize("dims", [(32, 32), (45, 38), (128, 128), (12, 14, 11), (96, 96, 48), (1, 7, 5), (5, 1, 3),
                                  (9, 4, 1), (1, 1, 1), (219, 219, 3), (700, 3)])
def test_filter_matches_fft_oracle(nfs, dims):
    L = int(np.prod(dims))
    rng = np.random.default_rng(L)
    rho = (rng.standard_normal(L) + 1j * rng.standard_normal(L)).astype(np.complex64)
    fr = PP.grid_frequencies(dims)
    # a soft, asymmetric filter: exercises the bin order and the weights
    f = (np.exp(-np.sum((fr / (0.3 * np.array(dims))) ** 2, axis=1)) * (fr[:, 0] > -dims[0] / 3)).astype(np.float32)
    got = nfs.apply_kspace_filter(torch.from_numpy(rho), torch.from_numpy(f), dims).cpu().numpy()
    want = PP.apply_kspace_filter(rho, f, dims)
    from _parity import check

    e = check(got, want, 1e-4, ("filter", dims))
    print(f"k-space filter {dims}: rel {e[0]:.2e}, max {e[1]:.2e}")


def test_filter_axis_limit_and_aliasing_rules(nfs):
    """An axis longer than 2048 is refused before any launch."""
    rho = torch.zeros(2049, dtype=torch.complex64)
    f = torch.ones(2049, dtype=torch.float32)
    with pytest.raises(nfs.NfsError) as ei:
        nfs.apply_kspace_filter(rho, f, (2049, 1))
    assert ei.value.code == nfs.NFS_ESHAPE


def test_hull_filter_on_the_2d_workload(nfs):
    """The paper's filter for the 2D 32x32 workload: mask from the hull of its
    first-order k positions, applied to the phantom."""
    d = synth.make_config("c1", with_noise=False)
    kpos = d["kcoef"][:, 1:3].astype(np.float64) / np.pi
    f = nfs.kspace_filter_mask(kpos, d["dims"])
    got = nfs.apply_kspace_filter(torch.from_numpy(d["rho_true"]), torch.from_numpy(f), d["dims"]).cpu().numpy()
    want = PP.apply_kspace_filter(d["rho_true"], f, d["dims"])
    e = rel(got, want)
    print(f"hull filter c1: {int(f.sum())} of {f.size} bins, rel {e:.2e}")
    assert e < 1e-4
