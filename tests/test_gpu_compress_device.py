"""The phase-basis compression on the GPU (nfs_compress_basis_device), through
the C ABI: the same number of kept terms as the host computation, the
compressed phase equal to the model's phase to the reported residual bound
plus the outputs' float32 rounding at every checked (sample, voxel) pair
(the host test's criterion), the residual bound equal to the host's, and a
CG solve on the device-compressed basis (data rotated by exp(-i theta))
against the FP64 oracle on the original problem."""
import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import TOL, check
from test_compress_host import basis_bound, check_phase

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available()
    mod.context(0)
    return mod


def device_compress(nfs, inp, rel_tol=0.0):
    prob = nfs.Problem(inp.get("sens", np.ones((1, inp["fields"].shape[1]), np.complex64)), inp["fields"], inp["b0"],
                       inp["kcoef"], inp["t"])
    cp, theta, info = nfs.compress_basis(prob, rel_tol, on_device=True)
    n, L, K = info["n_basis"], prob.L, prob.K
    out = dict(fields=cp.fields.cpu().numpy().reshape(n, L), b0=cp.b0.cpu().numpy(),
               kcoef=cp.kcoef.cpu().numpy().reshape(K, n), t=cp.t.cpu().numpy(), theta=theta.cpu().numpy(),
               n_basis=n, err_bound=info["err_bound"])
    return out, cp, theta


def volume_basis():
    x, y, z = synth.grid_coords((12, 10, 8))
    rng = np.random.default_rng(1)
    K = 700
    return dict(fields=synth.solid_harmonics(x, y, z, 16).astype(np.float32),
                b0=(300 * rng.standard_normal(x.size)).astype(np.float32),
                kcoef=(40 * rng.standard_normal((K, 16))).astype(np.float32),
                t=np.linspace(0, 0.03, K).astype(np.float32))


CASES = {
    "c2 slice": lambda: synth.make_config("c2", with_noise=False),
    "c1 slice": lambda: synth.make_config("c1", with_noise=False),
    "batch slice": lambda: synth.batched_slices(1, seed=2)[0],
    "3D volume": volume_basis,
    "random basis": lambda: synth.random_problem(300, 500, 2, 6, seed=3),
    "no field terms": lambda: synth.random_problem(200, 300, 2, 0, seed=4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_compression_matches_host(nfs, name):
    inp = CASES[name]()
    host = nfs.compress_basis_host(inp["fields"], inp["b0"], inp["kcoef"], inp["t"])
    dev, _, _ = device_compress(nfs, inp)
    assert dev["n_basis"] == host["n_basis"], (dev["n_basis"], host["n_basis"])
    assert dev["err_bound"] <= 2.0 ** -24 * basis_bound(inp) * (1 + 1e-9)
    assert abs(dev["err_bound"] - host["err_bound"]) <= 1e-12 * basis_bound(inp) + 1e-6 * host["err_bound"]
    K, L = inp["kcoef"].shape[0], inp["fields"].shape[1]
    rng = np.random.default_rng(0)
    ks = rng.choice(K, min(K, 400), replace=False)
    ls = rng.choice(L, min(L, 400), replace=False)
    d, slack = check_phase(inp, dev, ks, ls)
    print(f"{name}: {dev['n_basis'] + 1} terms (host {host['n_basis'] + 1}), max phase change {d:.2e} rad "
          f"(allowed {slack:.2e}), residual bound {dev['err_bound']:.3e} (host {host['err_bound']:.3e})")
    assert d <= slack
    np.testing.assert_allclose(dev["theta"], host["theta"], rtol=1e-12, atol=1e-12 * np.abs(host["theta"]).max())


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_cg_on_device_compressed_basis(nfs, prec):
    s = synth.batched_slices(1, seed=5, n_range=(40, 40), g_range=(6, 6), k_range=(3000, 3000))[0]
    a = (s["sens"], s["fields"], s["b0"], s["kcoef"], s["t"])
    m = oracle.apply_E(s["rho_true"], *a).astype(np.complex64)
    ref = oracle.cg_solve(m, *a, n_iter=8, reorth=True)
    _, cp, theta = device_compress(nfs, s)
    assert cp.P + 1 == 10
    mc = nfs.phase_shift(torch.from_numpy(m).cuda(), theta, -1)
    rho, _, info = nfs.cg_solve(cp, mc, 8, precision=prec, reorth=True)
    assert info.cpu().tolist() == [8, 1]
    e = check(rho.cpu().numpy(), ref["rho"], TOL[prec], ("device-compressed CG", prec))
    print(f"CG on the device-compressed basis, {prec}: rel {e[0]:.1e}, max {e[1]:.1e}")
