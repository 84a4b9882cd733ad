"""GPU parity of the compressed phase basis: operators and CG solves run on
the problem nfs_compress_basis returns (with the per-sample offset applied
to the data by nfs_phase_shift), compared with the FP64 oracle on the
ORIGINAL problem.  Same tolerances as the other parity tests: 1e-4 for the
FP32 operand path, 2e-3 for the BF16/FP16 operand paths."""
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-3, "fp16": 2e-3}
PRECS = ["fp32", "bf16", "fp16"]


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def args(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.context(0)
    return mod


def compressed(nfs, d):
    full = nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
    cp, theta, info = nfs.compress_basis(full)
    return cp, theta, info


@pytest.fixture(scope="module")
def c1(nfs):
    d = synth.make_config("c1")
    rng = np.random.default_rng(21)
    d["rho"] = (rng.standard_normal(d["L"]) + 1j * rng.standard_normal(d["L"])).astype(np.complex64)
    d["m"] = (rng.standard_normal((d["n_coil"], d["K"])) + 1j * rng.standard_normal((d["n_coil"], d["K"]))).astype(np.complex64)
    d["cp"], d["theta"], d["info"] = compressed(nfs, d)
    return d


def test_c1_basis_is_compressed(nfs, c1):
    # x, y and B0 remain of 1, x, y, z on one slice
    print("c1 compressed:", c1["info"])
    assert c1["cp"].P == 2


@pytest.mark.parametrize("prec", PRECS)
def test_compressed_E_c1(nfs, c1, prec):
    m = nfs.phase_shift(nfs.apply_E(c1["cp"], torch.from_numpy(c1["rho"]), prec), c1["theta"], +1).cpu().numpy()
    err = rel(m, oracle.apply_E(c1["rho"], *args(c1)))
    print(f"compressed E c1 {prec}: rel {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_compressed_EH_c1(nfs, c1, prec):
    mm = nfs.phase_shift(torch.from_numpy(c1["m"]).cuda(), c1["theta"], -1)
    x = nfs.apply_EH(c1["cp"], mm, prec).cpu().numpy()
    err = rel(x, oracle.apply_EH(c1["m"], *args(c1)))
    print(f"compressed EH c1 {prec}: rel {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_compressed_EHE_c1(nfs, c1, prec):
    # theta cancels in E^H E: no rotation at all
    q = nfs.apply_EHE(c1["cp"], torch.from_numpy(c1["rho"]), prec).cpu().numpy()
    err = rel(q, oracle.apply_EHE(c1["rho"], *args(c1)))
    print(f"compressed EHE c1 {prec}: rel {err:.3e}")
    assert err < TOL[prec]


def test_phase_shift_against_double_rotation(nfs):
    rng = np.random.default_rng(3)
    G, K = 3, 1001
    m = (rng.standard_normal((G, K)) + 1j * rng.standard_normal((G, K))).astype(np.complex64)
    th = rng.uniform(-2000.0, 2000.0, K)
    theta = torch.from_numpy(th).cuda()
    for sign in (+1, -1):
        got = nfs.phase_shift(torch.from_numpy(m).cuda(), theta, sign).cpu().numpy()
        want = m.astype(np.complex128) * np.exp(1j * sign * th)[None, :]
        assert rel(got, want) < 2e-7
    # in place, and back again
    x = torch.from_numpy(m).cuda()
    nfs.phase_shift(x, theta, +1, out=x)
    nfs.phase_shift(x, theta, -1, out=x)
    assert rel(x.cpu().numpy(), m) < 4e-7


# ------------------------------- full-size 2D workload: sampled E, CG vs the stored oracle solve
@pytest.fixture(scope="module")
def c2(nfs):
    d = synth.make_config("c2")
    d["cp"], d["theta"], d["info"] = compressed(nfs, d)
    clean = oracle.apply_E(d["rho_true"], *args(d))
    sigma = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30.0 * np.sqrt(2))
    d["m"] = (clean + sigma * d["noise"]).astype(np.complex64)  # recipe of tests/golden/make_golden.py
    d["g"] = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_cg.npz"))
    return d


def test_c2_basis_takes_one_phase_instruction(nfs, c2):
    print("c2 compressed:", c2["info"])
    assert c2["cp"].P == 9  # 10 terms: 30 k-slots, one 16x16x32 phase product per tile


@pytest.mark.parametrize("prec", PRECS)
def test_compressed_c2_E_sampled(nfs, c2, prec):
    d = c2
    rng = np.random.default_rng(99)
    ks = np.sort(rng.choice(d["K"], 1500, replace=False))
    m = nfs.phase_shift(nfs.apply_E(d["cp"], torch.from_numpy(d["rho_true"]), prec), d["theta"], +1).cpu().numpy()
    ref = oracle.apply_E(d["rho_true"], d["sens"], d["fields"], d["b0"], d["kcoef"][ks], d["t"][ks])
    err = rel(m[:, ks], ref)
    print(f"compressed c2 E sampled {prec}: rel {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_compressed_c2_cg_vs_stored_oracle(nfs, c2, prec):
    d = c2
    mm = nfs.phase_shift(torch.from_numpy(d["m"]).cuda(), d["theta"], -1)
    rho, hist, info = nfs.cg_solve(d["cp"], mm, 30, precision=prec, reorth=True)
    rho10, _, _ = nfs.cg_solve(d["cp"], mm, 10, precision=prec, reorth=True)
    e30 = rel(rho.cpu().numpy(), d["g"]["reorth_rho"])
    e10 = rel(rho10.cpu().numpy(), d["g"]["reorth_it_10"])
    print(f"compressed c2 CG reorth {prec}: iterate 10 rel {e10:.2e}, iterate 30 rel {e30:.2e}")
    assert info.cpu().tolist() == [30, 1]
    assert e30 < TOL[prec] and e10 < TOL[prec]


# ------------------------------------------ batched slices on compressed bases
@pytest.mark.parametrize("mode", ["streams", "persistent"])
def test_compressed_batched_slices_match_oracle(nfs, mode):
    """Uneven 2D slices, each compressed to 10 terms, solved in one batched
    call on the rotated data; every slice against the oracle's solve of its
    original problem."""
    sl = synth.batched_slices(4, seed=5, n_range=(20, 36), g_range=(2, 10), k_range=(800, 2500))
    probs, ms, refs = [], [], []
    for d in sl:
        cp, theta, _ = compressed(nfs, d)
        assert cp.P == 9
        clean = oracle.apply_E(d["rho_true"], *args(d))
        sig = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30 * np.sqrt(2))
        m = (clean + sig * d["noise"]).astype(np.complex64)
        probs.append(cp)
        ms.append(nfs.phase_shift(torch.from_numpy(m).cuda(), theta, -1))
        refs.append(oracle.cg_solve(m, *args(d), n_iter=10, reorth=True)["rho"])
    nfs.set_batch_mode(0, mode)
    try:
        for prec in ("fp32", "fp16"):
            rb, _, ib = nfs.cg_solve_batched(probs, ms, 10, precision=prec, reorth=True)
            torch.cuda.synchronize()
            for i in range(len(sl)):
                err = rel(rb[i].cpu().numpy(), refs[i])
                print(f"compressed batched {mode} {prec} slice {i}: rel {err:.2e}")
                assert ib[i].cpu().tolist() == [10, 1]
                assert err < TOL[prec]
    finally:
        nfs.set_batch_mode(0, "streams")


# ------------------------------------------------------------- edge cases
def test_basis_of_constants_leaves_only_the_offset(nfs):
    """Field rows constant over the voxels and no B0: the compressed problem
    has no term left (n_basis 0, zero (t, b0) slot), and E is the coil
    weighting times exp(i theta) alone."""
    rng = np.random.default_rng(8)
    L, K, G, P = 200, 333, 3, 4
    d = dict(sens=(rng.standard_normal((G, L)) + 1j * rng.standard_normal((G, L))).astype(np.complex64),
             fields=np.repeat(rng.uniform(-1, 1, (P, 1)), L, axis=1).astype(np.float32),
             b0=np.zeros(L, np.float32), kcoef=(5 * rng.standard_normal((K, P))).astype(np.float32),
             t=np.linspace(0, 0.01, K).astype(np.float32))
    cp, theta, info = compressed(nfs, d)
    assert cp.P == 0 and info["err_bound"] < 1e-10  # rounding of the row means only
    rho = (rng.standard_normal(L) + 1j * rng.standard_normal(L)).astype(np.complex64)
    for prec in PRECS:
        m = nfs.phase_shift(nfs.apply_E(cp, torch.from_numpy(rho), prec), theta, +1).cpu().numpy()
        err = rel(m, oracle.apply_E(rho, *args(d)))
        print(f"constant basis E {prec}: rel {err:.2e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_compressed_cg_with_intensity_correction(nfs, c1, prec):
    """icorr travels with the compressed problem: the solve on rotated data
    equals the oracle's corrected solve of the original problem."""
    rng = np.random.default_rng(12)
    j = rng.uniform(0.5, 1.5, c1["L"]).astype(np.float32)
    full = nfs.Problem(*args(c1), icorr=j)
    cp, theta, _ = nfs.compress_basis(full)
    assert cp.icorr is not None and cp.P == 2
    m = c1["m"]
    rho, _, info = nfs.cg_solve(cp, nfs.phase_shift(torch.from_numpy(m).cuda(), theta, -1), 6, precision=prec,
                                reorth=True)
    ref = oracle.cg_solve(m, *args(c1), n_iter=6, icorr=j, reorth=True)["rho"]
    err = rel(rho.cpu().numpy(), ref)
    print(f"compressed CG with icorr {prec}: rel {err:.2e}")
    assert info.cpu().tolist() == [6, 1] and err < TOL[prec]
