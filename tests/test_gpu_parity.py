"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over the whole complex vector): 1e-4 for the FP32
operand path, 2e-3 for the BF16/FP16 operand paths (the bars stated for the
FP32 and reduced-precision forms).  Inputs come from the seeded generators;
expected values come from the oracle only.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import PRECS, TOL, check, horizon, max_rel, rel, spread

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.context(0)
    return mod


def args(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


def gpu_problem(nfs, d, icorr=None):
    return nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"], icorr=icorr)


@pytest.fixture(scope="module")
def c1(nfs):
    d = synth.make_config("c1")
    rng = np.random.default_rng(11)
    d["rho"] = (rng.standard_normal(d["L"]) + 1j * rng.standard_normal(d["L"])).astype(np.complex64)
    d["m"] = (rng.standard_normal((d["n_coil"], d["K"])) + 1j * rng.standard_normal((d["n_coil"], d["K"]))).astype(np.complex64)
    d["E_ref"] = oracle.apply_E(d["rho"], *args(d))
    d["EH_ref"] = oracle.apply_EH(d["m"], *args(d))
    d["EHE_ref"] = oracle.apply_EHE(d["rho"], *args(d))
    d["gp"] = gpu_problem(nfs, d)
    return d


@pytest.mark.parametrize("prec", PRECS)
def test_E_c1(nfs, c1, prec):
    m = nfs.apply_E(c1["gp"], torch.from_numpy(c1["rho"]), prec).cpu().numpy()
    err, em = check(m, c1["E_ref"], TOL[prec], "E c1")
    print(f"E c1 {prec}: rel {err:.3e}, max {em:.3e}")


@pytest.mark.parametrize("prec", PRECS)
def test_EH_c1(nfs, c1, prec):
    x = nfs.apply_EH(c1["gp"], torch.from_numpy(c1["m"]), prec).cpu().numpy()
    err, em = check(x, c1["EH_ref"], TOL[prec], "EH c1")
    print(f"EH c1 {prec}: rel {err:.3e}, max {em:.3e}")


@pytest.mark.parametrize("prec", PRECS)
def test_EHE_c1(nfs, c1, prec):
    q = nfs.apply_EHE(c1["gp"], torch.from_numpy(c1["rho"]), prec).cpu().numpy()
    err, em = check(q, c1["EHE_ref"], TOL[prec], "EHE c1")
    print(f"EHE c1 {prec}: rel {err:.3e}, max {em:.3e}")


SHAPES = [
    (1000, 777, 5, 7),     # ragged everywhere, NB=1, NT=2
    (1, 1, 1, 0),          # single voxel/sample/coil, only the B0 term
    (33, 17, 16, 16),      # NB=2, NT=5, one full tile + 1
    (300, 500, 33, 20),    # NB=8 (66 real columns), NT=8
    (2048, 3000, 32, 16),  # several tiles, NB=4
    (16, 4096, 3, 4),      # one held tile for E^H, long stream
    (500, 700, 64, 31),    # the largest coil and term counts: NB=8, 32 terms (NQ=3)
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", PRECS)
def test_ragged_shapes(nfs, shape, prec):
    L, K, G, P = shape
    d = synth.random_problem(L, K, G, P, seed=21)
    gp = gpu_problem(nfs, d)
    a = args(d)
    m = nfs.apply_E(gp, torch.from_numpy(d["rho"]), prec).cpu().numpy()
    e1 = check(m, oracle.apply_E(d["rho"], *a), TOL[prec], ("E", shape))
    x = nfs.apply_EH(gp, torch.from_numpy(d["m"]), prec).cpu().numpy()
    e2 = check(x, oracle.apply_EH(d["m"], *a), TOL[prec], ("EH", shape))
    q = nfs.apply_EHE(gp, torch.from_numpy(d["rho"]), prec).cpu().numpy()
    e3 = check(q, oracle.apply_EHE(d["rho"], *a), TOL[prec], ("EHE", shape))
    print(f"shape {shape} {prec}: E {e1[0]:.2e}/{e1[1]:.2e} EH {e2[0]:.2e}/{e2[1]:.2e} EHE {e3[0]:.2e}/{e3[1]:.2e}")


@pytest.mark.parametrize("prec", PRECS)
def test_cg_at_the_largest_coil_and_term_counts(nfs, prec):
    """64 coils (8 column blocks) and 31 field terms (32 phase terms, three
    phase instructions per tile), the most the library takes: the
    re-orthogonalised CG against the oracle at every iterate, and the
    resident form (FP16) bit-identical to the split solve."""
    d = synth.random_problem(400, 600, 64, 31, seed=37)
    a = args(d)
    gp = gpu_problem(nfs, d)
    ref = oracle.cg_solve(d["m"], *a, n_iter=6, reorth=True, return_iterates=True)
    _, _, info, its = nfs.cg_solve_traced(gp, torch.from_numpy(d["m"]), 6, precision=prec, reorth=True)
    its = its.cpu().numpy()
    assert info.cpu().tolist() == [6, 1]
    errs = [check(its[k], ref["iterates"][k - 1], TOL[prec], ("CG max sizes", prec, k)) for k in range(1, 7)]
    print(f"64 coils, 32 terms, {prec}: " + " ".join(f"{e[0]:.1e}/{e[1]:.1e}" for e in errs))
    if prec == "fp16":
        rs, _, _ = nfs.cg_solve(gp, torch.from_numpy(d["m"]), 6, precision="fp16", reorth=True)
        rr, _, _ = nfs.cg_solve_resident(gp, torch.from_numpy(d["m"]), 6, precision="fp16", reorth=True)
        assert torch.equal(rs.cpu(), rr.cpu())


@pytest.mark.parametrize("prec", PRECS)
def test_empty_inputs(nfs, prec):
    # K = 0: E gives an empty array, E^H gives zeros
    d = synth.random_problem(40, 1, 3, 4, seed=3)
    d0 = dict(d, kcoef=d["kcoef"][:0], t=d["t"][:0])
    gp = gpu_problem(nfs, d0)
    m = nfs.apply_E(gp, torch.from_numpy(d["rho"]), prec)
    assert m.shape == (3, 0)
    x = nfs.apply_EH(gp, torch.zeros((3, 0), dtype=torch.complex64), prec).cpu().numpy()
    assert not np.any(x)
    rho, hist, info = nfs.cg_solve(gp, torch.zeros((3, 0), dtype=torch.complex64), 4, precision=prec)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 3]  # exact: E^H m == 0
    assert not torch.any(rho)
    # L = 0: E gives zeros
    d1 = dict(d, sens=d["sens"][:, :0], fields=d["fields"][:, :0], b0=d["b0"][:0])
    gp1 = gpu_problem(nfs, d1)
    m1 = nfs.apply_E(gp1, torch.zeros(0, dtype=torch.complex64), prec).cpu().numpy()
    assert m1.shape == (3, 1) and not np.any(m1)


def test_adjoint_identity_gpu(nfs, c1):
    gp = c1["gp"]
    Er = nfs.apply_E(gp, torch.from_numpy(c1["rho"]), "fp32").cpu().numpy().astype(np.complex128)
    EHm = nfs.apply_EH(gp, torch.from_numpy(c1["m"]), "fp32").cpu().numpy().astype(np.complex128)
    m64 = c1["m"].astype(np.complex128)
    lhs = np.vdot(Er, m64)
    rhs = np.vdot(c1["rho"].astype(np.complex128), EHm)
    # a random inner product cancels (|lhs| ~ ||E rho|| ||m|| / sqrt(N)), so the
    # error is measured against the Cauchy-Schwarz bound of either side
    assert abs(lhs - rhs) / (np.linalg.norm(Er) * np.linalg.norm(m64)) < 1e-6


def test_determinism(nfs, c1):
    gp = c1["gp"]
    for prec in PRECS:
        a = nfs.apply_EHE(gp, torch.from_numpy(c1["rho"]), prec).cpu()
        b = nfs.apply_EHE(gp, torch.from_numpy(c1["rho"]), prec).cpu()
        assert torch.equal(a, b)


# ------------------------------------------------------------------ CG
# Two reference trajectories.  "plain" follows the figure's recurrences as
# printed; "reorth" additionally re-orthogonalises each residual (identical
# in exact arithmetic).  On the paper-shaped spiral workloads E^H E is
# numerically singular (full field of view, unsampled k-space corners), and
# the FP64 plain recurrences themselves leave the exact-arithmetic trajectory
# once CG stagnates; the re-orthogonalised trajectory is stable under
# rounding.  So: the GPU reorth solve is compared with the oracle reorth
# solve at every iterate; the GPU plain solve is compared with the oracle
# plain solve at every iterate up to the horizon where the plain trajectory
# is stable at the GPU's working precision -- measured with the oracle's
# sensitivity probe (every E^H E p perturbed by relative noise delta, delta
# twice the measured relative error of one GPU E^H E application at that
# precision on this problem) as the last iterate the probe keeps within
# TOL/4 -- and beyond it only its validity is checked (same data residual
# and solution norm as the oracle, to 1%).


def noisy_data(d, snr=30.0):
    clean = oracle.apply_E(d["rho_true"], *args(d))
    sigma = np.sqrt(np.mean(np.abs(clean) ** 2)) / (snr * np.sqrt(2))
    return (clean + sigma * d["noise"]).astype(np.complex64)


@pytest.fixture(scope="module")
def c1_cg(nfs, c1):
    m = noisy_data(c1)
    n = c1["n_iter"]
    plain = oracle.cg_solve(m, *args(c1), n_iter=n, return_iterates=True)
    reo = oracle.cg_solve(m, *args(c1), n_iter=n, return_iterates=True, reorth=True)
    # the oracle's probes of each operand form's rounding on the plain
    # trajectory: relative noise at twice the measured E^H E error (three
    # seeded realisations) and, for FP16 / BF16, the operands rounded as
    # those forms round them.  The horizon comes from the probe that models
    # the form (operand rounding for FP16 / BF16, noise for FP32, whose split
    # operands round to ~2^-22); the spread past it is the largest deviation
    # over all of them.
    probes = {}
    for prec in PRECS:
        q = nfs.apply_EHE(c1["gp"], torch.from_numpy(c1["rho"]), prec).cpu().numpy()
        runs = [oracle.cg_solve(m, *args(c1), n_iter=n, return_iterates=True, perturb=(2 * rel(q, c1["EHE_ref"]), s))
                for s in (7, 8, 9)]
        if prec in ("fp16", "bf16"):
            runs.append(oracle.cg_solve(m, *args(c1), n_iter=n, return_iterates=True, operands=prec))
        devs = np.array([[rel(x, y) for x, y in zip(pr["iterates"], plain["iterates"])] for pr in runs])
        dev = np.max(devs, axis=0)
        d2 = np.max([np.abs(pr["hist"][1:, 2] - plain["hist"][1:, 2]) for pr in runs], axis=0)
        model = devs[-1] if prec in ("fp16", "bf16") else np.max(devs, axis=0)
        hz = horizon(model, TOL[prec])
        probes[prec] = dict(dev=dev, d2=d2, horizon=hz)
        print(f"plain CG horizon {prec}: {hz} iterations")
    return dict(m=m, plain=plain, reorth=reo, probes=probes)


@pytest.fixture(scope="module")
def wellcond(nfs):
    d = synth.random_problem(400, 1500, 4, 4, seed=31, phase_scale=20.0)
    ref = oracle.cg_solve(d["m"], *args(d), n_iter=12, return_iterates=True)
    return dict(d=d, gp=gpu_problem(nfs, d), ref=ref)


@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("prec", PRECS)
def test_cg_well_conditioned_every_iterate(nfs, wellcond, prec, reorth):
    d, ref = wellcond["d"], wellcond["ref"]
    for n in [1, 2, 3, 5, 8, 12]:
        rho, hist, info = nfs.cg_solve(wellcond["gp"], torch.from_numpy(d["m"]), n, precision=prec, reorth=reorth)
        check(rho.cpu().numpy(), ref["iterates"][n - 1], TOL[prec], ("well-conditioned CG", n))
    h = hist.cpu().numpy()
    assert info.cpu().tolist() == [12, 1]
    assert np.max(np.abs(h[:, 0] - ref["hist"][:, 0])) < TOL[prec] * ref["hist"][0, 0]
    assert np.max(np.abs(h[:, 1] - ref["hist"][:, 1])) < TOL[prec] * ref["hist"][-1, 1]
    assert np.max(np.abs(h[:, 2] - ref["hist"][:, 2])) < TOL[prec] * ref["hist"][0, 2]


@pytest.mark.parametrize("prec", PRECS)
def test_cg_c1_reorth_every_iterate(nfs, c1, c1_cg, prec):
    ref = c1_cg["reorth"]
    errs = []
    for n in [1, 3, 5, 8, 10, 12, 15, 18, 20]:
        rho, hist, info = nfs.cg_solve(c1["gp"], torch.from_numpy(c1_cg["m"]), n, precision=prec, reorth=True)
        errs.append(check(rho.cpu().numpy(), ref["iterates"][n - 1], TOL[prec], ("CG c1 reorth", n)))
    print(f"CG c1 reorth {prec}: " + " ".join(f"{e:.1e}/{m:.1e}" for e, m in errs))
    assert info.cpu().tolist() == [20, 1]
    h = hist.cpu().numpy()
    assert np.max(np.abs(h[:, 2] - ref["hist"][:, 2])) < TOL[prec] * ref["hist"][0, 2]


@pytest.mark.parametrize("prec", PRECS)
def test_cg_c1_plain(nfs, c1, c1_cg, prec):
    """The recurrences as printed against the FP64 plain solve at every
    iterate: at the bar up to the horizon of the oracle's probes for this
    operand form, past it within four times the probes' deviation (up to
    two iterates ahead, tests/_parity.py: spread) plus the bar (iterates,
    solution norm, data residual)."""
    ref = c1_cg["plain"]
    pb = c1_cg["probes"][prec]
    hz = pb["horizon"]
    assert hz >= 1
    n = c1["n_iter"]
    _, hist, info, its = nfs.cg_solve_traced(c1["gp"], torch.from_numpy(c1_cg["m"]), n, precision=prec)
    its = its.cpu().numpy()
    assert info.cpu().tolist() == [n, 1]
    for k in range(1, hz + 1):
        check(its[k], ref["iterates"][k - 1], TOL[prec], ("CG c1 plain", prec, k))
    bound = 4 * spread(pb["dev"]) + TOL[prec]
    errs = np.array([rel(its[k], ref["iterates"][k - 1]) for k in range(1, n + 1)])
    assert np.all(errs <= bound), (prec, errs, bound)
    h, rh = hist.cpu().numpy(), ref["hist"]
    assert np.all(np.abs(h[1:, 1] - rh[1:, 1]) <= bound * rh[1:, 1]), "solution norm"
    assert np.all(np.abs(h[1:, 2] - rh[1:, 2]) <= 4 * spread(pb["d2"]) + TOL[prec] * rh[1:, 2]), "data residual"
    print(f"CG c1 plain {prec}: horizon {hz} of {n}; errors at 5, 10, 20: "
          f"{errs[4]:.1e}, {errs[9]:.1e}, {errs[n - 1]:.1e} (probe {pb['dev'][4]:.1e}, {pb['dev'][9]:.1e}, "
          f"{pb['dev'][n - 1]:.1e}); oracle plain vs reorth {rel(ref['rho'], c1_cg['reorth']['rho']):.2e}")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_cg_residual_replacement(nfs, c1, c1_cg, prec):
    n = c1["n_iter"]
    rho, hist, info = nfs.cg_solve(c1["gp"], torch.from_numpy(c1_cg["m"]), n, replace_every=5, precision=prec,
                                   reorth=True)
    torch.cuda.synchronize()
    err = rel(rho.cpu().numpy(), c1_cg["reorth"]["rho"])
    print(f"CG c1 {prec} reorth + replace_every=5: rel {err:.3e}")
    assert err < TOL[prec]


def test_cg_tolerance_stop(nfs, c1, c1_cg):
    ref = c1_cg["reorth"]
    r = ref["hist"][:, 0] / ref["hist"][0, 0]
    # first step whose residual falls clearly below all earlier ones
    n_stop = next(n for n in range(3, len(r)) if r[n] < 0.98 * r[:n].min())
    tol = float(np.sqrt(r[n_stop] * r[:n_stop].min()))
    rho, hist, info = nfs.cg_solve(c1["gp"], torch.from_numpy(c1_cg["m"]), 50, tol=tol, precision="fp32",
                                   reorth=True)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [n_stop, 2]
    assert rel(rho.cpu().numpy(), ref["iterates"][n_stop - 1]) < 1e-4
    h = hist.cpu().numpy()
    assert np.all(np.isnan(h[n_stop + 1:]))


def test_cg_unitary_one_step(nfs):
    d = synth.dft_problem(16)
    gp = gpu_problem(nfs, d)
    rng = np.random.default_rng(1)
    m = (rng.standard_normal((1, d["K"])) + 1j * rng.standard_normal((1, d["K"]))).astype(np.complex64)
    rho, hist, info = nfs.cg_solve(gp, torch.from_numpy(m), 5, tol=1e-3, precision="fp32")
    torch.cuda.synchronize()
    it, st = info.cpu().tolist()
    assert it == 1 and st == 2
    want = oracle.apply_EH(m, *args(d)) / d["K"]
    assert rel(rho.cpu().numpy(), want) < 1e-4


def test_cg_n_iter_zero_and_intensity_correction(nfs, c1, c1_cg):
    rho, hist, info = nfs.cg_solve(c1["gp"], torch.from_numpy(c1_cg["m"]), 0)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 1] and not torch.any(rho)
    j = np.random.default_rng(2).uniform(0.5, 2.0, size=c1["L"]).astype(np.float32)
    gp = gpu_problem(nfs, c1, icorr=j)
    rho, hist, info = nfs.cg_solve(gp, torch.from_numpy(c1_cg["m"]), 5, precision="fp32")
    ref = oracle.cg_solve(c1_cg["m"], *args(c1), n_iter=5, icorr=j)
    assert rel(rho.cpu().numpy(), ref["rho"]) < 1e-4


def test_cg_determinism(nfs, c1, c1_cg):
    out = []
    for _ in range(2):
        rho, hist, info = nfs.cg_solve(c1["gp"], torch.from_numpy(c1_cg["m"]), 10, precision="fp16", reorth=True)
        out.append((rho.cpu(), hist.cpu()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


# ------------------------------------------- full-size workload, sampled outputs
@pytest.fixture(scope="module")
def c2(nfs):
    d = synth.make_config("c2")
    d["gp"] = gpu_problem(nfs, d)
    rng = np.random.default_rng(99)
    d["ks"] = np.sort(rng.choice(d["K"], 1500, replace=False))
    d["ls"] = np.sort(rng.choice(d["L"], 1500, replace=False))
    return d


@pytest.mark.parametrize("prec", PRECS)
def test_c2_E_sampled(nfs, c2, prec):
    d = c2
    rho = d["rho_true"]
    m = nfs.apply_E(d["gp"], torch.from_numpy(rho), prec).cpu().numpy()
    ks = d["ks"]
    ref = oracle.apply_E(rho, d["sens"], d["fields"], d["b0"], d["kcoef"][ks], d["t"][ks])
    err, em = check(m[:, ks], ref, TOL[prec], "c2 E sampled")
    print(f"c2 E sampled {prec}: rel {err:.3e}, max {em:.3e}")


@pytest.mark.parametrize("prec", PRECS)
def test_c2_EH_sampled(nfs, c2, prec):
    d = c2
    rng = np.random.default_rng(4)
    m = (rng.standard_normal((d["n_coil"], d["K"])) + 1j * rng.standard_normal((d["n_coil"], d["K"]))).astype(np.complex64)
    x = nfs.apply_EH(d["gp"], torch.from_numpy(m), prec).cpu().numpy()
    ls = d["ls"]
    ref = oracle.apply_EH(m, d["sens"][:, ls], d["fields"][:, ls], d["b0"][ls], d["kcoef"], d["t"])
    err, em = check(x[ls], ref, TOL[prec], "c2 EH sampled")
    print(f"c2 EH sampled {prec}: rel {err:.3e}, max {em:.3e}")


# --------------------------------------- full-size CG against the stored oracle solve
@pytest.fixture(scope="module")
def c2_golden(c2):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_cg.npz")
    g = np.load(path)
    m = noisy_data(c2)  # same recipe as tests/golden/make_golden.py (oracle E)
    return dict(g=g, m=m)


@pytest.mark.parametrize("prec", PRECS)
def test_c2_cg_reorth_vs_stored_oracle(nfs, c2, c2_golden, prec):
    g = c2_golden["g"]
    rho, hist, info = nfs.cg_solve(c2["gp"], torch.from_numpy(c2_golden["m"]), 30, precision=prec, reorth=True)
    err = check(rho.cpu().numpy(), g["reorth_rho"], TOL[prec], "c2 CG reorth 30")
    rho10, _, _ = nfs.cg_solve(c2["gp"], torch.from_numpy(c2_golden["m"]), 10, precision=prec, reorth=True)
    e10 = check(rho10.cpu().numpy(), g["reorth_it_10"], TOL[prec], "c2 CG reorth 10")
    print(f"c2 CG reorth {prec}: iterate 10 rel/max {e10[0]:.2e}/{e10[1]:.2e}, iterate 30 {err[0]:.2e}/{err[1]:.2e}")
    assert info.cpu().tolist() == [30, 1]


@pytest.mark.parametrize("prec", PRECS)
def test_c2_cg_plain_vs_stored_oracle(nfs, c2, c2_golden, prec):
    """The recurrences as printed at full size, every iterate against the
    stored FP64 plain solve: at the bar up to the horizon of the probe that
    models the operand form (the FP64 solve with the FP16 / BF16 operand
    rounding; for FP32, relative noise at the smallest stored level at
    least twice the measured E^H E error), past it within four times the
    largest probe deviation (up to two iterates ahead, tests/_parity.py:
    spread) plus the bar, with the solution-norm and data-residual
    histories."""
    g = c2_golden["g"]
    n = int(g["n_iter"])
    ref, rh = g["plain_its"], g["plain_hist"]
    devs, d2s = [], []
    if prec == "fp32":
        rng = np.random.default_rng(17)
        ls = np.sort(rng.choice(c2["L"], 400, replace=False))
        p = (rng.standard_normal(c2["L"]) + 1j * rng.standard_normal(c2["L"])).astype(np.complex64)
        q = nfs.apply_EHE(c2["gp"], torch.from_numpy(p), prec).cpu().numpy()
        # E^H E p at 400 sampled voxels: E p in full, E^H on the sampled voxels
        a = args(c2)
        y = oracle.apply_E(p, *a)
        q_ref = oracle.apply_EH(y, c2["sens"][:, ls], c2["fields"][:, ls], c2["b0"][ls], c2["kcoef"], c2["t"])
        err = rel(q[ls], q_ref)
        lv = [i for i, dl in enumerate(g["probe_deltas"]) if dl >= 2 * err]
        assert lv, ("operator error beyond the stored probes", err)
        devs.append(g["probe_dev"][lv[0]])
        d2s.append(np.abs(g["probe_hist"][lv[0]][1:, 2] - rh[1:, 2]))
        label = f"noise {g['probe_deltas'][lv[0]]:.0e} (E^H E error {err:.1e})"
    else:
        devs.append(g[f"emul_{prec}_plain_dev"])
        d2s.append(np.abs(g[f"emul_{prec}_plain_hist"][1:, 2] - rh[1:, 2]))
        label = f"{prec} operand rounding"
    model = devs[0]
    hz = horizon(model, TOL[prec])
    _, hist, info, its = nfs.cg_solve_traced(c2["gp"], torch.from_numpy(c2_golden["m"]), n, precision=prec)
    its = its.cpu().numpy()
    assert info.cpu().tolist() == [n, 1]
    for k in range(1, hz + 1):
        check(its[k], ref[k - 1], TOL[prec], ("c2 CG plain", prec, k))
    bound = 4 * spread(np.max(devs, axis=0)) + TOL[prec]
    errs = np.array([rel(its[k], ref[k - 1]) for k in range(1, n + 1)])
    assert np.all(errs <= bound), (prec, errs, bound)
    h = hist.cpu().numpy()
    assert np.all(np.abs(h[1:, 1] - rh[1:, 1]) <= bound * rh[1:, 1]), "solution norm"
    assert np.all(np.abs(h[1:, 2] - rh[1:, 2]) <= 4 * spread(np.max(d2s, axis=0)) + TOL[prec] * rh[1:, 2]), \
        "data residual"
    print(f"c2 CG plain {prec}: probe {label}, horizon {hz} of {n}; errors at 5, 10, 20, 30: "
          f"{errs[4]:.1e}, {errs[9]:.1e}, {errs[19]:.1e}, {errs[n - 1]:.1e} (probe {model[4]:.1e}, {model[9]:.1e}, "
          f"{model[19]:.1e}, {model[n - 1]:.1e}); FP64 plain vs exact arithmetic at {n}: "
          f"{g['plain_vs_reorth'][n - 1]:.1e}")
    assert hz >= 1


# ------------------------------------------ phases beyond the raw sin/cos range
@pytest.fixture(scope="module")
def big_phase(nfs):
    """A problem whose phase bound sum_b max|a_b| max|h_b| / 2pi exceeds the
    128 revolutions up to which the kernels feed the phase straight to the
    hardware sine/cosine: above it they reduce it with v_fract first (the
    paper's 219 x 219 field of view at Nyquist with +-150 Hz off-resonance
    comes close to that bound)."""
    d = synth.random_problem(1000, 1500, 5, 7, seed=41, phase_scale=380.0, b0_hz=300.0)
    tb = np.max(np.abs(d["t"].astype(np.float64))) * np.max(np.abs(d["b0"].astype(np.float64)))
    bound = (tb + sum(np.max(np.abs(d["kcoef"][:, b].astype(np.float64))) * np.max(np.abs(d["fields"][b]))
                      for b in range(d["n_basis"]))) / (2 * np.pi)
    assert 160 < bound < 256, bound  # v_fract branch taken; hardware range 256
    d["bound"] = bound
    d["gp"] = gpu_problem(nfs, d)
    d["E_ref"] = oracle.apply_E(d["rho"], *args(d))
    d["EH_ref"] = oracle.apply_EH(d["m"], *args(d))
    d["EHE_ref"] = oracle.apply_EHE(d["rho"], *args(d))
    d["cg_ref"] = oracle.cg_solve(d["m"], *args(d), n_iter=6)
    return d


@pytest.mark.parametrize("prec", PRECS)
def test_phase_beyond_raw_range(nfs, big_phase, prec):
    d = big_phase
    gp = d["gp"]
    m = nfs.apply_E(gp, torch.from_numpy(d["rho"]), prec).cpu().numpy()
    x = nfs.apply_EH(gp, torch.from_numpy(d["m"]), prec).cpu().numpy()
    q = nfs.apply_EHE(gp, torch.from_numpy(d["rho"]), prec).cpu().numpy()
    rho, _, info = nfs.cg_solve(gp, torch.from_numpy(d["m"]), 6, precision=prec)
    e = [check(m, d["E_ref"], TOL[prec], "E"), check(x, d["EH_ref"], TOL[prec], "EH"),
         check(q, d["EHE_ref"], TOL[prec], "EHE"), check(rho.cpu().numpy(), d["cg_ref"]["rho"], TOL[prec], "CG")]
    assert info.cpu().tolist() == [6, 1]
    print(f"phase bound {d['bound']:.0f} rev, {prec}: " + " ".join(f"{a:.1e}/{b:.1e}" for a, b in e))


def test_phase_beyond_raw_range_resident(nfs, big_phase):
    """The resident-P build takes the same v_fract branch."""
    d = big_phase
    rho_r, _, info = nfs.cg_solve_resident(d["gp"], torch.from_numpy(d["m"]), 6)
    rho_s, _, _ = nfs.cg_solve(d["gp"], torch.from_numpy(d["m"]), 6, precision="fp16")
    assert info.cpu().tolist() == [6, 1]
    e = check(rho_r.cpu().numpy(), d["cg_ref"]["rho"], TOL["fp16"], "resident CG")
    print(f"phase bound {d['bound']:.0f} rev, resident fp16 CG: {e[0]:.1e}/{e[1]:.1e}; "
          f"split vs resident {rel(rho_r.cpu().numpy(), rho_s.cpu().numpy()):.1e}")
