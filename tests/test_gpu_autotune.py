"""GPU checks of the encode-shape autotuner: the chosen shapes are valid and
are the ones later calls use, and E, E^H, E^H E and CG after tuning still
match the FP64 oracle (tuning changes only the order of the split sums).
Shapes here are unique to this file so the tuned entries do not reach the
problems of other test files."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-3, "fp16": 2e-3}


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.context(0)
    return mod


@pytest.fixture(scope="module")
def prob(nfs):
    d = synth.random_problem(1520, 2650, 11, 16, seed=77, phase_scale=8.0)
    a = (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
    d["E_ref"] = oracle.apply_E(d["rho"], *a)
    d["EH_ref"] = oracle.apply_EH(d["m"], *a)
    d["EHE_ref"] = oracle.apply_EHE(d["rho"], *a)
    d["gp"] = nfs.Problem(*a)
    return d


@pytest.mark.parametrize("prec", ["fp16", "fp32", "bf16"])
def test_autotune_then_operators_match_oracle(nfs, prob, prec):
    gp = prob["gp"]
    before = nfs.tuned_shape(gp, prec)
    rho = torch.from_numpy(prob["rho"])
    m = torch.from_numpy(prob["m"])
    e0 = nfs.apply_E(gp, rho, prec).cpu().numpy()
    shapes = nfs.autotune(gp, prec)
    print(f"autotune {prec}: default {before} -> tuned {shapes}")
    for k in ("E", "EH"):
        mt, ns = shapes[k]
        assert mt in (2, 4) and ns >= 1
    assert nfs.tuned_shape(gp, prec) == shapes
    e1 = nfs.apply_E(gp, rho, prec).cpu().numpy()
    eh = nfs.apply_EH(gp, m, prec).cpu().numpy()
    ehe = nfs.apply_EHE(gp, rho, prec).cpu().numpy()
    errs = [rel(e1, prob["E_ref"]), rel(eh, prob["EH_ref"]), rel(ehe, prob["EHE_ref"])]
    print(f"after tuning {prec}: E {errs[0]:.2e} EH {errs[1]:.2e} EHE {errs[2]:.2e}; E before/after {rel(e1, e0):.1e}")
    assert max(errs) < TOL[prec]
    # deterministic under the tuned shape
    assert np.array_equal(nfs.apply_E(gp, rho, prec).cpu().numpy(), e1)


def test_autotune_then_cg_matches_oracle(nfs, prob):
    gp = prob["gp"]
    nfs.autotune(gp, "fp32")
    n_iter = 6
    rho, hist, info = nfs.cg_solve(gp, torch.from_numpy(prob["m"]), n_iter, precision="fp32", reorth=True)
    a = (prob["sens"], prob["fields"], prob["b0"], prob["kcoef"], prob["t"])
    ref = oracle.cg_solve(prob["m"], *a, n_iter, reorth=True)
    e = rel(rho.cpu().numpy(), ref["rho"])
    print(f"CG after tuning fp32: rel {e:.2e}")
    assert e < 1e-4
    assert info.cpu().tolist()[0] == n_iter


def test_autotune_batched_then_batched_solve(nfs):
    sl = synth.batched_slices(5, seed=9, n_range=(20, 44), g_range=(2, 20), k_range=(900, 3200))
    a = [(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"]) for d in sl]
    probs = [nfs.Problem(*x) for x in a]
    ms = []
    for d, x in zip(sl, a):
        clean = oracle.apply_E(d["rho_true"], *x)
        sig = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30 * np.sqrt(2))
        ms.append((clean + sig * d["noise"]).astype(np.complex64))
    shapes = nfs.autotune_batched(probs, "fp32")
    print("batch-tuned shapes:", shapes)
    for sh in shapes:
        for k in ("E", "EH"):
            assert sh[k][0] in (2, 4) and sh[k][1] >= 1
    rb, hb, ib = nfs.cg_solve_batched(probs, [torch.from_numpy(m) for m in ms], 8, precision="fp32", reorth=True)
    torch.cuda.synchronize()
    for i in (0, 2):
        ref = oracle.cg_solve(ms[i], *a[i], n_iter=8, reorth=True)
        e = rel(rb[i].cpu().numpy(), ref["rho"])
        print(f"batch-tuned slice {i}: rel {e:.2e}")
        assert e < 1e-4
    # a single solve of a slice uses the same tuned shapes: bit-identical
    r1, _, _ = nfs.cg_solve(probs[1], torch.from_numpy(ms[1]), 8, precision="fp32", reorth=True)
    assert torch.equal(r1.cpu(), rb[1].cpu())


@pytest.mark.parametrize("shape", [(2, 1), (4, 3), (2, 64)])
def test_pinned_shape_is_used_and_matches_oracle(nfs, shape):
    """nfs_set_shape: the pinned shape is the one later calls report and use
    (a split count above the streamed chunk count leaves empty splits), and
    the operators still match the oracle."""
    d = synth.random_problem(700, 1300, 6, 9, seed=79, phase_scale=8.0)
    a = (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
    gp = nfs.Problem(*a)
    mt, ns = shape
    for op in ("E", "EH"):
        nfs.set_shape(gp, "fp16", op, mt, ns)
    assert nfs.tuned_shape(gp, "fp16") == {"E": shape, "EH": shape}
    e1 = rel(nfs.apply_E(gp, torch.from_numpy(d["rho"]), "fp16").cpu().numpy(), oracle.apply_E(d["rho"], *a))
    e2 = rel(nfs.apply_EHE(gp, torch.from_numpy(d["rho"]), "fp16").cpu().numpy(), oracle.apply_EHE(d["rho"], *a))
    print(f"pinned shape {shape}: E {e1:.1e}, EHE {e2:.1e}")
    assert max(e1, e2) < TOL["fp16"]
    with pytest.raises(nfs.NfsError):
        nfs.set_shape(gp, "fp16", "E", 3, 2)
