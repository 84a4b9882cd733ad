"""The 2D workload restricted to its reconstruction mask (the voxel set the
paper solves for), through the C ABI, against the stored FP64 oracle solves
(tests/golden/c2mask_cg.npz, oracle only).

The recurrences as printed (plain CG) are compared with the FP64 plain
solve at every iterate up to the horizon where that trajectory is stable
under the GPU's rounding: the golden file holds the oracle's sensitivity
probe (every E^H E p perturbed by relative noise delta) for several delta;
the test measures the GPU's E^H E error on this problem and takes the
horizon of the smallest stored delta at least twice that error, as the last
iterate the probe keeps within a quarter of the bar.  Past the horizon the
iterates depend on rounding at any precision (the FP64 plain solve itself
leaves the exact-arithmetic trajectory, see plain_vs_reorth), so they are
held to the spread that rounding of that size gives in the oracle: at every
iterate the distance from the FP64 plain iterate, and the data-residual and
solution-norm histories, within four times the probe's own deviation (plus
the bar).  The re-orthogonalised solve is compared at every stored iterate.
Both parity measures of tests/_parity.py.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import PRECS, TOL, check, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nfs():
    from paper_2604_09233_amd import nfs as mod

    assert torch.cuda.is_available()
    mod.context(0)
    return mod


def args(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


@pytest.fixture(scope="module")
def c2mask(nfs):
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2mask_cg.npz"))
    d = synth.make_config("c2")
    mask = synth.reconstruction_mask(d)
    assert np.array_equal(mask, g["mask"])
    clean = oracle.apply_E(d["rho_true"], *args(d))
    sigma = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30 * np.sqrt(2))
    m = (clean + sigma * d["noise"]).astype(np.complex64)
    dm = synth.restrict_voxels(d, mask)
    p = np.random.default_rng(5).standard_normal(dm["L"]) + 1j * np.random.default_rng(6).standard_normal(dm["L"])
    p = p.astype(np.complex64)
    return dict(g=g, d=dm, m=m, gp=nfs.Problem(*args(dm)), p=p, ehe_ref=oracle.apply_EHE(p, *args(dm)))


def probe_index(g, delta):
    """Index of the smallest stored probe delta >= `delta`."""
    ds = g["probe_deltas"]
    idx = [i for i in range(len(ds)) if ds[i] >= delta]
    assert idx, ("operator error beyond the stored probes", delta)
    return idx[0]


def horizon(g, i, tol):
    """Last iterate probe i keeps within tol / 4."""
    dev = g["probe_dev"][i]
    hz = 0
    while hz < len(dev) and dev[hz] <= tol / 4:
        hz += 1
    return hz


@pytest.mark.parametrize("prec", PRECS)
def test_c2mask_plain_cg_every_iterate_to_horizon(nfs, c2mask, prec):
    g, gp = c2mask["g"], c2mask["gp"]
    q = nfs.apply_EHE(gp, torch.from_numpy(c2mask["p"]), prec).cpu().numpy()
    delta = 2 * rel(q, c2mask["ehe_ref"])
    i = probe_index(g, delta)
    hz = horizon(g, i, TOL[prec])
    n = int(g["n_iter"])
    _, hist, info, its = nfs.cg_solve_traced(gp, torch.from_numpy(c2mask["m"]), n, precision=prec)
    its = its.cpu().numpy()
    assert info.cpu().tolist() == [n, 1]
    errs = [check(its[k], g["plain_its"][k - 1], TOL[prec], ("c2mask plain", prec, k)) for k in range(1, hz + 1)]
    # past the horizon: within the spread the oracle's probe shows for
    # rounding of this size (iterates, data residual, solution norm)
    dev = g["probe_dev"][i]
    for k in range(hz + 1, n + 1):
        e = rel(its[k], g["plain_its"][k - 1])
        assert e <= 4 * dev[k - 1] + TOL[prec], ("c2mask plain spread", prec, k, e, dev[k - 1])
    h = hist.cpu().numpy()
    ref, ph = g["plain_hist"], g["probe_hist"][i]
    for col in (1, 2):
        spread = np.abs(ph[1:, col] - ref[1:, col])
        assert np.all(np.abs(h[1:, col] - ref[1:, col]) <= 4 * spread + TOL[prec] * ref[1:, col]), col
    last = rel(its[n], g["plain_its"][n - 1])
    print(f"c2mask plain {prec}: E^H E error {delta / 2:.1e}, probe delta {g['probe_deltas'][i]:.0e}, horizon {hz} "
          f"of {n}; worst rel/max up to it "
          f"{max((e[0] for e in errs), default=0):.1e}/{max((e[1] for e in errs), default=0):.1e}; iterate {n} "
          f"rel {last:.1e} (FP64 plain vs exact arithmetic there {g['plain_vs_reorth'][n - 1]:.1e})")
    assert hz >= 1, hz


@pytest.mark.parametrize("prec", PRECS)
def test_c2mask_reorth_cg_every_stored_iterate(nfs, c2mask, prec):
    g = c2mask["g"]
    n = int(g["n_iter"])
    _, hist, info, its = nfs.cg_solve_traced(c2mask["gp"], torch.from_numpy(c2mask["m"]), n, precision=prec,
                                             reorth=True)
    its = its.cpu().numpy()
    assert info.cpu().tolist() == [n, 1]
    errs = [check(its[int(k)], g[f"reorth_it_{int(k)}"], TOL[prec], ("c2mask reorth", prec, int(k)))
            for k in g["reorth_iters"]]
    h = hist.cpu().numpy()
    assert np.max(np.abs(h[:, 2] - g["reorth_hist"][:, 2])) < TOL[prec] * g["reorth_hist"][0, 2]
    print(f"c2mask reorth {prec}: " + " ".join(f"{a:.1e}/{b:.1e}" for a, b in errs))
