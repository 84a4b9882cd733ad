"""Write the stored oracle results used by the full-size GPU checks.

Calls only the FP64 oracle and the seeded input generators.  Every target
builds its data as the tests do: m = E rho_phantom + noise at SNR 30, with
E the oracle's.

  c2      tests/golden/c2_cg.npz: the 2D 128x128 / 16-coil / 60000-sample /
          16-term workload, 30 CG iterations, plain recurrences ("plain_*")
          and re-orthogonalised ones ("reorth_*"):
            <kind>_rho        iterate 30 (complex64 copy of the FP64 result)
            <kind>_it_<n>     iterate n for n in <kind>_iters (complex64)
            <kind>_hist       per-iteration ||r_n||, ||rho_n||, ||d_n||^2
            plain_vs_reorth   [30] relative L2 distance of plain iterate n
                              from re-orthogonalised iterate n (FP64 both)
            plain_its         every plain iterate 1..30 (complex64)
            probe_deltas, probe_dev [delta][iterate], probe_hist: the plain
                              trajectory under relative noise delta on every
                              E^H E p (distance from the plain iterates,
                              histories)
            emul_<fmt>_plain_dev, _hist: the same under the FP16 / BF16
                              forms' operand rounding
            m_rms, sigma      data scale and noise level          (~80 min)
  c2mask  tests/golden/c2mask_cg.npz: the same workload restricted to its
          reconstruction mask (phantom support dilated by 2 voxels), same
          data; every plain iterate 1..30 (plain_its [30][Lm] complex64), the
          re-orthogonalised iterates listed in reorth_iters, both histories,
          plain_vs_reorth, mask (bool [L]), and the plain trajectory's
          rounding sensitivity (probe_deltas, probe_dev [delta][iterate]:
          distance from the plain iterates when every E^H E p is perturbed
          by relative noise delta; probe_hist [delta]: those runs' histories)
          and the same probe on the re-orthogonalised trajectory
          (reorth_probe_dev, reorth_probe_maxdev [delta][iterate]: relative L2
          and largest-element distances); and both solves with the FP16 and
          BF16 forms' operand rounding (emul_<fmt>_<kind>_dev, _maxdev
          [iterate], _hist)                                         (~45 min)
  c3s     tests/golden/c3s_cg.npz: the scaled 3D workload (48x48x24, 8 coils,
          4 x 8000 samples, 16 terms), 15 iterations, same keys as c2
                                                                   (~10 min)
  c3ehe   tests/golden/c3_ehe_sampled.npz: the 3D 96x96x48 / 32-coil /
          572000-sample workload, q = E^H E p for p = the phantom, at
          n_vox_sampled seeded voxels (vox [n], q [n] complex128); the full
          E p is formed, so this is one full-size E                 (~35 min)
  c3cg    tests/golden/c3_cg_noise.npz: the same workload's re-orthogonalised FP64
          CG on E^H E rho = E^H m with m = its unit coil noise, 3 iterations:
          it_<k> (iterate k at the seeded voxels vox), norms [k] (||rho_k||),
          rho (iterate 3, all voxels, complex64), hist          (~2-3 hours)
  batch24 tests/golden/batch24_cg.npz: the 24-slice batched workload (full
          phase bases), 30 re-orthogonalised iterations per slice; per slice
          s: vox_<s> (sampled voxel indices), rho_<s> (complex128 at those
          voxels), norm_<s> (||rho_30||)                            (~35 min)

Run: python tests/golden/make_golden.py <target> [<target> ...]
"""
import os
import sys
import time

# the oracle parallelises over sample blocks itself; one BLAS thread per block
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

N_VOX_SAMPLED = 1536
PROBE_DELTAS = [1e-6, 2e-6, 5e-6, 1e-5, 3e-5, 1e-4, 3e-4, 1e-3]
N_VOX_SLICE = 512


def args_of(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


def noisy_data(d):
    """m = E rho_phantom + complex Gaussian noise at SNR 30 (oracle E)."""
    clean = oracle.apply_E(d["rho_true"], *args_of(d))
    rms = float(np.sqrt(np.mean(np.abs(clean) ** 2)))
    sigma = rms / (30 * np.sqrt(2))
    return (clean + sigma * d["noise"]).astype(np.complex64), rms, sigma


def cg_pair(d, m, n_iter, iters, t0):
    """Plain and re-orthogonalised oracle CG; the keys shared by c2 and c3s."""
    out = {}
    runs = {}
    for kind, ro in (("plain", False), ("reorth", True)):
        res = oracle.cg_solve(m, *args_of(d), n_iter=n_iter, return_iterates=True, reorth=ro)
        runs[kind] = res["iterates"]
        out[f"{kind}_rho"] = res["rho"].astype(np.complex64)
        out[f"{kind}_hist"] = res["hist"]
        out[f"{kind}_iters"] = np.array(iters[kind])
        for n in iters[kind]:
            out[f"{kind}_it_{n}"] = res["iterates"][n - 1].astype(np.complex64)
        print(f"{kind} done at {time.time() - t0:.0f} s, status {res['status']}", flush=True)
    out["plain_vs_reorth"] = np.array([np.linalg.norm(x - y) / np.linalg.norm(y)
                                       for x, y in zip(runs["plain"], runs["reorth"])])
    print("plain vs reorth: " + " ".join(f"{v:.1e}" for v in out["plain_vs_reorth"]), flush=True)
    return out, runs


def plain_probes(out, d, m, plain_its, levels, t0):
    """The plain trajectory's probes: relative noise at `levels` (seed 7) and
    the FP16 / BF16 operand rounding; deviations per iterate and histories."""
    dev, hists = [], []
    for delta in levels:
        pr = oracle.cg_solve(m, *args_of(d), n_iter=len(plain_its), return_iterates=True, perturb=(delta, 7))
        dev.append([np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(pr["iterates"], plain_its)])
        hists.append(pr["hist"])
        print(f"probe {delta:.0e} at {time.time() - t0:.0f} s: " + " ".join(f"{v:.1e}" for v in dev[-1]), flush=True)
    out["probe_deltas"] = np.array(levels)
    out["probe_dev"] = np.array(dev)
    out["probe_hist"] = np.array(hists)
    for fmt in ("fp16", "bf16"):
        pr = oracle.cg_solve(m, *args_of(d), n_iter=len(plain_its), return_iterates=True, operands=fmt)
        out[f"emul_{fmt}_plain_dev"] = np.array([np.linalg.norm(x - y) / np.linalg.norm(y)
                                                  for x, y in zip(pr["iterates"], plain_its)])
        out[f"emul_{fmt}_plain_hist"] = pr["hist"]
        print(f"{fmt} operands at {time.time() - t0:.0f} s: "
              + " ".join(f"{v:.1e}" for v in out[f"emul_{fmt}_plain_dev"]), flush=True)


def make_c2():
    t0 = time.time()
    d = synth.make_config("c2")
    m, rms, sigma = noisy_data(d)
    out, runs = cg_pair(d, m, 30, {"plain": [1, 2, 3], "reorth": [1, 5, 10, 20]}, t0)
    out["plain_its"] = np.stack(runs["plain"]).astype(np.complex64)
    plain_probes(out, d, m, runs["plain"], [1e-6, 2e-6, 5e-6], t0)
    out.update(m_rms=rms, sigma=sigma, n_iter=30)
    np.savez_compressed(os.path.join(HERE, "c2_cg.npz"), **out)
    print(f"c2 CG golden written in {time.time() - t0:.0f} s")


def make_c2mask():
    t0 = time.time()
    d = synth.make_config("c2")
    m, rms, sigma = noisy_data(d)  # rho_true vanishes outside the mask: same data
    mask = synth.reconstruction_mask(d)
    dm = synth.restrict_voxels(d, mask)
    out, runs = cg_pair(dm, m, 30, {"plain": [], "reorth": [1, 5, 10, 20, 30]}, t0)
    out["plain_its"] = np.stack(runs["plain"]).astype(np.complex64)
    # sensitivity of the plain trajectory to rounding: every E^H E p
    # perturbed by relative noise delta (the oracle's probe); probe_dev[i][n]
    # = distance of perturbed iterate n+1 from the plain one for PROBE_DELTAS[i]
    dev, hists = [], []
    for delta in PROBE_DELTAS:
        pr = oracle.cg_solve(m, *args_of(dm), n_iter=30, return_iterates=True, perturb=(delta, 7))
        dev.append([np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(pr["iterates"], runs["plain"])])
        hists.append(pr["hist"])
        print(f"probe {delta:.0e}: " + " ".join(f"{v:.1e}" for v in dev[-1]), flush=True)
    out["probe_deltas"] = np.array(PROBE_DELTAS)
    out["probe_dev"] = np.array(dev)
    out["probe_hist"] = np.array(hists)
    # the same probe on the re-orthogonalised trajectory: relative L2
    # distance and largest-element distance (over the largest element) of
    # every perturbed iterate from the unperturbed one
    rdev, rmax = [], []
    for delta in PROBE_DELTAS:
        pr = oracle.cg_solve(m, *args_of(dm), n_iter=30, return_iterates=True, perturb=(delta, 7), reorth=True)
        rdev.append([np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(pr["iterates"], runs["reorth"])])
        rmax.append([np.max(np.abs(x - y)) / np.max(np.abs(y)) for x, y in zip(pr["iterates"], runs["reorth"])])
        print(f"reorth probe {delta:.0e}: " + " ".join(f"{v:.1e}" for v in rdev[-1]), flush=True)
    out["reorth_probe_dev"] = np.array(rdev)
    out["reorth_probe_maxdev"] = np.array(rmax)
    # the operand-rounding probe: the same solves with the matrix-core
    # operands rounded as the FP16 and BF16 operand forms round them
    for fmt in ("fp16", "bf16"):
        for kind, ro in (("plain", False), ("reorth", True)):
            pr = oracle.cg_solve(m, *args_of(dm), n_iter=30, return_iterates=True, operands=fmt, reorth=ro)
            ref = runs[kind]
            out[f"emul_{fmt}_{kind}_dev"] = np.array([np.linalg.norm(x - y) / np.linalg.norm(y)
                                                       for x, y in zip(pr["iterates"], ref)])
            out[f"emul_{fmt}_{kind}_maxdev"] = np.array([np.max(np.abs(x - y)) / np.max(np.abs(y))
                                                          for x, y in zip(pr["iterates"], ref)])
            out[f"emul_{fmt}_{kind}_hist"] = pr["hist"]
            print(f"{fmt} operands, {kind}: " + " ".join(f"{v:.1e}" for v in out[f"emul_{fmt}_{kind}_dev"]),
                  flush=True)
    out.update(m_rms=rms, sigma=sigma, n_iter=30, mask=mask)
    np.savez_compressed(os.path.join(HERE, "c2mask_cg.npz"), **out)
    print(f"c2mask CG golden written in {time.time() - t0:.0f} s")


def make_c3s():
    t0 = time.time()
    d = synth.make_config("c3s")
    m, rms, sigma = noisy_data(d)
    out, _ = cg_pair(d, m, 15, {"plain": [1, 2, 3, 5], "reorth": [1, 5, 10, 15]}, t0)
    out.update(m_rms=rms, sigma=sigma, n_iter=15)
    np.savez_compressed(os.path.join(HERE, "c3s_cg.npz"), **out)
    print(f"c3s CG golden written in {time.time() - t0:.0f} s")


def make_c3ehe():
    t0 = time.time()
    d = synth.make_config("c3", with_noise=False)
    a = args_of(d)
    vox = np.sort(np.random.default_rng(2024).choice(d["L"], N_VOX_SAMPLED, replace=False))
    y = oracle.apply_E(d["rho_true"], *a, block=64)
    print(f"full E done at {time.time() - t0:.0f} s", flush=True)
    q = oracle.apply_EH(y, d["sens"][:, vox], d["fields"][:, vox], d["b0"][vox], d["kcoef"], d["t"], block=256)
    np.savez_compressed(os.path.join(HERE, "c3_ehe_sampled.npz"), vox=vox, q=q, y_norm=np.linalg.norm(y))
    print(f"c3 sampled E^H E golden written in {time.time() - t0:.0f} s")


N_C3_ITERS = 3
N_VOX_C3 = 4096


def make_c3cg():
    """The full-size 3D CG: the re-orthogonalised FP64 solve of
    E^H E rho = E^H m with m the workload's unit coil noise (no E needed for
    the data), its first iterates."""
    t0 = time.time()
    d = synth.make_config("c3")
    res = oracle.cg_solve(d["noise"], *args_of(d), n_iter=N_C3_ITERS, return_iterates=True, reorth=True, block=128)
    vox = np.sort(np.random.default_rng(2025).choice(d["L"], N_VOX_C3, replace=False))
    out = dict(n_iter=N_C3_ITERS, vox=vox, hist=res["hist"], rho=res["rho"].astype(np.complex64),
               norms=np.array([np.linalg.norm(x) for x in res["iterates"]]))
    for k, x in enumerate(res["iterates"], 1):
        out[f"it_{k}"] = x[vox].astype(np.complex64)
    np.savez_compressed(os.path.join(HERE, "c3_cg_noise.npz"), **out)
    print(f"c3 CG golden written in {time.time() - t0:.0f} s, status {res['status']}")


def make_batch24():
    t0 = time.time()
    sl = synth.batched_slices(24)
    out = {}
    for s, d in enumerate(sl):
        m, _, _ = noisy_data(d)
        res = oracle.cg_solve(m, *args_of(d), n_iter=30, reorth=True)
        vox = np.sort(np.random.default_rng(500 + s).choice(d["L"], N_VOX_SLICE, replace=False))
        out[f"vox_{s}"] = vox
        out[f"rho_{s}"] = res["rho"][vox]
        out[f"norm_{s}"] = np.linalg.norm(res["rho"])
        print(f"slice {s} ({d['dims'][0]}^2, {d['n_coil']} coils, {d['K']} samples) done at "
              f"{time.time() - t0:.0f} s, status {res['status']}", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch24_cg.npz"), **out)
    print(f"batch24 CG golden written in {time.time() - t0:.0f} s")


TARGETS = {"c2": make_c2, "c2mask": make_c2mask, "c3s": make_c3s, "c3ehe": make_c3ehe, "c3cg": make_c3cg,
           "batch24": make_batch24}


def main():
    names = sys.argv[1:] or ["c2"]
    for n in names:
        if n not in TARGETS:
            raise SystemExit(f"unknown target {n}; choose from {sorted(TARGETS)}")
    for n in names:
        TARGETS[n]()


if __name__ == "__main__":
    main()
