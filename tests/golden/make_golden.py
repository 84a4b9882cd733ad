"""Write the stored oracle results used by the full-size GPU checks.

Calls only the FP64 oracle and the seeded input generators.  Output
tests/golden/c2_cg.npz, for the 2D 128x128 / 16-coil / 60000-sample /
16-term workload with data m = E rho_phantom + noise (SNR 30), 30 CG
iterations, for the plain recurrences ("plain_*") and for the
re-orthogonalised ones ("reorth_*"):
  <kind>_rho        -- iterate 30 (complex64 copy of the FP64 result)
  <kind>_it_<n>     -- iterate n for n in ``<kind>_iters`` (complex64 copies)
  <kind>_hist       -- per-iteration ||r_n||, ||rho_n||, ||d_n||^2 (float64)
  plain_vs_reorth   -- [30] relative L2 distance of plain iterate n from
                       re-orthogonalised iterate n (FP64 both)
  m_rms, sigma      -- data scale and noise level
Run: python tests/golden/make_golden.py   (about 16 min on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

ITERS = {"plain": [1, 2, 3], "reorth": [1, 5, 10, 20]}
N_ITER = 30


def c2_data():
    d = synth.make_config("c2")
    a = (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
    clean = oracle.apply_E(d["rho_true"], *a)
    rms = float(np.sqrt(np.mean(np.abs(clean) ** 2)))
    sigma = rms / (30 * np.sqrt(2))
    m = (clean + sigma * d["noise"]).astype(np.complex64)
    return d, a, m, rms, sigma


def main():
    t0 = time.time()
    d, a, m, rms, sigma = c2_data()
    out = dict(m_rms=rms, sigma=sigma, n_iter=N_ITER)
    runs = {}
    for kind, ro in (("plain", False), ("reorth", True)):
        res = oracle.cg_solve(m, *a, n_iter=N_ITER, return_iterates=True, reorth=ro)
        runs[kind] = res["iterates"]
        out[f"{kind}_rho"] = res["rho"].astype(np.complex64)
        out[f"{kind}_hist"] = res["hist"]
        out[f"{kind}_iters"] = np.array(ITERS[kind])
        for n in ITERS[kind]:
            out[f"{kind}_it_{n}"] = res["iterates"][n - 1].astype(np.complex64)
        print(f"{kind} done at {time.time() - t0:.0f} s, status {res['status']}", flush=True)
    out["plain_vs_reorth"] = np.array([np.linalg.norm(x - y) / np.linalg.norm(y)
                                       for x, y in zip(runs["plain"], runs["reorth"])])
    print("plain vs reorth: " + " ".join(f"{v:.1e}" for v in out["plain_vs_reorth"]))
    np.savez_compressed(os.path.join(HERE, "c2_cg.npz"), **out)
    print(f"c2 CG golden written in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
