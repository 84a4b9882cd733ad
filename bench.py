#!/usr/bin/env python3
"""Benchmark of the non-Fourier SENSE hot path on one MI355X.

One step = one full CG solve (setup, E^H m, n_iter iterations of E^H E with
the FP64 scalar updates and residual re-orthogonalisation) on the 3D
96x96x48 / 32-coil / 16 x 35750-sample / 16-field-term workload (15
iterations; the largest configuration), inputs resident in HBM, replayed
from a captured hipGraph (the library's graph mode).  Encode-kernel shapes
are autotuned before timing.

Reported value: E^H E voxel*sample*coil per second over the solve, i.e.
(n_iter + 1/2) * L * K * G / (solve time), the initial E^H m counting as half
an application.  ms_per_step is the CG solve time.

Accuracy.  A full 15-iteration FP64 oracle CG of the 3D workload takes many
hours on the host, so rel_err_vs_oracle is null; beside it go the errors
against stored FP64 oracle values that the tests also use: the scaled 3D
case's CG iterate (48x48x24, 8 coils, 4 x 8000 samples, 15 iterations;
tests/golden/c3s_cg.npz), E^H E of the phantom at 1536 voxels of the full
workload (tests/golden/c3_ehe_sampled.npz), and the third iterate of the
full-size CG with the workload's unit coil noise as data, at every voxel
(tests/golden/c3_cg_noise.npz).

Roofline: the fused encode kernel (phase tile, sin/cos, complex contraction),
its average launch duration from HIP events on its launch stream over an
eager pass of the same solve, against the peak of the pipe whose peak-rate
time for the launch's work is the larger (the matrix cores for the 3D
workload's 32 coils; see roofline()), with both pipes' fractions and the
HBM traffic per launch from the committed counter summary.

Side measurements: the BF16 and FP32 operand forms; one E^H E alone; the 2D
128x128 workload (all forms, the compressed phase basis with its setup
charged, the resident-P form, the plain recurrences, the plain and
re-orthogonalised solves inside the reconstruction mask, the
stopping-criteria study, the k-space filter); the 24-slice batch; the map estimation on the
paper's prescan geometry; the FP64 CPU oracle on a bounded sample of the
headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published / derived peaks.  Transcendental ops (v_sin_f32,
# v_cos_f32): a wave64 instruction occupies a SIMD for 8 clocks, i.e.
# 256 CUs x 4 SIMDs x 8 lanes per clock x 2.4 GHz = 1.966e13 ops/s.
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3}
N_CU, SIMD_PER_CU, TRANS_LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 8, 2.4
TRANS_PEAK = N_CU * SIMD_PER_CU * TRANS_LANES_PER_SIMD * CLOCK_GHZ * 1e9
GOLDEN = os.path.join(ROOT, "tests", "golden")

WORKLOADS = {
    "c3": "c3: 3D 96x96x48, 32 coils, 16 x 35750-sample tilted spiral shots (R~7), 16 field terms, B0 +-150 Hz, "
          "15 CG iterations, re-orthogonalised (one step = one CG solve)",
    "c2": "c2: 2D 128x128, 16 coils, 4 x 15000-sample R=4 spiral, 16 field terms, B0 +-100 Hz, 30 CG iterations, "
          "re-orthogonalised (one step = one CG solve)",
}


def progress(msg):
    """One line on stderr as each measurement leg starts (the JSON result is
    the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp16", choices=["fp16", "bf16", "fp32"])
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other operand forms of the headline")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D 128x128 side measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 24-slice batched-solve measurement")
    ap.add_argument("--no-tune", action="store_true", help="use the default encode shapes instead of autotuned ones")
    ap.add_argument("--no-maps", action="store_true", help="skip the sensitivity / B0 map-estimation measurement")
    ap.add_argument("--plain", action="store_true", help="plain CG recurrences (no re-orthogonalisation)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one solve of the headline workload only, for counter collection")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every solve eagerly instead of replaying it from a captured hipGraph")
    ap.add_argument("--shapes", default=None,
                    help="encode shapes of the headline workload at --precision instead of autotuning, "
                         "'E:<held tiles>:<splits>,EH:<held tiles>:<splits>' (as the autotuner reports them)")
    return ap.parse_args()


def apply_shapes(nfs, prob, precision, spec):
    """Pin the encode shapes given as 'E:4:2,EH:4:3'."""
    for part in spec.split(","):
        op, mt, ns = part.split(":")
        nfs.set_shape(prob, precision, op, int(mt), int(ns))


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def golden(name):
    p = os.path.join(GOLDEN, name)
    return np.load(p) if os.path.exists(p) else None


def cpu_baseline(d, stride):
    """FP64 oracle E^H E on every `stride`-th sample (all voxels, all coils),
    repeated for at least 10 s of wall time; returns v*s*c/s."""
    import oracle

    ks = np.arange(0, d["K"], stride)
    a = (d["sens"], d["fields"], d["b0"], d["kcoef"][ks], d["t"][ks])
    x = d["rho_true"]
    work = 0.0
    t0 = time.perf_counter()
    while True:
        oracle.apply_EHE(x, *a)
        work += d["L"] * len(ks) * d["n_coil"]
        el = time.perf_counter() - t0
        if el >= 10.0:
            break
    return dict(value=work / el, unit="voxel*sample*coil/s", cores=os.cpu_count(), kind="oracle",
                sample=f"FP64 E^H E on every {stride}th sample ({len(ks)} of {d['K']}) x {d['L']} voxels x "
                       f"{d['n_coil']} coils of the headline workload, repeated "
                       f"{work / (d['L'] * len(ks) * d['n_coil']):.0f}x in {el:.1f} s, numpy with "
                       f"{os.cpu_count()} threads")


class Solver:
    """One workload on the GPU: problem, synthetic data (E rho_phantom with
    the library's FP32 E, plus complex noise at SNR 30) and timed solves."""

    def __init__(self, nfs, torch, dev, d, reorth):
        self.nfs, self.torch, self.dev, self.d, self.reorth = nfs, torch, dev, d, reorth
        self.prob = nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"], device=dev)
        clean = nfs.apply_E(self.prob, torch.from_numpy(d["rho_true"]).to(dev), "fp32")
        sig = float(torch.sqrt(torch.mean(torch.abs(clean) ** 2))) / (30 * np.sqrt(2))
        self.m = clean + sig * torch.from_numpy(d["noise"]).to(dev)
        del clean
        torch.cuda.synchronize()
        self.L, self.K, self.G, self.n_iter = d["L"], d["K"], d["n_coil"], d["n_iter"]

    def buffers(self, n_iter=None):
        torch, dev = self.torch, self.dev
        n = self.n_iter if n_iter is None else n_iter
        return (torch.empty(self.L, dtype=torch.complex64, device=dev),
                torch.full((n + 1, 3), float("nan"), dtype=torch.float64, device=dev),
                torch.zeros(2, dtype=torch.int32, device=dev))

    def time_solves(self, prec, steps, warmup, graphs=True, prob=None, data=None, reorth=None):
        """Mean ms per solve over `steps` after `warmup`; data(): the CG
        right-hand side, called inside the timed region."""
        nfs, torch = self.nfs, self.torch
        prob = self.prob if prob is None else prob
        data = (lambda: self.m) if data is None else data
        reorth = self.reorth if reorth is None else reorth
        out, hist, info = self.buffers()
        nfs.set_graphs(0, graphs)
        try:
            for _ in range(warmup):
                nfs.cg_solve(prob, data(), self.n_iter, precision=prec, reorth=reorth, out=out, hist=hist, info=info)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            ev0.record()
            for _ in range(steps):
                nfs.cg_solve(prob, data(), self.n_iter, precision=prec, reorth=reorth, out=out, hist=hist, info=info)
            ev1.record()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        finally:
            nfs.set_graphs(0, False)
        return out, hist, info, ev0.elapsed_time(ev1) / steps, wall

    def kernel_times(self, prec, solves=1, prob=None):
        """Encode-kernel launch durations (HIP events on the launch stream,
        the library's profiling hook) over eager solves."""
        nfs, torch = self.nfs, self.torch
        prob = self.prob if prob is None else prob
        out, hist, info = self.buffers()
        nfs.cg_solve(prob, self.m, self.n_iter, precision=prec, reorth=self.reorth, out=out, hist=hist, info=info)
        torch.cuda.synchronize()
        nfs.profile_enable(0, True)
        nfs.profile_read(0, "E")
        nfs.profile_read(0, "EH")
        for _ in range(solves):
            nfs.cg_solve(prob, self.m, self.n_iter, precision=prec, reorth=self.reorth, out=out, hist=hist, info=info)
        torch.cuda.synchronize()
        kt = {k: nfs.profile_read(0, k) for k in ("E", "EH")}
        nfs.profile_enable(0, False)
        return kt

    def ehe_alone(self, prec, reps):
        nfs, torch = self.nfs, self.torch
        p = torch.from_numpy(self.d["rho_true"]).to(self.dev)
        q = torch.empty_like(p)
        for _ in range(3):
            nfs.apply_EHE(self.prob, p, prec, out=q)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nfs.apply_EHE(self.prob, p, prec, out=q)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times)), q


def phase_instrs(P):
    return -(-3 * (P + 1) // 32)


def col_blocks(G):
    return {1: 1, 2: 2, 3: 4, 4: 4}.get(-(-2 * G // 16), 8)


def roofline(kt, L, K, G, P, prec, counters_md):
    """Roofline object of the dominant encode launch (E or E^H).  The kernel
    keeps two pipes busy: the matrix cores (phase tile and contraction) and
    the VALU, whose transcendental unit takes one sin and one cos per
    voxel-sample pair.  The bound is the pipe whose peak-rate time for the
    launch's work is the larger: the matrix cores for the MFMA instructions
    the kernel issues, at the dense f16 peak, or the transcendental unit for
    its 2 sin/cos per pair (the matrix cores at 32 coils, where a 16 x 16
    tile takes six matrix-core instructions; at 16 coils, four, the two
    times are within 1 % and the matrix cores' is the larger).  For "mfma", achieved = the algorithmic contraction and
    phase flops (8 G + 2 (P + 1) per pair) over the launch's mean duration
    against the 2.5 PFLOP/s dense peak; for "alu", the 2 sin/cos per pair
    against the transcendental peak.  Both pipes' fractions are reported."""
    from paper_2604_09233_amd.profile_summary import read_traffic

    n_e, ms_e = kt["E"]
    n_h, ms_h = kt["EH"]
    kname, n_k, ms_k = ("EH", n_h, ms_h) if ms_h >= ms_e else ("E", n_e, ms_e)
    avg_ms = ms_k / max(n_k, 1)
    t = avg_ms * 1e-3
    pairs = L * K  # voxel-sample pairs per launch
    trans = 2 * pairs / t
    # MFMA instructions issued per 16 x 16 tile (256 pairs): ceil(3 (P+1) /
    # 32) f16 16x16x32 phase instructions, and per 16-column block of the 2G
    # real columns one f16 (fp16), two bf16 (bf16: hi and lo data parts) or
    # three f16 (fp32: split operands) 16x16x32 contraction instructions
    tiles = pairs / 256.0
    exec_flops = tiles * 16384 * (phase_instrs(P) + col_blocks(G) * {"fp16": 1, "bf16": 2, "fp32": 3}[prec])
    mfma_peak = MFMA_PEAK_TFLOPS["fp16"] * 1e12
    algo_flops = pairs * (8 * G + 2 * (P + 1))
    trans_frac = trans / TRANS_PEAK
    mfma_busy = exec_flops / mfma_peak / t
    tr = read_traffic(os.path.join(ROOT, "profiles", counters_md))
    out = dict(traffic=(tr or {}).get(kname), traffic_unit="bytes per launch", kernel=f"encode_kernel ({kname})",
               avg_launch_ms=avg_ms, launches=n_k, mfma_pipe_frac=mfma_busy, transcendental_frac=trans_frac,
               algorithmic_flops_per_launch=algo_flops, executed_mfma_flops_per_launch=exec_flops,
               encode_kernel_ms={"E": ms_e / max(n_e, 1), "EH": ms_h / max(n_h, 1)})
    if mfma_busy > trans_frac:
        out.update(bound="mfma", achieved=algo_flops / t / 1e12, peak=mfma_peak / 1e12, unit="TFLOP/s",
                   frac=algo_flops / t / mfma_peak)
    else:
        out.update(bound="alu", achieved=trans / 1e12, peak=TRANS_PEAK / 1e12, unit="Tsincos-ops/s",
                   frac=trans_frac, algorithmic_mfma_frac=algo_flops / t / mfma_peak)
    return out


def c3_oracle_checks(nfs, synth, torch, dev, prec, sv, reorth):
    """Errors against the stored FP64 oracle values of the 3D workloads: E^H E
    of the phantom at the stored voxels of the full workload, the CG iterates
    of the scaled 3D case (data from the library's FP32 E, which differs from
    the oracle-built data by ~1e-6 relative), and the first iterates of the
    full-size CG with the workload's unit coil noise as data."""
    out = {}
    g = golden("c3_ehe_sampled.npz")
    if g is not None:
        _, q = sv.ehe_alone(prec, 1)
        q = q.cpu().numpy()[g["vox"]]
        out["c3_EHE_sampled"] = dict(voxels=int(len(g["vox"])), rel=rel(q, g["q"]), max_rel=max_rel(q, g["q"]))
    g = golden("c3s_cg.npz")
    if g is not None:
        s = Solver(nfs, torch, dev, synth.make_config("c3s"), reorth)
        kind = "reorth" if reorth else "plain"
        n = int(g["n_iter"])
        rho, _, _ = nfs.cg_solve(s.prob, s.m, n, precision=prec, reorth=reorth)
        ref = g[f"{kind}_rho"]
        out["c3s_cg"] = dict(workload="3D 48x48x24, 8 coils, 4 x 8000 samples, 16 terms, 15 iterations",
                             iterate=n, rel=rel(rho.cpu().numpy(), ref), max_rel=max_rel(rho.cpu().numpy(), ref))
    g = golden("c3_cg_noise.npz")
    if g is not None:
        # the full-size re-orthogonalised CG with the workload's unit coil
        # noise as data, at the last stored iterate, every voxel
        n = int(g["n_iter"])
        rho, _, _ = nfs.cg_solve(sv.prob, torch.from_numpy(sv.d["noise"]).to(dev), n, precision=prec, reorth=True)
        x = rho.cpu().numpy()
        out["c3_cg_full_size"] = dict(data="unit coil noise", iterate=n, voxels=int(len(x)), rel=rel(x, g["rho"]),
                                      max_rel=max_rel(x, g["rho"]))
    return out


def threed_kspace_filter(nfs, torch, dev, d, rho):
    """The paper's k-space filter on the 3D reconstruction: bins inside the
    hull of the first-order k positions (x, y, z terms)."""
    t0 = time.perf_counter()
    f = nfs.kspace_filter_mask(d["kcoef"][:, 1:4].astype(np.float64) / np.pi, d["dims"])
    ms_mask = (time.perf_counter() - t0) * 1e3
    f_dev = torch.from_numpy(f).to(dev)
    nfs.apply_kspace_filter(rho, f_dev, d["dims"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out_f = nfs.apply_kspace_filter(rho, f_dev, d["dims"])
    e1.record()
    torch.cuda.synchronize()
    ref_img = torch.from_numpy(d["rho_true"])
    return dict(bins_inside=int(f.sum()), bins=int(f.size), ms_mask_host=ms_mask, ms_apply=e0.elapsed_time(e1),
                ssim_vs_phantom_before=float(nfs.ssim(rho, ref_img, d["dims"]).cpu()[0]),
                ssim_vs_phantom_after=float(nfs.ssim(out_f, ref_img, d["dims"]).cpu()[0]))


def twod_run(nfs, synth, torch, dev, args):
    """The 2D 128x128 workload: the 30-iteration solve in each operand form
    against the stored FP64 oracle solves, the compressed phase basis with
    its setup (host compression, data rotation) charged, the resident-P
    (non-split) form, the plain recurrences, the solves inside the
    reconstruction mask, the 250-iteration stopping study and the k-space
    filter."""
    reorth = not args.plain
    kind = "reorth" if reorth else "plain"
    d = synth.make_config("c2")
    sv = Solver(nfs, torch, dev, d, reorth)
    L, K, G, n_iter = sv.L, sv.K, sv.G, sv.n_iter
    vsc = L * K * G
    g = golden("c2_cg.npz")
    steps = max(2, args.steps // 2)
    precs = [args.precision] + [p for p in ("fp32", "bf16") if p != args.precision]
    forms = {}
    rho_main = None
    for prec in precs:
        if not args.no_tune:
            nfs.autotune(sv.prob, prec)
        rho, _, info, ms, _ = sv.time_solves(prec, steps, 1, graphs=not args.no_graphs)
        forms[prec] = dict(ms_per_step=ms, value=(n_iter + 0.5) * vsc / (ms * 1e-3),
                           rel_err_vs_oracle=rel(rho.cpu().numpy(), g[f"{kind}_rho"]) if g is not None else None,
                           cg_info=info.cpu().tolist())
        if prec == args.precision:
            rho_main = rho.clone()
    kt = sv.kernel_times(args.precision)
    roof = roofline(kt, L, K, G, d["n_basis"], args.precision, f"encode_kernel_c2_{args.precision}_counters.md")

    # compressed phase basis: 16 solid harmonics on one slice span 10
    # functions; the compression is redone per geometry (kcoef is measured
    # per scan), so its host time is charged to an end-to-end figure
    nfs.compress_basis(sv.prob)  # first call: loads the kernels
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    cprob, theta, cinfo = nfs.compress_basis(sv.prob)
    torch.cuda.synchronize()
    t_c = (time.perf_counter() - t_c) * 1e3
    if not args.no_tune:
        nfs.autotune(cprob, args.precision)
    mbuf = torch.empty_like(sv.m)
    rho_c, _, _, ms_c, _ = sv.time_solves(args.precision, steps, 1, graphs=not args.no_graphs, prob=cprob,
                                          data=lambda: nfs.phase_shift(sv.m, theta, -1, out=mbuf))
    compressed = dict(terms=d["n_basis"] + 1, compressed_terms=cprob.P + 1, err_bound_rad=cinfo["err_bound"],
                      ms_solve=ms_c, ms_setup_host=t_c, ms_end_to_end=ms_c + t_c,
                      rel_err_vs_oracle=rel(rho_c.cpu().numpy(), g[f"{kind}_rho"]) if g is not None else None,
                      note="solve on the compressed basis with the data rotation by exp(-i theta) inside the step; "
                           "ms_setup_host = wall time of nfs_compress_basis_device (FP64 on the GPU) including "
                           "the one synchronisation that reads the kept term count back")
    del rho_c

    # non-split form: P built once per solve (2 K L x 4 bytes), streamed by every E and E^H
    resident = None
    if args.precision == "fp16":
        def t_res(n):
            o, h, f = sv.buffers(n)
            nfs.cg_solve_resident(sv.prob, sv.m, n, reorth=reorth, out=o, hist=h, info=f)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nfs.cg_solve_resident(sv.prob, sv.m, n, reorth=reorth, out=o, hist=h, info=f)
            e1.record()
            torch.cuda.synchronize()
            return o, e0.elapsed_time(e1)
        # the shapes tuned for the split solve above (same shape class), so
        # that the two forms sum the same splits in the same order
        rr, ms_r = t_res(n_iter)
        _, ms_r1 = t_res(1)
        resident = dict(ms_per_step=ms_r, ms_per_iteration=(ms_r - ms_r1) / (n_iter - 1),
                        ms_build_and_first_iteration=ms_r1, P_bytes=2 * L * K * 4,
                        identical_to_split=bool(torch.equal(rr.cpu(), rho_main.cpu())),
                        rel_err_vs_oracle=rel(rr.cpu().numpy(), g[f"{kind}_rho"]) if g is not None else None)
        del rr
        sv.prob._ws.pop(("CG_RESIDENT", "fp16", n_iter, reorth), None)
        sv.prob._ws.pop(("CG_RESIDENT", "fp16", 1, reorth), None)
        torch.cuda.empty_cache()

    plain = None
    if reorth:
        rhop, _, _, msp, _ = sv.time_solves(args.precision, steps, 1, graphs=not args.no_graphs, reorth=False)
        plain = dict(ms_per_step=msp,
                     rel_err_vs_oracle_plain=rel(rhop.cpu().numpy(), g["plain_rho"]) if g is not None else None,
                     oracle_plain_vs_reorth=float(g["plain_vs_reorth"][-1]) if g is not None else None)

    # the problem the paper solves: the voxels inside the reconstruction mask
    # (the phantom's support dilated by two voxels; the same data), the
    # recurrences as printed and the re-orthogonalised solve, each against
    # its stored FP64 oracle solve at the last iterate
    mask = synth.reconstruction_mask(d)
    svm = Solver(nfs, torch, dev, synth.restrict_voxels(d, mask), reorth)
    if not args.no_tune:
        nfs.autotune(svm.prob, args.precision)
    gm = golden("c2mask_cg.npz")
    masked = dict(voxels=svm.L, note="FP64 plain recurrences leave exact-arithmetic CG on this problem "
                                      "(kappa ~ 1e14): oracle_plain_vs_reorth at the last iterate")
    for kind_m, ro in (("plain", False), ("reorth", True)):
        rho_m, _, info_m, ms_m, _ = svm.time_solves(args.precision, steps, 1, graphs=not args.no_graphs, reorth=ro)
        ref = None
        if gm is not None:
            ref = gm["plain_its"][n_iter - 1] if not ro else gm[f"reorth_it_{n_iter}"]
        masked[kind_m] = dict(ms_per_step=ms_m, value=(n_iter + 0.5) * svm.L * K * G / (ms_m * 1e-3),
                              rel_err_vs_oracle=rel(rho_m.cpu().numpy(), ref) if ref is not None else None,
                              cg_info=info_m.cpu().tolist())
    masked["oracle_plain_vs_reorth"] = float(gm["plain_vs_reorth"][n_iter - 1]) if gm is not None else None
    del svm

    # the paper's stopping-criteria study: 250 iterations, L-curve corner and
    # SSIM of every iterate against the phantom
    n_long = 250
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    _, h_long, i_long, its = nfs.cg_solve_traced(sv.prob, sv.m, n_long, precision=args.precision, reorth=reorth)
    ev[1].record()
    ss = nfs.ssim(its[1:], torch.from_numpy(d["rho_true"]), d["dims"])
    ev[2].record()
    torch.cuda.synchronize()
    ss = ss.cpu().numpy()
    corner, _ = nfs.lcurve_corner(h_long)
    stopping = dict(iterations=n_long, ms_solve=ev[0].elapsed_time(ev[1]), ms_ssim_all=ev[1].elapsed_time(ev[2]),
                    peak_ssim=float(ss.max()), peak_ssim_iteration=int(np.argmax(ss)) + 1,
                    ssim_at=dict((str(k), float(ss[k - 1])) for k in (5, 10, 30, 100, 250)),
                    lcurve_corner_iteration=corner, cg_info=i_long.cpu().tolist())
    del its

    # the paper's k-space filter: bins inside the hull of the first-order k
    # positions (linear x, y terms; kcoef / pi in cycles per FOV)
    f = nfs.kspace_filter_mask(d["kcoef"][:, 1:3].astype(np.float64) / np.pi, d["dims"])
    f_dev = torch.from_numpy(f).to(dev)
    nfs.apply_kspace_filter(rho_main, f_dev, d["dims"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rho_f = nfs.apply_kspace_filter(rho_main, f_dev, d["dims"])
    e1.record()
    torch.cuda.synchronize()
    ref_img = torch.from_numpy(d["rho_true"])
    kf = dict(bins_inside=int(f.sum()), bins=int(f.size), ms_apply=e0.elapsed_time(e1),
              ssim_vs_phantom_before=float(nfs.ssim(rho_main, ref_img, d["dims"]).cpu()[0]),
              ssim_vs_phantom_after=float(nfs.ssim(rho_f, ref_img, d["dims"]).cpu()[0]))
    return dict(workload=WORKLOADS["c2"], L=L, K=K, G=G, n_iter=n_iter, forms=forms, roofline=roof,
                encode_shapes=nfs.tuned_shape(sv.prob, args.precision), compressed_basis=compressed,
                resident_P=resident, plain_recurrences=plain, masked=masked, stopping_criteria=stopping,
                kspace_filter=kf)


def batched_run(nfs, synth, torch, dev, args, steps=2):
    """The 24-slice batched workload (uneven 2D slices, 8..32 coils, 8000..30000
    samples, 16 terms, per-slice B0): every slice's 30-iteration solve in one
    batched call, BF16 operands, re-orthogonalised CG, replayed from a
    captured hipGraph.  Reports whole-batch voxel*sample*coil/s."""
    sl = synth.batched_slices(24)
    probs = [nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"], device=dev) for d in sl]
    ms = []
    for d, pr in zip(sl, probs):
        clean = nfs.apply_E(pr, torch.from_numpy(d["rho_true"]), "fp32")
        sig = float(torch.sqrt(torch.mean(torch.abs(clean) ** 2))) / (30 * np.sqrt(2))
        ms.append(clean + sig * torch.from_numpy(d["noise"]).to(dev))
    n_iter = 30
    work = sum((n_iter + 0.5) * d["L"] * d["K"] * d["n_coil"] for d in sl)
    # compressed phase bases (each slice: 16 solid harmonics on one slice ->
    # 10 terms), the data rotations by exp(-i theta) inside the timed step;
    # the compression's host time per batch is reported beside it
    nfs.compress_basis(probs[0])  # first call: loads the kernels
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    comp = [nfs.compress_basis(pr) for pr in probs]
    torch.cuda.synchronize()
    t_c = (time.perf_counter() - t_c) * 1e3
    cprobs = [c[0] for c in comp]
    thetas = [c[1] for c in comp]
    bufs = [torch.empty_like(m) for m in ms]

    def timed(mode, prs):
        rot = prs is cprobs

        def data():
            if not rot:
                return ms
            return [nfs.phase_shift(m, th, -1, out=b) for m, th, b in zip(ms, thetas, bufs)]

        nfs.set_batch_mode(0, mode)
        nfs.set_graphs(0, not args.no_graphs)
        try:
            outs, hists, infos = nfs.cg_solve_batched(prs, data(), n_iter, precision="bf16", reorth=True)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(steps):
                nfs.cg_solve_batched(prs, data(), n_iter, precision="bf16", reorth=True, outs=outs, hists=hists,
                                     infos=infos)
            ev1.record()
            torch.cuda.synchronize()
        finally:
            nfs.set_graphs(0, False)
            nfs.set_batch_mode(0, "streams")
        return ev0.elapsed_time(ev1) / steps, outs

    if not args.no_tune:
        nfs.autotune_batched(probs, "bf16")
    t_f, out_f = timed("streams", probs)
    t_fp, out_fp = timed("persistent", probs)
    if not args.no_tune:
        nfs.autotune_batched(cprobs, "bf16")
    t_c_s, out_c = timed("streams", cprobs)
    t_c_p, out_cp = timed("persistent", cprobs)
    same = all(torch.equal(a, b) for a, b in zip(out_f, out_fp)) and all(
        torch.equal(a, b) for a, b in zip(out_c, out_cp))
    return dict(workload="24 slices, 2D 96..160 square, 8..32 coils, 8000..30000 samples, 16 terms, per-slice B0, "
                         "30 CG iterations each, BF16 operands, re-orthogonalised, one graph launch per batch",
                ms_per_batch=t_f, value=work / (t_f * 1e-3), unit="voxel*sample*coil/s",
                form="per-slice solves forked over 8 streams, full phase bases",
                persistent_form=dict(ms_per_batch=t_fp, value=work / (t_fp * 1e-3),
                                     form="lock-step; per iteration one persistent E and one persistent E^H launch "
                                          "per coil class over all slices, the packing and CG vector steps "
                                          "between them one batched launch each"),
                compressed_bases=dict(ms_per_batch_streams=t_c_s, ms_per_batch_persistent=t_c_p,
                                      ms_setup_host=t_c, ms_end_to_end_streams=t_c_s + t_c,
                                      terms=[pr.P + 1 for pr in cprobs],
                                      max_rel_diff_to_full=max(float(torch.linalg.vector_norm(a - b)
                                                                     / torch.linalg.vector_norm(b))
                                                               for a, b in zip(out_c, out_f))),
                persistent_equals_streams=same,
                pairs_per_EHE=sum(d["L"] * d["K"] for d in sl), steps=steps, tuned=not args.no_tune)


# Map estimation on the paper's prescan geometry (219x219x44 mm at 1x1x2 mm,
# 16 coils, 16 echoes, echo spacing 2.3 ms); smoothing weights and the CG
# tolerance are this benchmark's choice (the paper gives none).
MAP_DIMS, MAP_COILS, MAP_ECHOES = (219, 219, 22), 16, 16
MAP_ALPHA_S, MAP_ALPHA_B, MAP_TOL = 10.0, 10.0, 1e-6


def maps_run(nfs, synth, torch, dev):
    dims = MAP_DIMS
    d = synth.prescan(dims=dims, n_coil=MAP_COILS, n_echo=MAP_ECHOES)
    L = int(np.prod(dims))
    X = torch.from_numpy(d["imgs"]).to(dev)
    mT = torch.from_numpy(d["mask_T"]).to(dev)
    mR = torch.from_numpy(d["mask_R"]).to(dev)
    nfs.sens_maps(X, mT, mR, dims, MAP_ALPHA_S, tol=0.0, max_iter=2)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(3):
        nfs.sens_initial(X)
    ev[1].record()
    torch.cuda.synchronize()
    ms_init = ev[0].elapsed_time(ev[1]) / 3

    def wall(f):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    def per_iteration(precond, n):
        t0, _ = wall(lambda: nfs.sens_maps(X, mT, mR, dims, MAP_ALPHA_S, tol=0.0, max_iter=0, precond=precond))
        t1, _ = wall(lambda: nfs.sens_maps(X, mT, mR, dims, MAP_ALPHA_S, tol=0.0, max_iter=n, precond=precond))
        return (t1 - t0) / n * 1e3

    nrhs = 3 * MAP_COILS
    # algorithmic bytes per iteration and right-hand side.  Jacobi: apply
    # (r, p in; p, q out) + update (x, p, r, q in; x, r out) = 80 B per voxel.
    # Multigrid: apply (z, p in; p, q out) + update = 80 B per fine voxel, and
    # per voxel of every level above the coarsest the V-cycle's passes: the
    # two pre-sweeps (b in, x out) 16, residual (x, b in; r out) 24,
    # restriction 8, post-sweep with prolongation (x, b in; x out) 24, last
    # sweep (x, b in; x out; r.z on the finest level) 24 = 96 B.
    lv = [L]
    dd = list(dims)
    while lv[-1] > 64:
        c = [n // 2 + 1 if n >= 3 else n for n in dd]
        if c == dd:
            break
        dd = c
        lv.append(int(np.prod(dd)))
    bytes_jac = nrhs * L * 80
    bytes_mg = nrhs * (80 * L + 96 * sum(lv[:-1]))
    ms_jac = per_iteration("jacobi", 128)
    ms_mg = per_iteration("mg", 16)

    def roof(nbytes, ms):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS)

    ts, (s32, s64, shat, info_s) = wall(lambda: nfs.sens_maps(X, mT, mR, dims, MAP_ALPHA_S, tol=MAP_TOL,
                                                               max_iter=100000))
    tb, (b0, b064, fit, info_b) = wall(lambda: nfs.b0_map(X, s32, dims, d["delta_te"], MAP_ALPHA_B, tol=MAP_TOL,
                                                          max_iter=100000))
    # accuracy against the synthetic truth inside M_T (sensitivities up to a
    # common complex factor per voxel)
    inside = d["mask_T"] > 0
    a = s64.cpu().numpy()[:, inside]
    b = d["S_true"].astype(np.complex128)[:, inside]
    c = np.sum(np.conj(a) * b, axis=0) / np.sum(np.abs(a) ** 2, axis=0)
    s_err = float(np.linalg.norm(a * c - b) / np.linalg.norm(b))
    a0 = shat.cpu().numpy()[:, inside]
    c0 = np.sum(np.conj(a0) * b, axis=0) / np.sum(np.abs(a0) ** 2, axis=0)
    s0_err = float(np.linalg.norm(a0 * c0 - b) / np.linalg.norm(b))
    om = d["omega_true"][inside]
    b_err0 = float(np.sqrt(np.mean((fit[0].cpu().numpy()[inside] - om) ** 2)))
    b_err = float(np.sqrt(np.mean((b064.cpu().numpy()[inside] - om) ** 2)))
    out = dict(workload=f"prescan {dims[0]}x{dims[1]}x{dims[2]}, {MAP_COILS} coils, {MAP_ECHOES} echoes, "
                        f"dTE {d['delta_te'] * 1e3:.1f} ms, alpha_S {MAP_ALPHA_S}, alpha_B {MAP_ALPHA_B}, "
                        f"CG tol {MAP_TOL}",
               voxels=L, trusted=int(d["mask_T"].sum()), reconstruction_mask=int(d["mask_R"].sum()),
               ms_sens_initial=ms_init,
               sens_initial_GBs=(X.numel() * 8 + MAP_COILS * L * 16) / (ms_init * 1e-3) / 1e9,
               s_sens_maps=ts, sens_cg_iterations=info_s[0], sens_cg_status=nfs.CG_STATUS.get(info_s[1], info_s[1]),
               preconditioner="multigrid V(2,2), %d levels" % len(lv),
               ms_per_iteration=dict(multigrid=ms_mg, jacobi=ms_jac),
               iteration_roofline=dict(multigrid=roof(bytes_mg, ms_mg), jacobi=roof(bytes_jac, ms_jac)),
               s_b0_map=tb, b0_cg_iterations=info_b[0], b0_cg_status=nfs.CG_STATUS.get(info_b[1], info_b[1]),
               sens_rel_err_vs_truth_in_MT=dict(initial=s0_err, smoothed=s_err),
               b0_rms_err_vs_truth_in_MT_rad_s=dict(initial=b_err0, smoothed=b_err))
    del X, s32, s64, shat, b0, b064, fit
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding over samples "
                                   "is a design note only)"}))
        sys.exit(2)
    import torch

    import synth
    from paper_2604_09233_amd import nfs

    dev = torch.device("cuda:0")
    reorth = not args.plain
    progress(f"headline workload {args.config}: inputs")
    d = synth.make_config(args.config)
    sv = Solver(nfs, torch, dev, d, reorth)
    L, K, G, n_iter = sv.L, sv.K, sv.G, sv.n_iter
    if args.shapes:
        apply_shapes(nfs, sv.prob, args.precision, args.shapes)
    if args.profile_run:
        out, hist, info = sv.buffers()
        nfs.cg_solve(sv.prob, sv.m, n_iter, precision=args.precision, reorth=reorth, out=out, hist=hist, info=info)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "done", "config": args.config, "cg_info": info.cpu().tolist()}))
        return

    progress("autotune and the timed solves")
    if not args.no_tune and not args.shapes:
        nfs.autotune(sv.prob, args.precision)
    rho, hist, info, ms, wall = sv.time_solves(args.precision, args.steps, args.warmup, graphs=not args.no_graphs)
    rho = rho.clone()
    vsc = L * K * G
    value = (n_iter + 0.5) * vsc / (ms * 1e-3)
    st = info.cpu().tolist()

    progress("encode-kernel timing, E^H E alone, oracle checks")
    kt = sv.kernel_times(args.precision)
    roof = roofline(kt, L, K, G, d["n_basis"], args.precision, f"encode_kernel_{args.config}_{args.precision}_counters.md")
    ehe_ms, _ = sv.ehe_alone(args.precision, 20)  # median of 20 after 3 warm-ups
    err, checks = None, {}
    kind = "reorth" if reorth else "plain"
    g = golden(f"{args.config}_cg.npz")
    if g is not None:
        err = rel(rho.cpu().numpy(), g[f"{kind}_rho"])
    if args.config == "c3":
        checks = c3_oracle_checks(nfs, synth, torch, dev, args.precision, sv, reorth)

    forms = {}
    if not args.no_forms:
        progress("other operand forms")
        for prec in ("bf16", "fp32"):
            if prec == args.precision:
                continue
            if not args.no_tune:
                nfs.autotune(sv.prob, prec)
            rf, _, inf, msf, _ = sv.time_solves(prec, 1, 1, graphs=not args.no_graphs)
            forms[prec] = dict(ms_per_step=msf, value=(n_iter + 0.5) * vsc / (msf * 1e-3), cg_info=inf.cpu().tolist(),
                               rel_diff_to_headline=rel(rf.cpu().numpy(), rho.cpu().numpy()))
            if args.config == "c3":
                forms[prec].update(c3_oracle_checks(nfs, synth, torch, dev, prec, sv, reorth))
            del rf
    kf3 = threed_kspace_filter(nfs, torch, dev, d, rho) if len(d["dims"]) == 3 else None
    shapes = nfs.tuned_shape(sv.prob, args.precision)
    cpu_d = d
    del sv, rho
    torch.cuda.empty_cache()

    twod = None
    if not args.no_2d and args.config != "c2":
        progress("2D 128x128 leg")
        twod = twod_run(nfs, synth, torch, dev, args)
        torch.cuda.empty_cache()
    progress("batched leg")
    batched = None if args.no_batched else batched_run(nfs, synth, torch, dev, args)
    progress("maps leg")
    maps = None if args.no_maps else maps_run(nfs, synth, torch, dev)

    out = {
        "metric": "E^H·E voxel·sample·coil/s (over the CG solve); CG solve time at rel.err <=2e-3 vs FP64 oracle",
        "value": value,
        "unit": "voxel*sample*coil/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "L": L, "K": K, "G": G, "n_iter": n_iter,
                   "precision": args.precision, "cg": "re-orthogonalised" if reorth else "plain",
                   "hip_graphs": not args.no_graphs, "phase_basis_terms": d["n_basis"] + 1,
                   "phase_instructions_per_tile": phase_instrs(d["n_basis"])},
        "rel_err_vs_oracle": err,
        "rel_err_vs_oracle_note": None if err is not None else
            "no stored full-size FP64 oracle solve of this workload (many hours on the host); see oracle_checks",
        "oracle_checks": checks,
        "encode_shapes": {"tuned": not args.no_tune and not args.shapes, "pinned": args.shapes,
                          "held_tiles_nsplit": shapes},
        "cg_info": {"iterations": st[0], "status": nfs.CG_STATUS.get(st[1], st[1])},
        "ehe_alone": {"ms": ehe_ms, "value": vsc / (ehe_ms * 1e-3)},
        "forms": forms,
        "roofline": roof,
        "kspace_filter_3d": kf3,
        "2d": twod,
        "batched": batched,
        "maps": maps,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cpu_d, 512 if args.config == "c3" else 8)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
