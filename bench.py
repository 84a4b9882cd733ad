#!/usr/bin/env python3
"""Benchmark of the non-Fourier SENSE hot path on one MI355X.

One step = one full CG solve (setup, E^H m, n_iter iterations of E^H E with
the FP64 scalar updates and residual re-orthogonalisation) on the 2D
128x128 / 16-coil / 4 x 15000-sample / 16-field-term workload (30
iterations), inputs resident in HBM.

Solves are replayed from a captured hipGraph (the library's graph mode; the
pass that times the encode kernel alone runs eagerly, since per-launch HIP
events cannot live inside a graph).  Encode-kernel shapes are autotuned
before timing.

Reported value: E^H E voxel*sample*coil per second over the solve, i.e.
(n_iter + 1/2) * L * K * G / (solve time), the initial E^H m counting as half
an application.  ms_per_step is the CG solve time.  The result is checked
against the stored FP64 oracle solve of the same workload.

Also reported: the same for the FP32 operand form, one E^H E application
timed alone, the fused encode kernel's average duration (HIP events on its
launch stream, over the timed region) with its roofline, and the FP64 CPU
oracle timed on a bounded sample of the workload on this host, and the
map-estimation step (initial sensitivities, sensitivity and B0 smoothing) on
the paper's prescan geometry.
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
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-form", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 24-slice batched-solve measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D 96x96x48 / 32-coil solve measurement")
    ap.add_argument("--no-tune", action="store_true", help="use the default encode shapes instead of autotuned ones")
    ap.add_argument("--no-resident", action="store_true", help="skip the resident-P (non-split) solve measurement")
    ap.add_argument("--no-stopping", action="store_true", help="skip the 250-iteration L-curve / SSIM run")
    ap.add_argument("--plain", action="store_true", help="plain CG recurrences (no re-orthogonalisation)")
    ap.add_argument("--no-maps", action="store_true", help="skip the sensitivity / B0 map-estimation measurement")
    ap.add_argument("--profile-run", action="store_true",
                    help="one solve only (no side measurements, no CPU baseline), for counter collection")
    ap.add_argument("--no-compress", action="store_true",
                    help="solve with the full phase basis instead of its compressed form (nfs_compress_basis)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every solve eagerly instead of replaying it from a captured hipGraph")
    return ap.parse_args()


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cpu_baseline(d):
    """FP64 oracle E^H E on every 8th sample (all voxels, all coils), repeated
    for at least 10 s of wall time; returns v*s*c/s."""
    import oracle

    ks = np.arange(0, d["K"], 8)
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
                sample=f"FP64 E^H E on every 8th sample ({len(ks)} of {d['K']}) x {d['L']} voxels x "
                       f"{d['n_coil']} coils, repeated {work / (d['L'] * len(ks) * d['n_coil']):.0f}x "
                       f"in {el:.1f} s, numpy with {os.cpu_count()} threads")


def threed_run(nfs, synth, torch, dev, args):
    """The 3D workload (96x96x48, 32 coils, 16 x 35750 samples, 16 terms,
    B0 +-150 Hz, 15 CG iterations): one warm-up and one timed solve at the
    benchmark's precision, re-orthogonalised; E checked against the FP64
    oracle on 48 sampled k-space rows (all voxels, all coils)."""
    import oracle

    d = synth.make_config("c3")
    L, K, G, n_iter = d["L"], d["K"], d["n_coil"], d["n_iter"]
    prob = nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"], device=dev)
    rho_t = torch.from_numpy(d["rho_true"]).to(dev)
    clean = nfs.apply_E(prob, rho_t, "fp32")
    sig = float(torch.sqrt(torch.mean(torch.abs(clean) ** 2))) / (30 * np.sqrt(2))
    m = clean + sig * torch.from_numpy(d["noise"]).to(dev)
    del clean
    if not args.no_tune:
        nfs.autotune(prob, args.precision)
    ks = np.sort(np.random.default_rng(3).choice(K, 48, replace=False))
    e_gpu = nfs.apply_E(prob, rho_t, args.precision).cpu().numpy()[:, ks]
    e_ref = oracle.apply_E(d["rho_true"], d["sens"], d["fields"], d["b0"], d["kcoef"][ks], d["t"][ks])
    out = torch.empty(L, dtype=torch.complex64, device=dev)
    hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    nfs.cg_solve(prob, m, n_iter, precision=args.precision, reorth=True, out=out, hist=hist, info=info)
    torch.cuda.synchronize()
    nfs.profile_enable(0, True)
    nfs.profile_read(0, "E")
    nfs.profile_read(0, "EH")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    nfs.cg_solve(prob, m, n_iter, precision=args.precision, reorth=True, out=out, hist=hist, info=info)
    ev1.record()
    torch.cuda.synchronize()
    kt = {k: nfs.profile_read(0, k) for k in ("E", "EH")}
    nfs.profile_enable(0, False)
    ms = ev0.elapsed_time(ev1)
    # the paper's k-space filter on the 3D reconstruction: bins inside the
    # 3D hull of the first-order k positions (x, y, z terms)
    t0 = time.perf_counter()
    f = nfs.kspace_filter_mask(d["kcoef"][:, 1:4].astype(np.float64) / np.pi, d["dims"])
    ms_mask = (time.perf_counter() - t0) * 1e3
    f_dev = torch.from_numpy(f).to(dev)
    nfs.apply_kspace_filter(out, f_dev, d["dims"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out_f = nfs.apply_kspace_filter(out, f_dev, d["dims"])
    e1.record()
    torch.cuda.synchronize()
    ref_img = torch.from_numpy(d["rho_true"])
    kf3 = dict(bins_inside=int(f.sum()), bins=int(f.size), ms_mask_host=ms_mask, ms_apply=e0.elapsed_time(e1),
               ssim_vs_phantom_before=float(nfs.ssim(out, ref_img, d["dims"]).cpu()[0]),
               ssim_vs_phantom_after=float(nfs.ssim(out_f, ref_img, d["dims"]).cpu()[0]))
    del out_f, f_dev
    pairs = L * K
    enc = {k: v[1] / max(v[0], 1) for k, v in kt.items()}
    # MFMA instructions issued per 16 x 16 tile: the phase (f16) and the
    # contraction (one f16, two bf16 or three f16 per 16-column block)
    nq = -(-3 * (d["n_basis"] + 1) // 32)
    nb = {1: 1, 2: 2, 3: 4, 4: 4}.get(-(-2 * G // 16), 8)
    flops = pairs / 256.0 * 16384 * (nq + nb * {"fp16": 1, "bf16": 2, "fp32": 3}[args.precision])
    return dict(workload="3D 96x96x48, 32 coils, 16 x 35750-sample spiral shots, 16 field terms, B0 +-150 Hz, "
                         "15 CG iterations, re-orthogonalised",
                precision=args.precision, ms_per_solve=ms, value=(n_iter + 0.5) * pairs * G / (ms * 1e-3),
                unit="voxel*sample*coil/s", encode_kernel_ms=enc,
                sincos_frac_of_peak={k: 2 * pairs / (v * 1e-3) / TRANS_PEAK for k, v in enc.items()},
                mfma_frac_of_peak={k: flops / (v * 1e-3) / (MFMA_PEAK_TFLOPS["fp16"] * 1e12) for k, v in enc.items()},
                rel_err_E_sampled=rel(e_gpu, e_ref), sampled_rows=len(ks),
                held_tiles_nsplit=nfs.tuned_shape(prob, args.precision),
                cg_info=info.cpu().tolist(), kspace_filter=kf3)


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
    # compressed phase bases (each slice: 16 solid harmonics on one slice ->
    # 10 terms), the data rotations by exp(-i theta) inside the timed step
    full_probs, thetas = probs, None
    if not args.no_compress:
        comp = [nfs.compress_basis(pr) for pr in probs]
        probs = [c[0] for c in comp]
        thetas = [c[1] for c in comp]
    bufs = [torch.empty_like(m) for m in ms]
    if not args.no_tune:
        nfs.autotune_batched(probs, "bf16")
    work = sum((n_iter + 0.5) * d["L"] * d["K"] * d["n_coil"] for d in sl)

    def timed(mode, prs):
        rot = prs is not full_probs

        def data():
            if not rot:
                return ms
            return [nfs.phase_shift(m, th, -1, out=b) for m, th, b in zip(ms, thetas, bufs)]

        nfs.set_batch_mode(0, mode)
        nfs.set_graphs(0, True)
        outs, hists, infos = nfs.cg_solve_batched(prs, data(), n_iter, precision="bf16", reorth=True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            nfs.cg_solve_batched(prs, data(), n_iter, precision="bf16", reorth=True, outs=outs, hists=hists,
                                 infos=infos)
        ev1.record()
        torch.cuda.synchronize()
        nfs.set_graphs(0, False)
        return ev0.elapsed_time(ev1) / steps, outs

    t_p, out_p = timed("persistent", probs)
    t, out_s = timed("streams", probs)
    same = all(torch.equal(a, b) for a, b in zip(out_s, out_p))
    full = None
    if thetas is not None:
        if not args.no_tune:
            nfs.autotune_batched(full_probs, "bf16")
        t_f, out_f = timed("streams", full_probs)
        full = dict(ms_per_batch=t_f, value=work / (t_f * 1e-3),
                    max_rel_diff_to_compressed=max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                                                   for a, b in zip(out_s, out_f)))
    return dict(workload="24 slices, 2D 96..160 square, 8..32 coils, 8000..30000 samples, 16 terms, per-slice B0, "
                         "30 CG iterations each, BF16 operands, re-orthogonalised, one graph launch (slices' solves "
                         "forked over 8 streams)",
                ms_per_batch=t, value=work / (t * 1e-3), unit="voxel*sample*coil/s",
                persistent_form=dict(ms_per_batch=t_p, value=work / (t_p * 1e-3),
                                     form="lock-step; per iteration one persistent E and one persistent E^H launch "
                                          "per coil class over all slices"),
                persistent_equals_streams=same,
                phase_basis_terms=[pr.P + 1 for pr in probs], full_basis_form=full,
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
    d = synth.make_config(args.config)
    L, K, G, n_iter = d["L"], d["K"], d["n_coil"], d["n_iter"]
    prob = nfs.Problem(d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"], device=dev)
    # synthetic data: m = E rho_phantom + complex noise at SNR 30
    clean = nfs.apply_E(prob, torch.from_numpy(d["rho_true"]), "fp32")
    rms = float(torch.sqrt(torch.mean(torch.abs(clean) ** 2)))
    sigma = rms / (30 * np.sqrt(2))
    m = clean + sigma * torch.from_numpy(d["noise"]).to(dev)
    torch.cuda.synchronize()

    # Phase-basis compression, once per geometry (like the shape tuning):
    # the 16 solid harmonics on one slice span 10 functions, and the
    # per-sample offset theta cancels in E^H E.  The solve then runs on the
    # compressed problem with data exp(-i theta) m, the rotation inside the
    # timed step.
    prob_full = prob
    theta, basis = None, None
    if not args.no_compress:
        t_c = time.perf_counter()
        prob, theta, cinfo = nfs.compress_basis(prob_full)
        t_c = time.perf_counter() - t_c
        basis = dict(terms=d["n_basis"] + 1, compressed_terms=prob.P + 1, err_bound_rad=cinfo["err_bound"],
                     untimed_setup_s=t_c, setup="once per geometry (host copies of the basis, host compression, "
                                                "device copies back), like the shape tuning; not in ms_per_step")
    m_solve = m if theta is None else nfs.phase_shift(m, theta, -1)
    m_buf = torch.empty_like(m)
    torch.cuda.synchronize()

    progress("autotune and the c2 solve")
    tuned = {}
    if not args.no_tune:
        for prec in {args.precision, "fp32", "bf16"}:
            tuned[prec] = nfs.autotune(prob, prec)

    def solve(prec, out, hist, info, reorth, p=None):
        p = prob if p is None else p
        data = m
        if p is not prob_full:
            data = nfs.phase_shift(m, theta, -1, out=m_buf)
        return nfs.cg_solve(p, data, n_iter, precision=prec, reorth=reorth, out=out, hist=hist, info=info)

    def time_solves(prec, steps, warmup, profile=False, reorth=not args.plain, p=None):
        out = torch.empty(L, dtype=torch.complex64, device=dev)
        hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=dev)
        info = torch.zeros(2, dtype=torch.int32, device=dev)
        for _ in range(warmup):
            solve(prec, out, hist, info, reorth, p)
        torch.cuda.synchronize()
        if profile:
            nfs.profile_enable(0, True)
            nfs.profile_read(0, "E")
            nfs.profile_read(0, "EH")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(steps):
            solve(prec, out, hist, info, reorth, p)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1) / steps
        kt = None
        if profile:
            kt = {k: nfs.profile_read(0, k) for k in ("E", "EH")}
            nfs.profile_enable(0, False)
        return out, hist, info, ms, wall, kt

    if args.profile_run:
        time_solves(args.precision, 1, 0, profile=False)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "done"}))
        return
    if not args.no_graphs:
        nfs.set_graphs(0, True)
        rho, hist, info, ms, wall, _ = time_solves(args.precision, args.steps, args.warmup)
        nfs.set_graphs(0, False)
        # kernel timing (HIP events around every encode launch) on eager solves
        _, _, _, _, _, kt = time_solves(args.precision, max(1, args.steps // 2), 0, profile=True)
    else:
        rho, hist, info, ms, wall, kt = time_solves(args.precision, args.steps, args.warmup, profile=True)
    vsc = L * K * G
    value = (n_iter + 0.5) * vsc / (ms * 1e-3)

    # accuracy against the stored FP64 oracle solve of this workload
    err = None
    kind = "plain" if args.plain else "reorth"
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.config}_cg.npz")
    if os.path.exists(gpath):
        g = np.load(gpath)
        err = rel(rho.cpu().numpy(), g[f"{kind}_rho"])

    # one E^H E application alone (median of 20 after 3 warm-ups)
    p = torch.from_numpy(d["rho_true"]).to(dev)
    q = torch.empty_like(p)
    for _ in range(3):
        nfs.apply_EHE(prob, p, args.precision, out=q)
    torch.cuda.synchronize()
    times = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nfs.apply_EHE(prob, p, args.precision, out=q)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ehe_ms = float(np.median(times))

    # FP32 and BF16 operand forms for comparison (same workload, same solve)
    def form(prec):
        rho_f, _, _, ms_f, _, _ = time_solves(prec, max(1, args.steps // 2), 1)
        return dict(ms_per_step=ms_f, value=(n_iter + 0.5) * vsc / (ms_f * 1e-3),
                    rel_err_vs_oracle=rel(rho_f.cpu().numpy(), g[f"{kind}_rho"]) if err is not None else None)

    full_basis = None
    if basis is not None:
        # the same solve on the uncompressed basis (17 terms: two phase
        # instructions per tile)
        if not args.no_tune:
            nfs.autotune(prob_full, args.precision)
        rho_u, _, _, ms_u, _, _ = time_solves(args.precision, max(1, args.steps // 2), 1, p=prob_full)
        full_basis = dict(ms_per_step=ms_u, value=(n_iter + 0.5) * vsc / (ms_u * 1e-3),
                          rel_err_vs_oracle=rel(rho_u.cpu().numpy(), g[f"{kind}_rho"]) if err is not None else None)
        basis["full_basis_form"] = full_basis
        del rho_u
    fp32 = form("fp32") if not args.no_fp32_form and args.precision != "fp32" else None
    bf16 = form("bf16") if not args.no_fp32_form and args.precision != "bf16" else None
    # plain recurrences, same precision, for reference
    plain = None
    if not args.plain:
        rhop, _, _, msp, _, _ = time_solves(args.precision, max(1, args.steps // 2), 1, reorth=False)
        plain = dict(ms_per_step=msp,
                     rel_err_vs_oracle_plain=rel(rhop.cpu().numpy(), g["plain_rho"]) if err is not None else None,
                     oracle_plain_vs_reorth=float(g["plain_vs_reorth"][-1]) if err is not None else None)

    # roofline of the dominant kernel (the fused encode kernel, E or E^H)
    n_e, ms_e = kt["E"]
    n_h, ms_h = kt["EH"]
    kname, n_k, ms_k = ("EH", n_h, ms_h) if ms_h >= ms_e else ("E", n_e, ms_e)
    avg_ms = ms_k / max(n_k, 1)
    pairs = L * K  # voxel-sample pairs per launch
    # ALU bound: one sin and one cos per voxel-sample pair on the transcendental unit
    trans_peak = TRANS_PEAK  # ops/s
    achieved = 2 * pairs / (avg_ms * 1e-3)
    # matrix-pipe time of the MFMA instructions the kernel issues, at the
    # published dense peaks, as a fraction of the measured launch time: per
    # 16 x 16 tile (256 pairs) ceil(3 (P+1) / 32) f16 16x16x32 phase
    # instructions, and per 16-column block of the 2G real columns one f16
    # 16x16x32 (fp16), two bf16 16x16x32 (bf16: hi and lo data parts) or
    # three f16 16x16x32 (fp32: split operands) contraction instructions
    P = prob.P  # terms of the basis the solve runs on
    nq = -(-3 * (P + 1) // 32)
    nb = {1: 1, 2: 2, 3: 4, 4: 4}.get(-(-2 * G // 16), 8)
    tiles = pairs / 256.0
    flops_phase = tiles * nq * 16384
    flops_con = tiles * nb * {"fp16": 16384, "bf16": 2 * 16384, "fp32": 3 * 16384}[args.precision]
    t_mfma = (flops_phase + flops_con) / (MFMA_PEAK_TFLOPS["fp16"] * 1e12)
    # HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    # WRITE_SIZE, copy-calibrated), only while the kernel sources match the
    # ones the counters were taken on
    from paper_2604_09233_amd.profile_summary import read_traffic
    tr = read_traffic(os.path.join(ROOT, "profiles", f"encode_kernel_{args.config}_{args.precision}_counters.md"))
    traffic = tr.get(kname) if tr else None
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=trans_peak / 1e12, unit="Tsincos-ops/s",
                    frac=achieved / trans_peak, traffic=traffic, traffic_unit="bytes per launch",
                    kernel=f"encode_kernel ({kname})",
                    avg_launch_ms=avg_ms, launches=n_k,
                    mfma_pipe_frac=t_mfma / (avg_ms * 1e-3))

    resident = None
    if not args.no_resident and args.precision == "fp16":
        # non-split form: P built once per solve (2 K L x 4 bytes), streamed by every E and E^H
        def t_res(n):
            o = torch.empty(L, dtype=torch.complex64, device=dev)
            h = torch.full((n + 1, 3), float("nan"), dtype=torch.float64, device=dev)
            f = torch.zeros(2, dtype=torch.int32, device=dev)
            nfs.cg_solve_resident(prob, m_solve, n, reorth=not args.plain, out=o, hist=h, info=f)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nfs.cg_solve_resident(prob, m_solve, n, reorth=not args.plain, out=o, hist=h, info=f)
            e1.record()
            torch.cuda.synchronize()
            return o, e0.elapsed_time(e1)
        rr, ms_r = t_res(n_iter)
        _, ms_r1 = t_res(1)
        resident = dict(ms_per_step=ms_r, ms_per_iteration=(ms_r - ms_r1) / (n_iter - 1),
                        ms_build_and_first_iteration=ms_r1, P_bytes=2 * L * K * 4,
                        identical_to_split=bool(torch.equal(rr.cpu(), rho.cpu())),
                        rel_err_vs_oracle=rel(rr.cpu().numpy(), g[f"{kind}_rho"]) if err is not None else None)
        del rr
        prob._ws.pop(("CG_RESIDENT", args.precision, n_iter, not args.plain), None)
        prob._ws.pop(("CG_RESIDENT", args.precision, 1, not args.plain), None)
        torch.cuda.empty_cache()

    stopping = None
    if not args.no_stopping:
        # the paper's stopping-criteria study: 250 iterations, L-curve corner
        # and SSIM of every iterate against the phantom
        n_long = 250
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        _, h_long, i_long, its = nfs.cg_solve_traced(prob, m_solve, n_long, precision=args.precision,
                                                     reorth=not args.plain)
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

    progress("operand forms, stopping study, k-space filter")
    # the paper's k-space filter on the reconstruction: bins inside the hull
    # of the first-order k positions (linear x, y terms; kcoef / pi in
    # cycles per FOV for the normalised coordinates), IFFT(FFT(rho) o f)
    kf = None
    if len(d["dims"]) == 2:
        f = nfs.kspace_filter_mask(d["kcoef"][:, 1:3].astype(np.float64) / np.pi, d["dims"])
        f_dev = torch.from_numpy(f).to(dev)
        nfs.apply_kspace_filter(rho, f_dev, d["dims"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rho_f = nfs.apply_kspace_filter(rho, f_dev, d["dims"])
        e1.record()
        torch.cuda.synchronize()
        ref_img = torch.from_numpy(d["rho_true"])
        s_before = float(nfs.ssim(rho, ref_img, d["dims"]).cpu()[0])
        s_after = float(nfs.ssim(rho_f, ref_img, d["dims"]).cpu()[0])
        kf = dict(bins_inside=int(f.sum()), bins=int(f.size), ms_apply=e0.elapsed_time(e1),
                  ssim_vs_phantom_before=s_before, ssim_vs_phantom_after=s_after)

    progress("batched leg")
    batched = None if args.no_batched else batched_run(nfs, synth, torch, dev, args)
    progress("3D leg")
    threed = None if args.no_3d else threed_run(nfs, synth, torch, dev, args)
    progress("maps leg")
    maps = None if args.no_maps else maps_run(nfs, synth, torch, dev)

    st = info.cpu().tolist()
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
        "config": {"workload": f"{args.config}: 2D 128x128, 16 coils, 4x15000-sample R=4 spiral, 16 field terms, "
                               f"B0 +-100 Hz, {n_iter} CG iterations (one step = one CG solve)",
                   "L": L, "K": K, "G": G, "n_iter": n_iter, "precision": args.precision,
                   "cg": "plain" if args.plain else "re-orthogonalised", "hip_graphs": not args.no_graphs,
                   "phase_basis": basis, "phase_instructions_per_tile": nq},
        "rel_err_vs_oracle": err,
        "encode_shapes": {"tuned": not args.no_tune,
                          "held_tiles_nsplit": nfs.tuned_shape(prob, args.precision)},
        "cg_info": {"iterations": st[0], "status": nfs.CG_STATUS.get(st[1], st[1])},
        "ehe_alone": {"ms": ehe_ms, "value": vsc / (ehe_ms * 1e-3)},
        "fp32_form": fp32,
        "bf16_form": bf16,
        "plain_recurrences": plain,
        "encode_kernel_ms": {"E": ms_e / max(n_e, 1), "EH": ms_h / max(n_h, 1)},
        "roofline": roofline,
        "resident_P": resident,
        "stopping_criteria": stopping,
        "kspace_filter": kf,
        "batched": batched,
        "3d": threed,
        "maps": maps,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
