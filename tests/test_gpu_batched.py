"""Batched multi-slice solves and graph replay, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth

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


def args(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


@pytest.fixture(scope="module")
def small_batch(nfs):
    sl = synth.batched_slices(6, seed=3, n_range=(20, 40), g_range=(2, 12), k_range=(800, 3000))
    probs, ms = [], []
    for d in sl:
        probs.append(nfs.Problem(*args(d)))
        clean = oracle.apply_E(d["rho_true"], *args(d))
        sig = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30 * np.sqrt(2))
        ms.append((clean + sig * d["noise"]).astype(np.complex64))
    return sl, probs, ms


@pytest.fixture(params=["persistent", "streams"])
def mode(nfs, request):
    nfs.set_batch_mode(0, request.param)
    yield request.param
    nfs.set_batch_mode(0, "streams")


@pytest.mark.parametrize("prec,reorth", [("fp16", True), ("fp32", True), ("bf16", False)])
def test_batched_equals_single_solves(nfs, small_batch, prec, reorth, mode):
    """Each slice of the batch is bit-identical to its single solve, in both
    batch modes (FP32 operands run the streams form in either)."""
    sl, probs, ms = small_batch
    rb, hb, ib = nfs.cg_solve_batched(probs, [torch.from_numpy(m) for m in ms], 12, precision=prec, reorth=reorth)
    torch.cuda.synchronize()
    for i, (p, m) in enumerate(zip(probs, ms)):
        r1, h1, i1 = nfs.cg_solve(p, torch.from_numpy(m), 12, precision=prec, reorth=reorth)
        torch.cuda.synchronize()
        assert torch.equal(rb[i].cpu(), r1.cpu()), i
        assert torch.equal(ib[i].cpu(), i1.cpu()), i
        assert np.array_equal(hb[i].cpu().numpy(), h1.cpu().numpy(), equal_nan=True), i


def test_batched_slice_matches_oracle(nfs, small_batch):
    sl, probs, ms = small_batch
    rb, hb, ib = nfs.cg_solve_batched(probs, [torch.from_numpy(m) for m in ms], 10, precision="fp32", reorth=True)
    torch.cuda.synchronize()
    from _parity import check

    for i in (0, 3):
        ref = oracle.cg_solve(ms[i], *args(sl[i]), n_iter=10, reorth=True)
        err, em = check(rb[i].cpu().numpy(), ref["rho"], 1e-4, ("batched slice", i))
        print(f"batched slice {i} (L={sl[i]['L']}, K={sl[i]['K']}, G={sl[i]['n_coil']}): rel {err:.2e}, max {em:.2e}")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_batched_tolerance_freezes_slices_independently(nfs, small_batch, prec, mode):
    sl, probs, ms = small_batch
    rb, hb, ib = nfs.cg_solve_batched(probs, [torch.from_numpy(m) for m in ms], 40, tol=1e-2, precision=prec,
                                      reorth=True)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        it, st = ib[i].cpu().tolist()
        h = hb[i].cpu().numpy()
        assert st == 2 and 1 <= it < 40
        assert h[it, 0] <= 1e-2 * h[0, 0] and h[it - 1, 0] > 1e-2 * h[0, 0]


def test_graph_replay_matches_eager(nfs, small_batch):
    sl, probs, ms = small_batch
    p, m = probs[1], torch.from_numpy(ms[1]).cuda()
    out = torch.empty(p.L, dtype=torch.complex64, device="cuda")
    hist = torch.full((16, 3), float("nan"), dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    nfs.set_graphs(0, False)
    eager, _, _ = nfs.cg_solve(p, m, 15, precision="fp16", reorth=True)
    eager = eager.cpu()
    nfs.set_graphs(0, True)
    try:
        for rep in range(4):
            out.zero_()
            hist.fill_(float("nan"))
            nfs.cg_solve(p, m, 15, precision="fp16", reorth=True, out=out, hist=hist, info=info)
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), eager), rep
            assert info.cpu().tolist() == [15, 1]
            # eager work in between replays
            nfs.apply_EHE(p, out, "fp32")
            torch.cuda.synchronize()
        # batched graph replay: device-resident data and fixed output buffers,
        # so that every call after the first replays the captured graph
        dms = [torch.from_numpy(x).cuda() for x in ms]
        outs = [torch.empty(q.L, dtype=torch.complex64, device="cuda") for q in probs]
        hists = [torch.empty((9, 3), dtype=torch.float64, device="cuda") for _ in probs]
        infos = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in probs]
        nfs.set_graphs(0, False)
        ref, _, _ = nfs.cg_solve_batched(probs, dms, 8, precision="fp16", reorth=True)
        ref = [r.clone() for r in ref]
        nfs.set_graphs(0, True)
        for rep in range(3):
            for o in outs:
                o.zero_()
            nfs.cg_solve_batched(probs, dms, 8, precision="fp16", reorth=True, outs=outs, hists=hists, infos=infos)
            torch.cuda.synchronize()
            for a, b in zip(outs, ref):
                assert torch.equal(a, b), rep
            nfs.apply_E(probs[0], outs[0], "fp16")
            torch.cuda.synchronize()
    finally:
        nfs.set_graphs(0, False)


def test_persistent_batch_with_mixed_shapes_and_replacement(nfs):
    """Slices of 4 to 32 coils (one to four column blocks), different held-
    tile counts (untuned defaults, so several launch classes), residual
    replacement every 4 iterations: the lock-step persistent batch equals
    the single solves bit for bit."""
    sl = synth.batched_slices(7, seed=11, n_range=(24, 48), g_range=(4, 32), k_range=(1000, 4000))
    probs, ms = [], []
    for d in sl:
        probs.append(nfs.Problem(*args(d)))
        ms.append(torch.from_numpy((d["noise"] * 0.1).astype(np.complex64)))
    print("coils", [d["n_coil"] for d in sl], "samples", [d["K"] for d in sl])
    nfs.set_batch_mode(0, "persistent")
    rb, hb, ib = nfs.cg_solve_batched(probs, ms, 9, replace_every=4, precision="bf16", reorth=True)
    torch.cuda.synchronize()
    nfs.set_batch_mode(0, "streams")
    for i, (p, m) in enumerate(zip(probs, ms)):
        r1, h1, i1 = nfs.cg_solve(p, m, 9, replace_every=4, precision="bf16", reorth=True)
        torch.cuda.synchronize()
        assert torch.equal(rb[i].cpu(), r1.cpu()), i
        assert np.array_equal(hb[i].cpu().numpy(), h1.cpu().numpy(), equal_nan=True), i


def test_persistent_batch_of_more_than_24_slices(nfs):
    """30 slices of 2 to 8 coils (one column block: one launch class, more
    slices than one persistent launch takes, so the class is cut into two
    launches), FP16 operands with their per-slice scale bounds, plain
    recurrences: the batched packing and vector launches cover every slice,
    and each slice equals its single solve bit for bit."""
    sl = synth.batched_slices(30, seed=17, n_range=(16, 40), g_range=(2, 8), k_range=(500, 2000))
    probs, ms = [], []
    for d in sl:
        probs.append(nfs.Problem(*args(d)))
        ms.append(torch.from_numpy((d["noise"] * 0.1).astype(np.complex64)))
    nfs.set_batch_mode(0, "persistent")
    try:
        rb, hb, ib = nfs.cg_solve_batched(probs, ms, 7, precision="fp16", reorth=False)
        torch.cuda.synchronize()
    finally:
        nfs.set_batch_mode(0, "streams")
    for i, (p, m) in enumerate(zip(probs, ms)):
        r1, h1, i1 = nfs.cg_solve(p, m, 7, precision="fp16", reorth=False)
        torch.cuda.synchronize()
        assert torch.equal(ib[i].cpu(), i1.cpu()), i
        assert torch.equal(rb[i].cpu(), r1.cpu()), i
        assert np.array_equal(hb[i].cpu().numpy(), h1.cpu().numpy(), equal_nan=True), i


def test_persistent_mode_falls_back_for_shapes_it_does_not_take(nfs):
    """A batch holding a slice of 32 phase terms (three phase instructions
    per tile, which the persistent kernel is not built for) runs as the
    streams form under NFS_BATCH_PERSISTENT: every slice still equals its
    single solve bit for bit."""
    sl = [synth.random_problem(300, 900, 12, 31, seed=51), synth.random_problem(350, 800, 64, 9, seed=52)]
    probs = [nfs.Problem(*args(d)) for d in sl]
    ms = [torch.from_numpy(d["m"]) for d in sl]
    nfs.set_batch_mode(0, "persistent")
    try:
        rb, _, ib = nfs.cg_solve_batched(probs, ms, 5, precision="fp16", reorth=True)
        torch.cuda.synchronize()
    finally:
        nfs.set_batch_mode(0, "streams")
    for i, (p, m) in enumerate(zip(probs, ms)):
        r1, _, i1 = nfs.cg_solve(p, m, 5, precision="fp16", reorth=True)
        torch.cuda.synchronize()
        assert ib[i].cpu().tolist() == [5, 1], i
        assert torch.equal(rb[i].cpu(), r1.cpu()), i


def test_graph_cache_evicts_and_stays_correct(nfs, small_batch):
    """Graph mode with fresh output buffers on every call: each call is a new
    graph key, so after 32 captures the least recently used graphs are
    destroyed; every result (including replays of graphs that survived and
    re-captures of evicted ones) equals the eager solve."""
    sl, probs, ms = small_batch
    p, m = probs[2], torch.from_numpy(ms[2]).cuda()
    nfs.set_graphs(0, False)
    eager, _, _ = nfs.cg_solve(p, m, 6, precision="fp16", reorth=True)
    eager = eager.cpu()
    nfs.set_graphs(0, True)
    try:
        keep = []
        for rep in range(40):
            out, _, info = nfs.cg_solve(p, m, 6, precision="fp16", reorth=True)
            keep.append(out)  # keeps every pointer distinct
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), eager), rep
        # the first buffers' graphs were evicted: their calls capture again
        for rep in range(3):
            out, _, _ = nfs.cg_solve(p, m, 6, precision="fp16", reorth=True, out=keep[rep])
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), eager), rep
    finally:
        nfs.set_graphs(0, False)


@pytest.fixture(scope="module")
def batch24(nfs):
    import os

    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "batch24_cg.npz"))
    sl = synth.batched_slices(24)
    probs, ms = [], []
    for d in sl:
        probs.append(nfs.Problem(*args(d)))
        clean = oracle.apply_E(d["rho_true"], *args(d))
        sig = np.sqrt(np.mean(np.abs(clean) ** 2)) / (30 * np.sqrt(2))
        ms.append(torch.from_numpy((clean + sig * d["noise"]).astype(np.complex64)).cuda())
    return sl, probs, ms, g


@pytest.mark.parametrize("mode_name", ["streams", "persistent"])
def test_full_batch_sampled_vs_stored_oracle(nfs, batch24, mode_name):
    """The 24-slice workload (96..160 square, 8..32 coils, 8000..30000
    samples, 16 terms, per-slice B0), all slices in one batched call with
    BF16 operands and 30 re-orthogonalised iterations, against the stored
    FP64 oracle solves (tests/golden/batch24_cg.npz) on 512 sampled voxels
    per slice, both measures at the BF16 bar."""
    from _parity import check

    sl, probs, ms, g = batch24
    nfs.set_batch_mode(0, mode_name)
    try:
        rb, hb, ib = nfs.cg_solve_batched(probs, ms, 30, precision="bf16", reorth=True)
        torch.cuda.synchronize()
    finally:
        nfs.set_batch_mode(0, "streams")
    worst = (0.0, 0.0)
    for s in range(len(sl)):
        assert ib[s].cpu().tolist() == [30, 1], s
        x = rb[s].cpu().numpy()
        e = check(x[g[f"vox_{s}"]], g[f"rho_{s}"], 2e-3, ("slice", s))
        worst = max(worst, e)
        assert abs(np.linalg.norm(x) - g[f"norm_{s}"]) < 2e-3 * g[f"norm_{s}"], s
    print(f"24-slice batch ({mode_name}), BF16, sampled voxels vs oracle: worst rel {worst[0]:.2e} max {worst[1]:.2e}")
