"""nfs_cg_solve_noalloc: the CG solve on the library's own device scratch
(for callers that cannot allocate), against nfs_cg_solve through the C ABI.

Host checks (no GPU): the limit and argument errors come back before any
device work.  GPU checks: two calls in a row, the second on a smaller
problem, each equal to nfs_cg_solve on the same inputs (same kernels and
shapes, so bit for bit) and within the FP32 bar of the FP64 oracle.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import TOL, check
from paper_2604_09233_amd import nfs

A = 0x100000
FAKE_CTX = ctypes.create_string_buffer(4096)


def host_prob(L, K, G, P):
    return nfs.nfs_problem(L, K, G, P, A, A, A, A, A, None)


def test_noalloc_host_rejects_oversized_and_bad_arguments():
    lib = nfs.lib()
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    # a 3D-sized solve needs far more than the scratch holds
    big = host_prob(1 << 22, 1 << 20, 32, 16)
    rc = lib.nfs_cg_solve_noalloc(c, ctypes.byref(big), A, A, 15, 0.0, 0, 1, 2, None, None, None)
    assert rc == nfs.NFS_EWORKSPACE
    assert b"scratch" in lib.nfs_last_error()
    small = host_prob(1000, 777, 5, 7)
    assert lib.nfs_cg_solve_noalloc(c, ctypes.byref(small), None, A, 5, 0.0, 0, 0, 0, None, None,
                                    None) == nfs.NFS_EINVAL
    assert lib.nfs_cg_solve_noalloc(None, ctypes.byref(small), A, A, 5, 0.0, 0, 0, 0, None, None,
                                    None) == nfs.NFS_EINVAL
    assert lib.nfs_cg_solve_noalloc(c, ctypes.byref(small), A, A, -1, 0.0, 0, 0, 0, None, None,
                                    None) == nfs.NFS_EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_noalloc_equals_workspace_solve_twice(prec):
    assert torch.cuda.is_available()
    nfs.context(0)
    runs = []
    for L, K, G, P, n in ((2500, 3000, 12, 16, 8), (700, 900, 4, 7, 5)):
        d = synth.random_problem(L, K, G, P, seed=61)
        a = (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
        gp = nfs.Problem(*a)
        m = torch.from_numpy(d["m"]).cuda()
        r0, h0, i0 = nfs.cg_solve(gp, m, n, precision=prec, reorth=True)
        r1, h1, i1 = nfs.cg_solve_noalloc(gp, m, n, precision=prec, reorth=True)
        torch.cuda.synchronize()
        assert torch.equal(r1.cpu(), r0.cpu())
        assert np.array_equal(h1.cpu().numpy(), h0.cpu().numpy(), equal_nan=True)
        assert i1.cpu().tolist() == i0.cpu().tolist() == [n, 1]
        ref = oracle.cg_solve(d["m"], *a, n_iter=n, reorth=True)
        e = check(r1.cpu().numpy(), ref["rho"], TOL[prec], ("noalloc vs oracle", L, prec))
        runs.append((L, e))
    print(f"noalloc {prec}: " + ", ".join(f"L={L}: {e[0]:.1e}/{e[1]:.1e}" for L, e in runs))
