"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/nfs.h declares, and rejects bad arguments with the
documented status codes before anything touches a device."""
import ctypes
import math
import os
import re

import pytest

from paper_2604_09233_amd import nfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nfs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nfs_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return nfs.lib()


def test_every_declared_function_is_exported(L):
    names = declared_functions()
    assert set(names) >= {"nfs_create", "nfs_destroy", "nfs_workspace_bytes", "nfs_apply_E", "nfs_apply_EH",
                          "nfs_apply_EHE", "nfs_cg_solve", "nfs_last_error", "nfs_version"}
    for n in names:
        assert hasattr(L, n), n


def test_version(L):
    assert L.nfs_version() == 100


# fake but aligned host addresses: validation never dereferences them
A = 0x100000


def prob(L=1000, K=777, G=5, P=7, **over):
    kw = dict(sens=A, fields=A, b0=A, kcoef=A, t=A, icorr=None)
    kw.update(over)
    return nfs.nfs_problem(L, K, G, P, kw["sens"], kw["fields"], kw["b0"], kw["kcoef"], kw["t"], kw["icorr"])


# a zero-filled stand-in context, larger than the library's context struct:
# validation paths read only its plain fields (CU count 0, empty tuning
# table) and never a device handle
FAKE_CTX = ctypes.create_string_buffer(4096)


def call(L, fn, pr, prec=0, ws=A, ws_bytes=1 << 40, a=A, b=A, ctx=True):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p) if ctx else None
    p = ctypes.byref(pr) if pr is not None else None
    if fn == "cg":
        return L.nfs_cg_solve(c, p, a, b, 5, 0.0, 0, 0, prec, None, None, ws, ws_bytes, None)
    return getattr(L, fn)(c, p, a, b, prec, ws, ws_bytes, None)


FNS = ["nfs_apply_E", "nfs_apply_EH", "nfs_apply_EHE", "cg"]


@pytest.mark.parametrize("fn", FNS)
def test_validation_codes(L, fn):
    assert call(L, fn, prob(), ctx=False) == nfs.NFS_EINVAL
    assert b"ctx" in L.nfs_last_error()
    assert call(L, fn, None) == nfs.NFS_EINVAL
    assert call(L, fn, prob(G=0)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(G=65)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(P=32)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(P=-1)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(L=-1)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(K=(1 << 26) + 1)) == nfs.NFS_ESHAPE
    assert call(L, fn, prob(sens=None)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(b0=None)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(fields=None)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(kcoef=None)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(t=None)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(sens=A + 4)) == nfs.NFS_EINVAL   # complex needs 8-byte alignment
    assert call(L, fn, prob(b0=A + 2)) == nfs.NFS_EINVAL
    assert call(L, fn, prob(), prec=3) == nfs.NFS_EINVAL
    assert call(L, fn, prob(), a=None) == nfs.NFS_EINVAL
    assert call(L, fn, prob(), b=None) == nfs.NFS_EINVAL
    assert call(L, fn, prob(), a=A + 4) == nfs.NFS_EINVAL
    assert call(L, fn, prob(), ws=None) == nfs.NFS_EWORKSPACE
    assert call(L, fn, prob(), ws=A + 128) == nfs.NFS_EWORKSPACE
    assert call(L, fn, prob(), ws_bytes=1) == nfs.NFS_EWORKSPACE
    assert b"workspace" in L.nfs_last_error()


def test_fields_may_be_null_without_basis_terms(L):
    # P = 0: only the B0 term; fields/kcoef are not read
    assert call(L, "nfs_apply_E", prob(P=0, fields=None, kcoef=None), ws_bytes=1) == nfs.NFS_EWORKSPACE


def test_cg_specific_validation(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    pr = prob()
    f = L.nfs_cg_solve
    assert f(c, ctypes.byref(pr), A, A, -1, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, math.nan, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, math.inf, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, -1e-3, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, -2, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, A + 4, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, A + 2, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, None, A, 1, None) == nfs.NFS_EWORKSPACE
    # reorth flag: only 0/1, and at most 2048 iterations
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 2, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 3000, 0.0, 0, 1, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL


def test_workspace_bytes(L):
    n = ctypes.c_size_t()
    pr = prob()
    for op in range(4):
        for prec in range(3):
            assert L.nfs_workspace_bytes(None, ctypes.byref(pr), op, prec, 10, 0, ctypes.byref(n)) == 0
            assert n.value > 0 and n.value % 256 == 0
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 5, 0, 0, 0, ctypes.byref(n)) == nfs.NFS_EINVAL
    # the resident (non-split) CG: FP16 only, and 2 K L x 4 bytes more than CG
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 4, 0, 10, 0, ctypes.byref(n)) == nfs.NFS_EUNSUPPORTED
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 4, 2, 10, 0, ctypes.byref(n)) == 0
    res = n.value
    L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 2, 10, 0, ctypes.byref(n))
    assert res >= n.value + 2 * 1008 * 784 * 4
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 0, 7, 0, 0, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 0, -1, 0, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 0, 0, 0, 0, None) == nfs.NFS_EINVAL
    assert L.nfs_workspace_bytes(None, ctypes.byref(prob(G=0)), 0, 0, 0, 0, ctypes.byref(n)) == nfs.NFS_ESHAPE
    # CG needs at least what E^H E needs, and grows with n_iter
    L.nfs_workspace_bytes(None, ctypes.byref(pr), 2, 0, 0, 0, ctypes.byref(n))
    ehe = n.value
    L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 0, 10, 0, ctypes.byref(n))
    cg10 = n.value
    L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 0, 1000, 0, ctypes.byref(n))
    assert cg10 > ehe and n.value > cg10
    # re-orthogonalisation stores n_iter + 1 residuals
    L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 0, 10, 1, ctypes.byref(n))
    assert n.value >= cg10 + 11 * 1000 * 8
    assert L.nfs_workspace_bytes(None, ctypes.byref(pr), 3, 0, 3000, 1, ctypes.byref(n)) == nfs.NFS_EINVAL
    # empty problems are valid
    assert L.nfs_workspace_bytes(None, ctypes.byref(prob(L=0, K=0)), 3, 2, 3, 0, ctypes.byref(n)) == 0


def test_create_without_gpu_reports_hip_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.nfs_create(ctypes.byref(h), 0) == nfs.NFS_EHIP
    assert not h.value
    assert L.nfs_create(None, 0) == nfs.NFS_EINVAL


def test_batched_validation(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    arr = (nfs.nfs_problem * 2)(prob(), prob(G=65))
    ptrs = (ctypes.c_void_p * 2)(A, A)
    f = L.nfs_cg_solve_batched
    assert f(None, 2, arr, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, -1, arr, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, 2, None, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, 2, arr, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_ESHAPE  # slice 1
    ok = (nfs.nfs_problem * 2)(prob(), prob(L=64, K=99, G=3, P=16))
    assert f(c, 2, ok, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1, None) == nfs.NFS_EWORKSPACE
    assert f(c, 0, ok, ptrs, ptrs, 5, 0.0, 0, 0, 0, None, None, A, 1, None) == nfs.NFS_OK  # nothing to do
    assert f(c, 0, None, None, None, 5, 0.0, 0, 0, 0, None, None, None, 0, None) == nfs.NFS_OK
    n = ctypes.c_size_t()
    assert L.nfs_workspace_bytes_batched(None, 2, ok, 2, 30, 1, ctypes.byref(n)) == 0
    one = ctypes.c_size_t()
    L.nfs_workspace_bytes(None, ctypes.byref(ok[0]), 3, 2, 30, 1, ctypes.byref(one))
    two = ctypes.c_size_t()
    L.nfs_workspace_bytes(None, ctypes.byref(ok[1]), 3, 2, 30, 1, ctypes.byref(two))
    al = lambda b: (b + 255) // 256 * 256
    # per-slice workspaces, the work-list counters, the persistent form's per-slice launch arguments
    assert n.value == al(one.value) + al(two.value) + 1024 + al(192 * 2) + 2 * al(128 * 2)
    z = ctypes.c_size_t(7)
    assert L.nfs_workspace_bytes_batched(None, 0, None, 2, 30, 1, ctypes.byref(z)) == 0 and z.value == 0
    assert L.nfs_set_graphs(None, 1) == nfs.NFS_EINVAL


def test_autotune_validation(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    pr = prob(L=3000, K=5000, G=12, P=16)
    n = ctypes.c_size_t()
    assert L.nfs_tune_workspace_bytes(None, ctypes.byref(pr), 2, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert L.nfs_tune_workspace_bytes(c, ctypes.byref(pr), 2, None) == nfs.NFS_EINVAL
    assert L.nfs_tune_workspace_bytes(c, ctypes.byref(pr), 9, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert L.nfs_tune_workspace_bytes(c, ctypes.byref(prob(G=0)), 2, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert L.nfs_tune_workspace_bytes(c, ctypes.byref(pr), 2, ctypes.byref(n)) == 0
    ehe = ctypes.c_size_t()
    assert L.nfs_workspace_bytes(c, ctypes.byref(pr), 2, 2, 0, 0, ctypes.byref(ehe)) == 0
    assert n.value > ehe.value and n.value % 256 == 0
    f = L.nfs_autotune
    assert f(None, ctypes.byref(pr), 2, A, n.value, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), 2, None, n.value, None) == nfs.NFS_EWORKSPACE
    assert f(c, ctypes.byref(pr), 2, A + 128, n.value, None) == nfs.NFS_EWORKSPACE
    assert f(c, ctypes.byref(pr), 2, A, n.value - 256, None) == nfs.NFS_EWORKSPACE
    assert f(c, ctypes.byref(prob(sens=None)), 2, A, n.value, None) == nfs.NFS_EINVAL
    mt, ns = ctypes.c_int(), ctypes.c_int()
    assert L.nfs_tuned_shape(c, ctypes.byref(pr), 2, 0, ctypes.byref(mt), ctypes.byref(ns)) == 0
    assert mt.value in (2, 4) and ns.value >= 1
    assert L.nfs_tuned_shape(c, ctypes.byref(pr), 2, 2, ctypes.byref(mt), ctypes.byref(ns)) == nfs.NFS_EINVAL
    assert L.nfs_tuned_shape(c, ctypes.byref(pr), 2, 1, None, ctypes.byref(ns)) == nfs.NFS_EINVAL


def test_autotune_batched_validation(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    arr = (nfs.nfs_problem * 2)(prob(), prob(L=64, K=99, G=3, P=16))
    n = ctypes.c_size_t()
    f = L.nfs_tune_workspace_bytes_batched
    assert f(None, 2, arr, 2, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert f(c, -1, arr, 2, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert f(c, 2, None, 2, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert f(c, 2, arr, 2, None) == nfs.NFS_EINVAL
    assert f(c, 2, (nfs.nfs_problem * 2)(prob(), prob(G=65)), 2, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert f(c, 2, arr, 2, ctypes.byref(n)) == 0 and n.value > 0 and n.value % 256 == 0
    g = L.nfs_autotune_batched
    assert g(None, 2, arr, 2, A, n.value, None) == nfs.NFS_EINVAL
    assert g(c, 2, arr, 2, None, n.value, None) == nfs.NFS_EWORKSPACE
    assert g(c, 2, arr, 2, A, n.value - 256, None) == nfs.NFS_EWORKSPACE
    assert g(c, 2, (nfs.nfs_problem * 2)(prob(), prob(t=None)), 2, A, n.value, None) == nfs.NFS_EINVAL
    assert g(c, 0, arr, 2, A, 0, None) == 0  # an empty batch has nothing to tune


def test_resident_cg_validation(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    pr = prob()
    f = L.nfs_cg_solve_resident
    assert f(None, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 2, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, None, A, 1 << 40, None) == nfs.NFS_EUNSUPPORTED
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 1, None, None, A, 1 << 40, None) == nfs.NFS_EUNSUPPORTED
    assert f(c, ctypes.byref(pr), A, A, -1, 0.0, 0, 0, 2, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert f(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 2, None, None, A, 1, None) == nfs.NFS_EWORKSPACE
    assert f(c, ctypes.byref(prob(G=0)), A, A, 5, 0.0, 0, 0, 2, None, None, A, 1 << 40, None) == nfs.NFS_ESHAPE


def test_lcurve_corner_host_function_matches_oracle():
    """nfs_lcurve_corner is host arithmetic over the CG history: it must pick
    the oracle's corner and reproduce its curvatures."""
    import numpy as np

    from oracle import quality as Q

    rng = np.random.default_rng(12)
    for trial in range(5):
        n = 40
        # a noisy L shape: ||d|| falls fast then flattens while ||rho|| grows
        t = np.arange(1, n + 1, dtype=np.float64)
        lx = np.log(1 + t) + 0.01 * rng.standard_normal(n)
        ly = -2.5 * np.tanh(t / (4 + trial)) + 0.003 * rng.standard_normal(n)
        hist = np.zeros((n + 1, 3))
        hist[0] = [1.0, 0.0, 1.0]
        hist[1:, 0] = 1.0
        hist[1:, 1] = np.exp(lx)
        hist[1:, 2] = np.exp(2 * ly)
        if trial == 3:
            hist[17, 2] = -1e-3  # a recurrence value gone negative: left out
        corner, kap = nfs.lcurve_corner(hist)
        c_ref, k_ref = Q.lcurve_corner(hist)
        assert corner == c_ref
        ok = np.isfinite(k_ref)
        assert np.array_equal(ok, np.isfinite(kap))
        assert np.allclose(kap[ok], k_ref[ok], rtol=1e-12, atol=1e-14)
    c = ctypes.c_int()
    assert nfs.lib().nfs_lcurve_corner(None, 3, ctypes.byref(c), None) == nfs.NFS_EINVAL
    assert nfs.lib().nfs_lcurve_corner(None, 0, ctypes.byref(c), None) == 0 and c.value == -1


def test_ssim_and_traced_validation(L):
    n = ctypes.c_size_t()
    f = L.nfs_ssim_workspace_bytes
    assert f(3, 20, 20, 1, ctypes.byref(n)) == 0 and n.value > 0
    assert f(3, 10, 20, 1, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert f(3, 20, 20, 5, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert f(-1, 20, 20, 1, ctypes.byref(n)) == nfs.NFS_EINVAL
    assert f(3, 20, 20, 1, None) == nfs.NFS_EINVAL
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    g = L.nfs_ssim
    f(2, 20, 20, 1, ctypes.byref(n))
    assert g(None, A, 2, A, 20, 20, 1, A, A, n.value, None) == nfs.NFS_EINVAL
    assert g(c, None, 2, A, 20, 20, 1, A, A, n.value, None) == nfs.NFS_EINVAL
    assert g(c, A, 2, A, 20, 20, 1, None, A, n.value, None) == nfs.NFS_EINVAL
    assert g(c, A, 2, A, 20, 20, 1, A, A, n.value - 8, None) == nfs.NFS_EWORKSPACE
    assert g(c, A, 2, A, 20, 20, 1, A, A + 64, n.value, None) == nfs.NFS_EWORKSPACE
    t = L.nfs_cg_solve_traced
    pr = prob()
    assert t(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, None, None, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert t(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, None, A + 4, A, 1 << 40, None) == nfs.NFS_EINVAL
    assert t(c, ctypes.byref(pr), A, A, 5, 0.0, 0, 0, 0, None, None, A, A, 1, None) == nfs.NFS_EWORKSPACE


def test_kspace_filter_mask_host_function_matches_oracle():
    """nfs_kspace_filter_mask (host geometry) against the oracle's Delaunay
    point location, bit for bit except for bins within 1e-6 of the hull
    boundary (where both answers are valid)."""
    import numpy as np

    import synth
    from oracle import postproc as PP

    for cfg, seed in (("c1", 0), (None, 1), (None, 2)):
        if cfg:
            d = synth.make_config(cfg, with_noise=False)
            dims = d["dims"]
            kpos = d["kcoef"][:, 1:3].astype(np.float64) / np.pi
        else:
            rng = np.random.default_rng(seed)
            dims = (40, 34)
            kpos = rng.uniform(-14, 14, size=(300, 2)) * np.array([1.0, 0.7])
        f = nfs.kspace_filter_mask(kpos, dims)
        ref = PP.kspace_filter_mask(kpos, dims)
        from scipy.spatial import ConvexHull
        hull = ConvexHull(kpos)
        fr = PP.grid_frequencies(dims)
        # distance of every bin to the hull boundary (max over facet equations)
        dist = np.max(fr @ hull.equations[:, :2].T + hull.equations[:, 2], axis=1)
        clear = np.abs(dist) > 1e-6
        assert np.array_equal(f[clear], ref[clear]), cfg
        assert f.sum() > 0
    c = ctypes.c_int64()
    m = (ctypes.c_uint8 * 16)()
    k = (ctypes.c_double * 6)(0, 0, 1, 0, 0, 1)
    assert nfs.lib().nfs_kspace_filter_mask(k, 3, 4, 4, 4, 1, m, ctypes.byref(c)) == nfs.NFS_EUNSUPPORTED
    assert nfs.lib().nfs_kspace_filter_mask(k, 3, 2, 4, 4, 2, m, ctypes.byref(c)) == nfs.NFS_EUNSUPPORTED
    assert nfs.lib().nfs_kspace_filter_mask(None, 3, 2, 4, 4, 1, m, ctypes.byref(c)) == nfs.NFS_EINVAL
    n = ctypes.c_size_t()
    assert nfs.lib().nfs_kspace_filter_workspace_bytes(None, 0, 4, 1, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert nfs.lib().nfs_kspace_filter_workspace_bytes(None, 32, 32, 1, ctypes.byref(n)) == 0 and n.value > 0


# ---- map estimation: argument checks (nothing reaches a device) ----

def _ctx():
    return ctypes.cast(FAKE_CTX, ctypes.c_void_p)


def _sens_maps(L, G=8, ne=6, dims=(20, 16, 1), alpha=1.0, tol=1e-8, max_iter=10, ws_bytes=1 << 40, out=A,
               masks=A, precond=1):
    info = (ctypes.c_int * 2)()
    return L.nfs_sens_maps(_ctx(), A, G, ne, masks, masks, *dims, alpha, tol, max_iter, precond, out, None, None,
                           None, info, A, ws_bytes, None)


def _b0_map(L, G=8, ne=6, dims=(20, 16, 1), dte=2.3e-3, alpha=1.0, tol=1e-8, max_iter=10, ws_bytes=1 << 40,
            precond=1):
    info = (ctypes.c_int * 2)()
    return L.nfs_b0_map(_ctx(), A, G, ne, A, *dims, dte, alpha, tol, max_iter, precond, A, None, None, info, A,
                        ws_bytes, None)


def test_map_workspace_sizes(L):
    sz = ctypes.c_size_t()
    assert L.nfs_maps_workspace_bytes(0, 8, 20, 16, 1, 0, ctypes.byref(sz)) == 0
    small = sz.value
    assert L.nfs_maps_workspace_bytes(0, 8, 40, 16, 3, 0, ctypes.byref(sz)) == 0
    assert sz.value > small
    # sensitivities: 3G float64 CG systems of 5 vectors each at least
    assert sz.value >= 3 * 8 * 40 * 16 * 3 * 8 * 5
    jac = sz.value
    # multigrid: a sixth fine vector, a fine scratch vector and the coarse levels
    assert L.nfs_maps_workspace_bytes(0, 8, 40, 16, 3, 1, ctypes.byref(sz)) == 0
    assert sz.value >= jac + 2 * 3 * 8 * 40 * 16 * 3 * 8
    assert L.nfs_maps_workspace_bytes(1, 8, 20, 16, 1, 0, ctypes.byref(sz)) == 0
    assert sz.value >= 20 * 16 * 8 * 8
    assert L.nfs_maps_workspace_bytes(2, 8, 20, 16, 1, 0, ctypes.byref(sz)) == nfs.NFS_EINVAL
    assert L.nfs_maps_workspace_bytes(0, 8, 20, 16, 1, 2, ctypes.byref(sz)) == nfs.NFS_EINVAL
    assert L.nfs_maps_workspace_bytes(0, 17, 20, 16, 1, 0, ctypes.byref(sz)) == nfs.NFS_ESHAPE
    assert L.nfs_maps_workspace_bytes(1, 64, 20, 16, 1, 1, ctypes.byref(sz)) == 0
    assert L.nfs_maps_workspace_bytes(0, 8, 0, 16, 1, 0, ctypes.byref(sz)) == nfs.NFS_ESHAPE


def test_map_argument_checks(L):
    assert _sens_maps(L, G=17) == nfs.NFS_ESHAPE
    assert _sens_maps(L, G=0) == nfs.NFS_ESHAPE
    assert _sens_maps(L, ne=0) == nfs.NFS_ESHAPE
    assert _sens_maps(L, dims=(20, 0, 1)) == nfs.NFS_ESHAPE
    assert _sens_maps(L, alpha=-1.0) == nfs.NFS_EINVAL
    assert _sens_maps(L, alpha=math.inf) == nfs.NFS_EINVAL
    assert _sens_maps(L, tol=math.nan) == nfs.NFS_EINVAL
    assert _sens_maps(L, max_iter=-1) == nfs.NFS_EINVAL
    assert _sens_maps(L, precond=2) == nfs.NFS_EINVAL
    assert _b0_map(L, precond=-1) == nfs.NFS_EINVAL
    assert _sens_maps(L, out=None) == nfs.NFS_EINVAL
    assert _sens_maps(L, masks=None) == nfs.NFS_EINVAL
    assert _sens_maps(L, masks=A + 2) == nfs.NFS_EINVAL
    assert _sens_maps(L, ws_bytes=1024) == nfs.NFS_EWORKSPACE
    assert "workspace" in L.nfs_last_error().decode()
    assert _b0_map(L, ne=2) == nfs.NFS_ESHAPE
    assert _b0_map(L, ne=65) == nfs.NFS_ESHAPE
    assert _b0_map(L, G=65) == nfs.NFS_ESHAPE
    assert _b0_map(L, dte=0.0) == nfs.NFS_EINVAL
    assert _b0_map(L, dte=-1e-3) == nfs.NFS_EINVAL
    assert _b0_map(L, alpha=-0.5) == nfs.NFS_EINVAL
    assert _b0_map(L, ws_bytes=64) == nfs.NFS_EWORKSPACE
    assert L.nfs_sens_initial(None, A, 8, 6, 100, A, None) == nfs.NFS_EINVAL
    assert L.nfs_sens_initial(_ctx(), A, 17, 6, 100, A, None) == nfs.NFS_ESHAPE
    assert L.nfs_sens_initial(_ctx(), A, 8, 6, -1, A, None) == nfs.NFS_ESHAPE
    assert L.nfs_sens_initial(_ctx(), A, 8, 6, 100, None, None) == nfs.NFS_EINVAL


def test_kspace_filter_mask_3d_matches_oracle():
    """3D hull mask (host quickhull, per-column plane intervals) against the
    oracle's Delaunay point location, bit for bit except for bins within
    1e-6 of the hull boundary: a cube (closed form), random ellipsoid clouds
    and the first-order positions of the 3D spiral workload."""
    import numpy as np

    import synth
    from oracle import postproc as PP
    from scipy.spatial import ConvexHull

    cube = np.array([[x, y, z] for x in (-3.5, 4.5) for y in (-2.5, 3.5) for z in (-1.5, 2.5)] + [[0.1, 0.2, 0.3]])
    dims = (12, 10, 8)
    f = nfs.kspace_filter_mask(cube, dims)
    fr = PP.grid_frequencies(dims)
    want = ((fr[:, 0] >= -3.5) & (fr[:, 0] <= 4.5) & (fr[:, 1] >= -2.5) & (fr[:, 1] <= 3.5)
            & (fr[:, 2] >= -1.5) & (fr[:, 2] <= 2.5))
    assert np.array_equal(f.astype(bool), want)
    d = synth.make_config("c3s", with_noise=False)
    # every 16th position: the oracle's 3D Delaunay of all 32000 takes minutes
    cases = [(d["dims"], d["kcoef"][::16, 1:4].astype(np.float64) / np.pi)]
    for seed in (1, 2):
        rng = np.random.default_rng(seed)
        v = rng.standard_normal((500, 3))
        v *= (rng.random(500) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
        cases.append(((20, 18, 14), v * np.array([9.0, 7.0, 5.0])))
    for dims, kpos in cases:
        f = nfs.kspace_filter_mask(kpos, dims)
        ref = PP.kspace_filter_mask(kpos, dims)
        hull = ConvexHull(kpos)
        fr = PP.grid_frequencies(dims)
        dist = np.max(fr @ hull.equations[:, :3].T + hull.equations[:, 3], axis=1)
        clear = np.abs(dist) > 1e-6
        print(f"3D mask {dims}, {len(kpos)} positions: {int(f.sum())} bins inside, "
              f"{int((~clear).sum())} within 1e-6 of the hull")
        assert np.array_equal(f[clear], ref[clear])
        assert 0 < f.sum() < f.size
    L = nfs.lib()
    c = ctypes.c_int64()
    m = (ctypes.c_uint8 * 64)()
    flat = (ctypes.c_double * 15)(0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0, 0.5, 0.5, 0)  # coplanar
    assert L.nfs_kspace_filter_mask(flat, 5, 3, 4, 4, 4, m, ctypes.byref(c)) == nfs.NFS_EINVAL
    assert L.nfs_kspace_filter_mask(flat, 3, 3, 4, 4, 4, m, ctypes.byref(c)) == nfs.NFS_EINVAL  # too few


def test_kspace_filter_mask_3d_full_trajectory_sampled():
    """All 572000 first-order positions of the 96x96x48 3D spiral workload:
    sampled bins of the native mask against a half-space test with the face
    equations of scipy's ConvexHull (an independent hull), off the 1e-6
    boundary band."""
    import numpy as np

    import synth
    from oracle import postproc as PP
    from scipy.spatial import ConvexHull

    d = synth.make_config("c3", with_noise=False)
    kpos = d["kcoef"][:, 1:4].astype(np.float64) / np.pi
    f = nfs.kspace_filter_mask(kpos, d["dims"])
    eq = ConvexHull(kpos).equations
    fr = PP.grid_frequencies(d["dims"])
    idx = np.random.default_rng(0).choice(fr.shape[0], 3000, replace=False)
    dist = np.max(fr[idx] @ eq[:, :3].T + eq[:, 3], axis=1)
    clear = np.abs(dist) > 1e-6
    assert np.array_equal(f[idx][clear].astype(bool), dist[clear] < 0)
    assert 0.3 < f.mean() < 0.9


def test_kspace_filter_workspace_and_limits(L):
    n = ctypes.c_size_t()
    assert L.nfs_kspace_filter_workspace_bytes(None, 96, 96, 48, ctypes.byref(n)) == 0
    assert n.value == 96 * 96 * 48 * 8  # one complex grid, already a multiple of 256
    assert L.nfs_kspace_filter_workspace_bytes(None, 5, 3, 1, ctypes.byref(n)) == 0
    assert n.value == 256  # 120 bytes rounded up to the 256-byte segment
    assert L.nfs_kspace_filter_workspace_bytes(None, 2049, 2, 1, ctypes.byref(n)) == nfs.NFS_ESHAPE
    assert L.nfs_kspace_filter_workspace_bytes(None, 2048, 2048, 1, ctypes.byref(n)) == 0
    assert L.nfs_kspace_filter_workspace_bytes(None, 0, 2, 1, ctypes.byref(n)) == nfs.NFS_ESHAPE
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    # too-long axis, then a short workspace: refused before any launch
    assert L.nfs_apply_kspace_filter(c, A, A + 4096, 4096, 1, 1, A, A, 1 << 20, None) == nfs.NFS_ESHAPE
    assert L.nfs_apply_kspace_filter(c, A, A + 4096, 16, 16, 1, A, A, 255, None) == nfs.NFS_EWORKSPACE
    assert L.nfs_apply_kspace_filter(c, A, A + 4096, 16, 16, 1, None, A, 1 << 20, None) == nfs.NFS_EINVAL


def test_set_shape_rejects_bad_shapes(L):
    c = ctypes.cast(FAKE_CTX, ctypes.c_void_p)
    pr = prob(G=32)  # four column blocks
    assert L.nfs_set_shape(None, ctypes.byref(pr), 2, 0, 4, 2) == nfs.NFS_EINVAL
    assert L.nfs_set_shape(c, ctypes.byref(pr), 7, 0, 4, 2) == nfs.NFS_EINVAL
    assert L.nfs_set_shape(c, ctypes.byref(pr), 2, 2, 4, 2) == nfs.NFS_EINVAL  # only E and E^H
    assert L.nfs_set_shape(c, ctypes.byref(pr), 2, 0, 3, 2) == nfs.NFS_EINVAL
    assert L.nfs_set_shape(c, ctypes.byref(pr), 2, 0, 2, 0) == nfs.NFS_EINVAL
    assert L.nfs_set_shape(c, ctypes.byref(pr), 2, 1, 2, 65) == nfs.NFS_EINVAL
    pr8 = prob(G=64)  # eight column blocks: four held tiles are not built
    assert L.nfs_set_shape(c, ctypes.byref(pr8), 2, 0, 4, 2) == nfs.NFS_EINVAL
    assert b"held tiles" in L.nfs_last_error()
