"""Thin ctypes binding of libnfs.so (the C ABI declared in include/nfs.h).

Argument marshalling only: every step of E, E^H, E^H E and the CG solve runs
in the library's HIP kernels.  PyTorch provides device memory (inputs,
outputs and the workspace) and the stream (the current torch stream).  There
is no fallback: if the library is not built, or the device is not gfx950,
every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnfs.so")

NFS_OK, NFS_EINVAL, NFS_ESHAPE, NFS_EHIP, NFS_EWORKSPACE, NFS_EUNSUPPORTED = 0, -1, -2, -3, -4, -6
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
OPS = {"E": 0, "EH": 1, "EHE": 2, "CG": 3, "CG_RESIDENT": 4}
CG_STATUS = {1: "max_iter", 2: "tol", 3: "exact", 4: "breakdown"}

_lib = None
_lib_lock = threading.Lock()


class NfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nfs error {code}: {msg}")
        self.code = code


class nfs_problem(ctypes.Structure):
    _fields_ = [
        ("n_vox", ctypes.c_int64),
        ("n_samp", ctypes.c_int64),
        ("n_coil", ctypes.c_int32),
        ("n_basis", ctypes.c_int32),
        ("sens", ctypes.c_void_p),
        ("fields", ctypes.c_void_p),
        ("b0", ctypes.c_void_p),
        ("kcoef", ctypes.c_void_p),
        ("t", ctypes.c_void_p),
        ("icorr", ctypes.c_void_p),
    ]


def lib():
    """Load libnfs.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2604_09233_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
            pp = ctypes.POINTER(nfs_problem)
            L.nfs_create.argtypes = [ctypes.POINTER(vp), i32]
            L.nfs_destroy.argtypes = [vp]
            L.nfs_workspace_bytes.argtypes = [vp, pp, i32, i32, i32, i32, ctypes.POINTER(sz)]
            for name in ("nfs_apply_E", "nfs_apply_EH", "nfs_apply_EHE"):
                getattr(L, name).argtypes = [vp, pp, vp, vp, i32, vp, sz, vp]
            L.nfs_cg_solve.argtypes = [vp, pp, vp, vp, i32, dbl, i32, i32, i32, vp, vp, vp, sz, vp]
            L.nfs_cg_solve_resident.argtypes = [vp, pp, vp, vp, i32, dbl, i32, i32, i32, vp, vp, vp, sz, vp]
            L.nfs_cg_solve_noalloc.argtypes = [vp, pp, vp, vp, i32, dbl, i32, i32, i32, vp, vp, vp]
            L.nfs_cg_solve_traced.argtypes = [vp, pp, vp, vp, i32, dbl, i32, i32, i32, vp, vp, vp, vp, sz, vp]
            L.nfs_ssim_workspace_bytes.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
            L.nfs_ssim.argtypes = [vp, vp, i32, vp, i32, i32, i32, vp, vp, sz, vp]
            L.nfs_lcurve_corner.argtypes = [vp, i32, ctypes.POINTER(i32), vp]
            L.nfs_kspace_filter_workspace_bytes.argtypes = [vp, i32, i32, i32, ctypes.POINTER(sz)]
            L.nfs_apply_kspace_filter.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, sz, vp]
            L.nfs_kspace_filter_mask.argtypes = [vp, ctypes.c_int64, i32, i32, i32, i32, vp,
                                                 ctypes.POINTER(ctypes.c_int64)]
            L.nfs_encode_backward.argtypes = [vp, pp, vp, vp, vp, vp, vp, i32, vp, sz, vp]
            L.nfs_compress_basis.argtypes = [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int64, i32, dbl, vp, vp, vp,
                                             vp, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
            L.nfs_phase_shift.argtypes = [vp, vp, vp, i32, ctypes.c_int64, vp, i32, vp]
            L.nfs_compress_workspace_bytes.argtypes = [pp, ctypes.POINTER(sz)]
            L.nfs_compress_basis_device.argtypes = [vp, pp, dbl, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
            L.nfs_workspace_bytes_batched.argtypes = [vp, i32, pp, i32, i32, i32, ctypes.POINTER(sz)]
            L.nfs_cg_solve_batched.argtypes = [vp, i32, pp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, dbl, i32,
                                               i32, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp]
            L.nfs_set_graphs.argtypes = [vp, i32]
            L.nfs_set_batch_mode.argtypes = [vp, i32]
            L.nfs_tune_workspace_bytes.argtypes = [vp, pp, i32, ctypes.POINTER(sz)]
            L.nfs_autotune.argtypes = [vp, pp, i32, vp, sz, vp]
            L.nfs_tuned_shape.argtypes = [vp, pp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
            L.nfs_set_shape.argtypes = [vp, pp, i32, i32, i32, i32]
            L.nfs_tune_workspace_bytes_batched.argtypes = [vp, i32, pp, i32, ctypes.POINTER(sz)]
            L.nfs_autotune_batched.argtypes = [vp, i32, pp, i32, vp, sz, vp]
            L.nfs_profile_enable.argtypes = [vp, i32]
            L.nfs_profile_read.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
            L.nfs_maps_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
            L.nfs_sens_initial.argtypes = [vp, vp, i32, i32, ctypes.c_int64, vp, vp]
            L.nfs_sens_maps.argtypes = [vp, vp, i32, i32, vp, vp, i32, i32, i32, dbl, dbl, i32, i32, vp, vp, vp,
                                        vp, ctypes.POINTER(i32), vp, sz, vp]
            L.nfs_b0_map.argtypes = [vp, vp, i32, i32, vp, i32, i32, i32, dbl, dbl, dbl, i32, i32, vp, vp, vp,
                                     ctypes.POINTER(i32), vp, sz, vp]
            L.nfs_last_error.restype = ctypes.c_char_p
            L.nfs_last_error.argtypes = []
            L.nfs_version.argtypes = []
            for name in ("nfs_create", "nfs_destroy", "nfs_workspace_bytes", "nfs_apply_E", "nfs_apply_EH",
                         "nfs_apply_EHE", "nfs_cg_solve", "nfs_version", "nfs_profile_enable", "nfs_profile_read",
                         "nfs_encode_backward", "nfs_workspace_bytes_batched", "nfs_cg_solve_batched",
                         "nfs_set_graphs", "nfs_tune_workspace_bytes", "nfs_autotune", "nfs_tuned_shape",
                         "nfs_tune_workspace_bytes_batched", "nfs_autotune_batched", "nfs_cg_solve_resident",
                         "nfs_cg_solve_traced", "nfs_ssim_workspace_bytes", "nfs_ssim", "nfs_lcurve_corner",
                         "nfs_kspace_filter_workspace_bytes", "nfs_apply_kspace_filter", "nfs_kspace_filter_mask",
                         "nfs_maps_workspace_bytes", "nfs_sens_initial", "nfs_sens_maps", "nfs_b0_map",
                         "nfs_set_batch_mode"):
                getattr(L, name).restype = ctypes.c_int
            _lib = L
        return _lib


def _check(rc):
    if rc != NFS_OK:
        raise NfsError(rc, lib().nfs_last_error().decode())


_ctx = {}


def context(device: int):
    """Per-device library context (created once)."""
    if device not in _ctx:
        h = ctypes.c_void_p()
        _check(lib().nfs_create(ctypes.byref(h), device))
        _ctx[device] = h
    return _ctx[device]


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None and x.numel() > 0 else ctypes.c_void_p(0)


def _f32(x, dev):
    return x.to(device=dev, dtype=torch.float32).contiguous()


def _c64(x, dev):
    return x.to(device=dev, dtype=torch.complex64).contiguous()


class Problem:
    """Device copies of the model arrays and the matching nfs_problem struct.

    sens [G][L] complex64, fields [P][L] float32, b0 [L] float32 (rad/s),
    kcoef [K][P] float32 (rad), t [K] float32 (s), icorr [L] float32 or None.
    Inputs may be numpy arrays or tensors; they are copied to `device`.
    """

    def __init__(self, sens, fields, b0, kcoef, t, icorr=None, device="cuda:0"):
        dev = torch.device(device)
        if dev.type != "cuda":
            raise ValueError("the library runs on a GPU device only")
        as_t = lambda a: a if isinstance(a, torch.Tensor) else torch.as_tensor(a)  # noqa: E731
        self.device = dev
        self.sens = _c64(as_t(sens), dev)
        self.fields = _f32(as_t(fields), dev)
        self.b0 = _f32(as_t(b0), dev)
        self.kcoef = _f32(as_t(kcoef), dev)
        self.t = _f32(as_t(t), dev)
        self.icorr = None if icorr is None else _f32(as_t(icorr), dev)
        G, L = self.sens.shape
        K = self.t.shape[0]
        P = self.fields.shape[0]
        if self.kcoef.shape != (K, P) or self.fields.shape != (P, L) or self.b0.shape != (L,):
            raise ValueError("inconsistent problem shapes")
        self.L, self.K, self.G, self.P = L, K, G, P
        self.st = nfs_problem(L, K, G, P, _ptr(self.sens), _ptr(self.fields), _ptr(self.b0), _ptr(self.kcoef),
                              _ptr(self.t), _ptr(self.icorr))
        self._ws = {}

    @property
    def index(self):
        return self.device.index if self.device.index is not None else torch.cuda.current_device()

    def workspace_bytes(self, op: str, precision: str, n_iter: int = 0, reorth: bool = False) -> int:
        n = ctypes.c_size_t()
        _check(lib().nfs_workspace_bytes(context(self.index), ctypes.byref(self.st), OPS[op],
                                         PRECISIONS[precision], n_iter, int(reorth), ctypes.byref(n)))
        return n.value

    def workspace(self, op: str, precision: str, n_iter: int = 0, reorth: bool = False):
        nbytes = max(256, self.workspace_bytes(op, precision, n_iter, reorth))
        key = (op, precision, n_iter, reorth)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        off = (-ws.data_ptr()) % 256
        return ws[off:off + nbytes]

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)


def apply_E(prob: Problem, rho, precision: str = "fp32", out=None):
    """m = E rho; rho [L] complex64 -> m [G][K] complex64."""
    rho = _c64(rho, prob.device)
    m = out if out is not None else torch.empty((prob.G, prob.K), dtype=torch.complex64, device=prob.device)
    ws = prob.workspace("E", precision)
    _check(lib().nfs_apply_E(context(prob.index), ctypes.byref(prob.st), _ptr(rho), _ptr(m), PRECISIONS[precision],
                             _ptr(ws), ws.numel(), prob._stream()))
    return m


def apply_EH(prob: Problem, m, precision: str = "fp32", out=None):
    """x = E^H m; m [G][K] complex64 -> x [L] complex64."""
    m = _c64(m, prob.device)
    x = out if out is not None else torch.empty(prob.L, dtype=torch.complex64, device=prob.device)
    ws = prob.workspace("EH", precision)
    _check(lib().nfs_apply_EH(context(prob.index), ctypes.byref(prob.st), _ptr(m), _ptr(x), PRECISIONS[precision],
                              _ptr(ws), ws.numel(), prob._stream()))
    return x


def apply_EHE(prob: Problem, p, precision: str = "fp32", out=None):
    """q = E^H E p; p, q [L] complex64."""
    p = _c64(p, prob.device)
    q = out if out is not None else torch.empty(prob.L, dtype=torch.complex64, device=prob.device)
    ws = prob.workspace("EHE", precision)
    _check(lib().nfs_apply_EHE(context(prob.index), ctypes.byref(prob.st), _ptr(p), _ptr(q),
                               PRECISIONS[precision], _ptr(ws), ws.numel(), prob._stream()))
    return q


def cg_solve(prob: Problem, m, n_iter: int, tol: float = 0.0, replace_every: int = 0, precision: str = "fp32",
             reorth: bool = False, out=None, hist=None, info=None):
    """CG on E^H E rho = E^H m.  Returns (rho [L] complex64, hist [n_iter+1][3]
    float64 device tensor, info [2] int32 device tensor: iterations, status).
    Rows of hist past the last iteration are NaN.  reorth: re-orthogonalise
    each residual against the earlier ones (see include/nfs.h)."""
    m = _c64(m, prob.device)
    rho = out if out is not None else torch.empty(prob.L, dtype=torch.complex64, device=prob.device)
    if hist is None:
        hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=prob.device)
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=prob.device)
    ws = prob.workspace("CG", precision, n_iter, reorth)
    _check(lib().nfs_cg_solve(context(prob.index), ctypes.byref(prob.st), _ptr(m), _ptr(rho), int(n_iter),
                              float(tol), int(replace_every), int(reorth), PRECISIONS[precision], _ptr(hist),
                              _ptr(info), _ptr(ws), ws.numel(), prob._stream()))
    return rho, hist, info


def cg_solve_noalloc(prob: Problem, m, n_iter: int, tol: float = 0.0, replace_every: int = 0,
                     precision: str = "fp32", reorth: bool = False, out=None, hist=None, info=None):
    """cg_solve on the library's own device scratch (no workspace; for
    callers that cannot allocate, see include/nfs.h).  Same returns."""
    m = _c64(m, prob.device)
    rho = out if out is not None else torch.empty(prob.L, dtype=torch.complex64, device=prob.device)
    if hist is None:
        hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=prob.device)
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=prob.device)
    _check(lib().nfs_cg_solve_noalloc(context(prob.index), ctypes.byref(prob.st), _ptr(m), _ptr(rho), int(n_iter),
                                      float(tol), int(replace_every), int(reorth), PRECISIONS[precision],
                                      _ptr(hist), _ptr(info), prob._stream()))
    return rho, hist, info


def cg_solve_resident(prob: Problem, m, n_iter: int, tol: float = 0.0, replace_every: int = 0,
                      precision: str = "fp16", reorth: bool = False, out=None, hist=None, info=None):
    """cg_solve in the non-split form: P = exp(i phi) built once per solve
    (2 K L x 4 bytes of workspace) and streamed by every E and E^H.  FP16
    operands only (see include/nfs.h)."""
    m = _c64(m, prob.device)
    rho = out if out is not None else torch.empty(prob.L, dtype=torch.complex64, device=prob.device)
    if hist is None:
        hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=prob.device)
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=prob.device)
    ws = prob.workspace("CG_RESIDENT", precision, n_iter, reorth)
    _check(lib().nfs_cg_solve_resident(context(prob.index), ctypes.byref(prob.st), _ptr(m), _ptr(rho), int(n_iter),
                                       float(tol), int(replace_every), int(reorth), PRECISIONS[precision],
                                       _ptr(hist), _ptr(info), _ptr(ws), ws.numel(), prob._stream()))
    return rho, hist, info


def cg_solve_traced(prob: Problem, m, n_iter: int, tol: float = 0.0, replace_every: int = 0,
                    precision: str = "fp32", reorth: bool = False):
    """cg_solve that also returns every iterate: (rho, hist, info, iterates
    [n_iter+1][L] complex64, row n = rho_n)."""
    m = _c64(m, prob.device)
    dev = prob.device
    rho = torch.empty(prob.L, dtype=torch.complex64, device=dev)
    hist = torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    its = torch.full((n_iter + 1, prob.L), float("nan"), dtype=torch.complex64, device=dev)
    ws = prob.workspace("CG", precision, n_iter, reorth)
    _check(lib().nfs_cg_solve_traced(context(prob.index), ctypes.byref(prob.st), _ptr(m), _ptr(rho), int(n_iter),
                                     float(tol), int(replace_every), int(reorth), PRECISIONS[precision], _ptr(hist),
                                     _ptr(info), _ptr(its), _ptr(ws), ws.numel(), prob._stream()))
    return rho, hist, info, its


def ssim(imgs, ref, dims, device: int = 0):
    """Mean SSIM of |imgs[i]| against |ref| (see include/nfs.h) for a stack
    imgs [n][L] (or one image [L]) of device complex64 tensors; dims (nx, ny)
    or (nx, ny, nz), x fastest.  Returns a float64 device tensor [n]."""
    dev = torch.device("cuda", device)
    imgs = _c64(imgs, dev)
    one = imgs.dim() == 1
    imgs = imgs.reshape(1, -1) if one else imgs
    ref = _c64(ref, dev)
    nx, ny = int(dims[0]), int(dims[1])
    nz = int(dims[2]) if len(dims) > 2 else 1
    n = imgs.shape[0]
    nbytes = ctypes.c_size_t()
    _check(lib().nfs_ssim_workspace_bytes(n, nx, ny, nz, ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    out = torch.empty(n, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().nfs_ssim(context(device), _ptr(imgs), n, _ptr(ref), nx, ny, nz, _ptr(out),
                          ctypes.c_void_p(ws.data_ptr() + off), nbytes.value, stream))
    return out


def lcurve_corner(hist):
    """(corner row, curvature per row) of the L-curve of a CG history
    [n+1][3] (host computation on a host copy; see include/nfs.h)."""
    import numpy as np

    h = np.ascontiguousarray(hist.cpu().numpy() if hasattr(hist, "cpu") else hist, dtype=np.float64)
    n = h.shape[0]
    kap = np.empty(n, dtype=np.float64)
    c = ctypes.c_int()
    _check(lib().nfs_lcurve_corner(h.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(c),
                                   kap.ctypes.data_as(ctypes.c_void_p)))
    return c.value, kap


def kspace_filter_mask(kpos, dims):
    """k-space filter f (float32 numpy [L], 0/1) of the bins inside the convex
    hull of the first-order k positions kpos [K][2] (2D grid) or [K][3] (3D
    grid), in cycles per FOV; host computation (see include/nfs.h)."""
    import numpy as np

    k = np.ascontiguousarray(kpos, dtype=np.float64)
    nx, ny = int(dims[0]), int(dims[1])
    nz = int(dims[2]) if len(dims) > 2 else 1
    mask = np.empty(nx * ny * nz, dtype=np.uint8)
    cnt = ctypes.c_int64()
    _check(lib().nfs_kspace_filter_mask(k.ctypes.data_as(ctypes.c_void_p), k.shape[0], k.shape[1], nx, ny, nz,
                                        mask.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cnt)))
    return mask.astype(np.float32)


def compress_basis_host(fields, b0, kcoef, t, rel_tol: float = 0.0):
    """The compressed phase basis of nfs_compress_basis from host arrays
    fields [P][L], b0 [L], kcoef [K][P], t [K]: dict with fields [P'][L],
    b0 [L], kcoef [K][P'], t [K] (float32), theta [K] (float64, rad),
    n_basis P' and err_bound (rad).  Host computation."""
    import numpy as np

    f = np.ascontiguousarray(fields, dtype=np.float32)
    b = np.ascontiguousarray(b0, dtype=np.float32)
    kc = np.ascontiguousarray(kcoef, dtype=np.float32)
    tt = np.ascontiguousarray(t, dtype=np.float32)
    P, L = f.shape
    K = tt.shape[0]
    fo = np.zeros((P, L), dtype=np.float32)
    bo = np.zeros(L, dtype=np.float32)
    ko = np.zeros(K * P, dtype=np.float32)
    to = np.zeros(K, dtype=np.float32)
    th = np.zeros(K, dtype=np.float64)
    pn, err = ctypes.c_int(), ctypes.c_double()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(lib().nfs_compress_basis(vp(f), vp(b), vp(kc), vp(tt), L, K, P, float(rel_tol), vp(fo), vp(bo), vp(ko),
                                    vp(to), vp(th), ctypes.byref(pn), ctypes.byref(err)))
    n = pn.value
    return dict(fields=fo[:n].copy(), b0=bo, kcoef=ko[:K * n].reshape(K, n).copy(), t=to, theta=th, n_basis=n,
                err_bound=err.value)


def compress_basis(prob: Problem, rel_tol: float = 0.0, on_device: bool = True):
    """(Problem with the compressed phase basis and prob's sens and icorr,
    theta [K] float64 device tensor, info dict with n_basis and err_bound).
    on_device: computed on the GPU (nfs_compress_basis_device; one
    synchronisation to read the new term count); else the basis is copied to
    the host, compressed there (nfs_compress_basis) and copied back."""
    if on_device:
        dev, L, K, P = prob.device, prob.L, prob.K, prob.P
        nbytes = ctypes.c_size_t()
        _check(lib().nfs_compress_workspace_bytes(ctypes.byref(prob.st), ctypes.byref(nbytes)))
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        fo = torch.empty((max(P, 1), L), dtype=torch.float32, device=dev)
        bo = torch.empty(L, dtype=torch.float32, device=dev)
        ko = torch.empty(max(K * P, 1), dtype=torch.float32, device=dev)
        to = torch.empty(K, dtype=torch.float32, device=dev)
        theta = torch.empty(K, dtype=torch.float64, device=dev)
        sc = torch.zeros(2, dtype=torch.float64, device=dev)  # [P' (int bits), err_bound]
        _check(lib().nfs_compress_basis_device(context(prob.index), ctypes.byref(prob.st), float(rel_tol), _ptr(fo),
                                               _ptr(bo), _ptr(ko), _ptr(to), _ptr(theta), _ptr(sc),
                                               ctypes.c_void_p(sc.data_ptr() + 8), ctypes.c_void_p(ws.data_ptr() + off),
                                               nbytes.value, prob._stream()))
        host = sc.cpu()
        n = int(host[:1].view(torch.int32)[0])
        out = Problem(prob.sens, fo[:n], bo, ko[:K * n].view(K, n), to, prob.icorr, device=dev)
        return out, theta, dict(n_basis=n, err_bound=float(host[1]))
    c = compress_basis_host(prob.fields.cpu().numpy(), prob.b0.cpu().numpy(), prob.kcoef.cpu().numpy(),
                            prob.t.cpu().numpy(), rel_tol)
    out = Problem(prob.sens, c["fields"], c["b0"], c["kcoef"], c["t"], prob.icorr, device=prob.device)
    theta = torch.as_tensor(c["theta"], dtype=torch.float64, device=prob.device)
    return out, theta, dict(n_basis=c["n_basis"], err_bound=c["err_bound"])


def phase_shift(m, theta, sign: int, out=None):
    """out[c][k] = m[c][k] exp(i sign theta[k]) on m's device (m [G][K]
    complex64, theta [K] float64 device tensor); returns out."""
    m = m if m.dtype == torch.complex64 and m.is_contiguous() else m.to(torch.complex64).contiguous()
    if m.dim() != 2 or theta.dim() != 1 or theta.shape[0] != m.shape[1] or theta.dtype != torch.float64:
        raise ValueError("m must be [G][K] and theta [K] float64")
    o = out if out is not None else torch.empty_like(m)
    dev = m.device
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    _check(lib().nfs_phase_shift(context(idx), _ptr(m), _ptr(o), m.shape[0], m.shape[1], _ptr(theta.contiguous()),
                                 int(sign), ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)))
    return o


def apply_kspace_filter(rho, f, dims, device: int = 0):
    """IFFT(FFT(rho) o f) on the image grid dims (x fastest), on the GPU,
    one DFT pass per axis and direction (see include/nfs.h)."""
    dev = torch.device("cuda", device)
    rho = _c64(rho, dev)
    f = f.to(device=dev, dtype=torch.float32).contiguous() if torch.is_tensor(f) else \
        torch.as_tensor(f, dtype=torch.float32, device=dev)
    nx, ny = int(dims[0]), int(dims[1])
    nz = int(dims[2]) if len(dims) > 2 else 1
    nbytes = ctypes.c_size_t()
    ctx = context(device)
    _check(lib().nfs_kspace_filter_workspace_bytes(ctx, nx, ny, nz, ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    out = torch.empty_like(rho)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().nfs_apply_kspace_filter(ctx, _ptr(rho), _ptr(out), nx, ny, nz, _ptr(f),
                                         ctypes.c_void_p(ws.data_ptr() + off), nbytes.value, stream))
    return out


def encode_backward(prob: Problem, rho, grad_m, precision: str = "fp32", need_rho: bool = True,
                    need_b0: bool = True, need_kcoef: bool = True):
    """Gradients through m = E rho (see include/nfs.h): returns (grad_rho [L]
    complex64 or None, grad_b0 [L] float32 or None, grad_kcoef [K][P] float32
    or None)."""
    rho = _c64(rho, prob.device)
    grad_m = _c64(grad_m, prob.device)
    dev = prob.device
    g_rho = torch.empty(prob.L, dtype=torch.complex64, device=dev) if need_rho else None
    g_b0 = torch.empty(prob.L, dtype=torch.float32, device=dev) if need_b0 else None
    g_k = torch.empty((prob.K, prob.P), dtype=torch.float32, device=dev) if need_kcoef else None
    ws = prob.workspace("EHE", precision)
    p = lambda x: _ptr(x) if x is not None else ctypes.c_void_p(0)  # noqa: E731
    _check(lib().nfs_encode_backward(context(prob.index), ctypes.byref(prob.st), _ptr(rho), _ptr(grad_m), p(g_rho),
                                     p(g_b0), p(g_k), PRECISIONS[precision], _ptr(ws), ws.numel(), prob._stream()))
    return g_rho, g_b0, g_k


def autotune(prob: Problem, precision: str = "fp16"):
    """Time the encode-kernel tile shapes for this problem's shape class and
    keep the fastest in the device context (see include/nfs.h).  Returns the
    chosen {"E": (held_tiles, nsplit), "EH": (...)}; synchronises the stream."""
    ctx = context(prob.index)
    n = ctypes.c_size_t()
    _check(lib().nfs_tune_workspace_bytes(ctx, ctypes.byref(prob.st), PRECISIONS[precision], ctypes.byref(n)))
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=prob.device)
    off = (-ws.data_ptr()) % 256
    w = ws[off:off + n.value]
    _check(lib().nfs_autotune(ctx, ctypes.byref(prob.st), PRECISIONS[precision], _ptr(w), n.value, prob._stream()))
    return tuned_shape(prob, precision)


def autotune_batched(probs, precision: str = "fp16"):
    """Batch-wide tuning of the encode shapes for solving `probs` together
    with cg_solve_batched (see include/nfs.h).  Returns the per-slice shapes."""
    if not probs:
        return []
    dev = probs[0].device
    ctx = context(probs[0].index)
    n = len(probs)
    arr = (nfs_problem * n)(*[p.st for p in probs])
    nbytes = ctypes.c_size_t()
    _check(lib().nfs_tune_workspace_bytes_batched(ctx, n, arr, PRECISIONS[precision], ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    w = ws[off:off + nbytes.value]
    _check(lib().nfs_autotune_batched(ctx, n, arr, PRECISIONS[precision], _ptr(w), nbytes.value, probs[0]._stream()))
    return [tuned_shape(p, precision) for p in probs]


def tuned_shape(prob: Problem, precision: str = "fp16"):
    """{"E": (held_tiles, nsplit), "EH": (held_tiles, nsplit)} that calls on
    this problem's shape class will use."""
    out = {}
    for name, op in (("E", OPS["E"]), ("EH", OPS["EH"])):
        mt, ns = ctypes.c_int(), ctypes.c_int()
        _check(lib().nfs_tuned_shape(context(prob.index), ctypes.byref(prob.st), PRECISIONS[precision], op,
                                     ctypes.byref(mt), ctypes.byref(ns)))
        out[name] = (mt.value, ns.value)
    return out


def set_shape(prob: Problem, precision: str, op: str, held_tiles: int, nsplit: int):
    """Pin the encode shape of op ("E" or "EH") for prob's shape class
    (see include/nfs.h)."""
    _check(lib().nfs_set_shape(context(prob.index), ctypes.byref(prob.st), PRECISIONS[precision], OPS[op],
                               int(held_tiles), int(nsplit)))


def set_graphs(device: int, on: bool = True):
    """Capture repeated solves into hipGraphs and replay them (see include/nfs.h)."""
    _check(lib().nfs_set_graphs(context(device), int(on)))


BATCH_MODES = {"streams": 0, "persistent": 1}


def set_batch_mode(device: int, mode: str = "streams"):
    """How cg_solve_batched runs its slices: "streams" (each slice's own
    solve, spread over library streams; the default) or "persistent"
    (lock-step, persistent E and E^H launches over all slices per
    iteration); see include/nfs.h."""
    _check(lib().nfs_set_batch_mode(context(device), BATCH_MODES[mode]))


_batch_ws = {}


def cg_solve_batched(probs, ms, n_iter: int, tol: float = 0.0, replace_every: int = 0, precision: str = "fp32",
                     reorth: bool = False, outs=None, hists=None, infos=None):
    """Solve every slice (Problem, data) pair in one batched call.  Returns
    lists (rho, hist, info) per slice, as cg_solve does."""
    n = len(probs)
    if n == 0:
        return [], [], []
    dev = probs[0].device
    if any(p.device != dev for p in probs):
        raise ValueError("all slices must live on one device")
    ms = [_c64(m, dev) for m in ms]
    outs = outs or [torch.empty(p.L, dtype=torch.complex64, device=dev) for p in probs]
    hists = hists or [torch.full((n_iter + 1, 3), float("nan"), dtype=torch.float64, device=dev) for _ in probs]
    infos = infos or [torch.zeros(2, dtype=torch.int32, device=dev) for _ in probs]
    arr = (nfs_problem * n)(*[p.st for p in probs])
    vp = ctypes.c_void_p
    nbytes = ctypes.c_size_t()
    idx = probs[0].index
    _check(lib().nfs_workspace_bytes_batched(context(idx), n, arr, PRECISIONS[precision], n_iter, int(reorth),
                                             ctypes.byref(nbytes)))
    key = (id(probs[0]), n, precision, n_iter, reorth)
    ws = _batch_ws.get(key)
    if ws is None or ws.numel() < nbytes.value + 256:
        ws = torch.empty(max(256, nbytes.value) + 256, dtype=torch.uint8, device=dev)
        _batch_ws[key] = ws
    off = (-ws.data_ptr()) % 256
    w = ws[off:off + max(256, nbytes.value)]
    P = lambda xs: (vp * n)(*[vp(x.data_ptr()) if x is not None and x.numel() else vp(0) for x in xs])  # noqa: E731
    _check(lib().nfs_cg_solve_batched(context(idx), n, arr, P(ms), P(outs), int(n_iter), float(tol),
                                      int(replace_every), int(reorth), PRECISIONS[precision], P(hists), P(infos),
                                      _ptr(w), w.numel(), probs[0]._stream()))
    return outs, hists, infos


def profile_enable(device: int, on: bool = True):
    """Bracket every fused encode-kernel launch on `device` with HIP events."""
    _check(lib().nfs_profile_enable(context(device), int(on)))


def profile_read(device: int, kind: str):
    """(launch count, summed milliseconds) of the encode kernel of `kind`
    ("E" or "EH") since the last read; waits for the recorded events."""
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().nfs_profile_read(context(device), {"E": 0, "EH": 1}[kind], ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


MAP_KINDS = {"sens": 0, "b0": 1}
PRECONDS = {"jacobi": 0, "mg": 1}


def _grid(dims):
    nx, ny = int(dims[0]), int(dims[1])
    return nx, ny, int(dims[2]) if len(dims) > 2 else 1


def _map_workspace(kind, n_coil, dims, precond, dev):
    nbytes = ctypes.c_size_t()
    _check(lib().nfs_maps_workspace_bytes(MAP_KINDS[kind], n_coil, *_grid(dims), PRECONDS[precond],
                                          ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    return ctypes.c_void_p(ws.data_ptr() + off), nbytes.value, ws


def sens_initial(imgs, device: int = 0):
    """Initial sensitivities S^ [G][L] (complex128 device tensor) from prescan
    images imgs [G][n_echo][L] complex64 (see include/nfs.h)."""
    dev = torch.device("cuda", device)
    X = _c64(torch.as_tensor(imgs), dev)
    G, ne, L = X.shape
    out = torch.empty(G, L, dtype=torch.complex128, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().nfs_sens_initial(context(device), _ptr(X), G, ne, L, _ptr(out), stream))
    return out


def sens_maps(imgs, mask_T, mask_R, dims, alpha: float, tol: float = 1e-10, max_iter: int = 100000,
              device: int = 0, parts: bool = False, precond: str = "mg"):
    """Smoothed and extrapolated sensitivity maps from prescan images
    imgs [G][n_echo][L] and the masks M_T, M_R [L] on the grid dims.
    Returns (S complex64 [G][L], S complex128 [G][L], S^ complex128 [G][L],
    (iterations, status)), and with parts=True also the smoothed components
    float64 [3G][L] (|S|_s, Re n_s, Im n_s) as a fifth item."""
    dev = torch.device("cuda", device)
    X = _c64(torch.as_tensor(imgs), dev)
    G, ne, L = X.shape
    mT = _f32(torch.as_tensor(mask_T), dev)
    mR = _f32(torch.as_tensor(mask_R), dev)
    s32 = torch.empty(G, L, dtype=torch.complex64, device=dev)
    s64 = torch.empty(G, L, dtype=torch.complex128, device=dev)
    shat = torch.empty(G, L, dtype=torch.complex128, device=dev)
    comp = torch.empty(3 * G, L, dtype=torch.float64, device=dev) if parts else None
    ws, nb, keep = _map_workspace("sens", G, dims, precond, dev)
    info = (ctypes.c_int * 2)()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().nfs_sens_maps(context(device), _ptr(X), G, ne, _ptr(mT), _ptr(mR), *_grid(dims), float(alpha),
                               float(tol), int(max_iter), PRECONDS[precond], _ptr(s32), _ptr(s64), _ptr(shat),
                               _ptr(comp), info, ws, nb, stream))
    if parts:
        return s32, s64, shat, (info[0], info[1]), comp
    return s32, s64, shat, (info[0], info[1])


def b0_map(imgs, sens, dims, delta_te: float, alpha: float, tol: float = 1e-10, max_iter: int = 100000,
           device: int = 0, precond: str = "mg"):
    """B0 map (rad/s) from prescan images imgs [G][n_echo][L] and
    sensitivities sens [G][L] complex64.  Returns (B0 float32 [L], B0 float64
    [L], fit float64 [3][L] = (B0^, beta, eps), (iterations, status))."""
    dev = torch.device("cuda", device)
    X = _c64(torch.as_tensor(imgs), dev)
    G, ne, L = X.shape
    S = _c64(torch.as_tensor(sens), dev)
    b0 = torch.empty(L, dtype=torch.float32, device=dev)
    b064 = torch.empty(L, dtype=torch.float64, device=dev)
    fit = torch.empty(3, L, dtype=torch.float64, device=dev)
    ws, nb, keep = _map_workspace("b0", G, dims, precond, dev)
    info = (ctypes.c_int * 2)()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().nfs_b0_map(context(device), _ptr(X), G, ne, _ptr(S), *_grid(dims), float(delta_te), float(alpha),
                            float(tol), int(max_iter), PRECONDS[precond], _ptr(b0), _ptr(b064), _ptr(fit), info, ws,
                            nb, stream))
    return b0, b064, fit, (info[0], info[1])
