"""Sensitivity and B0 map estimation from multi-echo prescan data, float64
(test infrastructure only).

Methods, "Computation of sensitivity maps" and "Computation of B0 maps":

* initial sensitivities: per voxel, the coil x echo matrix of prescan
  values; its first left singular vector (numpy's SVD) gives the initial
  estimate of every coil's sensitivity at that voxel.  Singular vectors are
  defined up to a complex phase; it is fixed here (a reading) by rotating
  each voxel's vector so that its coil sum is real and non-negative; a
  voxel whose prescan values are all zero gets the zero vector (a reading:
  without data there is no estimate);
* smoothing and extrapolation (the sensitivity-smoothing equation): per coil
  the least-squares solution of
      [diag(M_T); sqrt(a) diag(M_R) D2x; sqrt(a) diag(M_R) D2y; ...] S = [S^; 0; ...],
  i.e. the normal equations
      (diag(M_T^2) + a sum_d D2_d^T diag(M_R^2) D2_d) S = M_T o S^, solved
  directly (scipy sparse LU); magnitude |S^| and the magnitude-normalised
  S^/|S^| are solved separately and recombined as |S|_s * n_s / |n_s|;
* initial B0: the SENSE combination of each echo, c_n = sum_c conj(S_c) x_cn /
  sum_c |S_c|^2, its phase relative to the first echo, unwrapped along the
  echoes, and the least-squares fit phi_n = a n + b mod(n, 2) (the B0-fit
  equation, with gamma B0 dTE = a; B0 in rad/s here); eps = sqrt(mean of
  the squared fit residuals);
* B0 smoothing (the B0-smoothing equation): (I + a sum_d D1_d^T diag(eps^2)
  D1_d) B0 = B0^ for the forward first differences.

Difference operators (readings): D2 along an axis has one row per voxel
whose two neighbours along it exist, (x[i-1] - 2 x[i] + x[i+1]), weighted by
the mask at that centre voxel; D1 has one row per voxel whose next
neighbour exists, (x[i+1] - x[i]), weighted by eps at that first voxel.
Voxel index x + nx (y + ny z).

Only tests/, the smoke check and the benchmark's CPU baseline use this
module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _diff_matrix(dims, axis, order):
    """Sparse D1 or D2 along `axis` (0 = x) with the row-centre voxel index of
    every row: (matrix [rows][L], centre voxel [rows])."""
    nx = dims[0]
    strides = [1, nx, nx * dims[1]] if len(dims) == 3 else [1, nx]
    L = int(np.prod(dims))
    idx = np.arange(L)
    coord = (idx // strides[axis]) % dims[axis]
    st = strides[axis]
    if order == 2:
        rows = idx[(coord >= 1) & (coord <= dims[axis] - 2)]
        cols = [rows - st, rows, rows + st]
        vals = [1.0, -2.0, 1.0]
    else:
        rows = idx[coord <= dims[axis] - 2]
        cols = [rows, rows + st]
        vals = [-1.0, 1.0]
    n = len(rows)
    r = np.concatenate([np.arange(n)] * len(cols))
    c = np.concatenate(cols)
    v = np.concatenate([np.full(n, x) for x in vals])
    return sp.csr_matrix((v, (r, c)), shape=(n, L)), rows


def sens_initial(imgs):
    """imgs [G][n_echo][L] -> initial sensitivities [G][L] (complex128)."""
    X = np.asarray(imgs, dtype=np.complex128)
    G, ne, L = X.shape
    out = np.zeros((G, L), dtype=np.complex128)
    for l in range(L):
        if not np.any(X[:, :, l]):
            continue
        u, s, vh = np.linalg.svd(X[:, :, l], full_matrices=False)
        u1 = u[:, 0]
        t = u1.sum()
        if abs(t) > 0:
            u1 = u1 * (np.conj(t) / abs(t))
        out[:, l] = u1
    return out


def smoothing_matrix(dims, w_data, w_pen, alpha, order):
    """Normal matrix of the stacked least-squares system
    [diag(w_data); sqrt(alpha) diag(w_pen[centre]) D_d] :
    diag(w_data^2) + alpha sum_d D_d^T diag(w_pen[centre]^2) D_d (sparse)."""
    L = int(np.prod(dims))
    A = sp.diags(np.asarray(w_data, dtype=np.float64) ** 2)
    for axis in range(len(dims)):
        D, rows = _diff_matrix(dims, axis, order)
        A = A + alpha * (D.T @ sp.diags(np.asarray(w_pen, dtype=np.float64)[rows] ** 2) @ D)
    return sp.csc_matrix(A, shape=(L, L))


def _solver(A):
    """Solve A x = b on the voxels whose row of A is not empty (the others
    carry neither data nor penalty and stay 0)."""
    act = np.flatnonzero(A.diagonal() != 0)
    lu = spla.splu(sp.csc_matrix(A[act][:, act]))

    def solve(b):
        x = np.zeros(A.shape[0])
        x[act] = lu.solve(np.asarray(b, dtype=np.float64)[act])
        return x
    return solve


def smooth_sens(shat, mask_T, mask_R, dims, alpha):
    """Smoothed and extrapolated sensitivities [G][L] from the initial ones."""
    solve = _solver(smoothing_matrix(dims, mask_T, mask_R, alpha, 2))
    mT = np.asarray(mask_T, dtype=np.float64)
    out = []
    for s in np.asarray(shat, dtype=np.complex128):
        mag = np.abs(s)
        nrm = np.where(mag > 0, s / np.where(mag > 0, mag, 1.0), 0.0)
        mag_s = solve(mT * mag)
        nrm_s = solve(mT * nrm.real) + 1j * solve(mT * nrm.imag)
        a = np.abs(nrm_s)
        out.append(np.where(a > 0, mag_s * nrm_s / np.where(a > 0, a, 1.0), 0.0))
    return np.array(out)


def b0_initial(imgs, sens, delta_te):
    """(B0^ [L] rad/s, fitted b [L], eps [L]) from prescan images and maps."""
    X = np.asarray(imgs, dtype=np.complex128)
    S = np.asarray(sens, dtype=np.complex128)
    G, ne, L = X.shape
    w = np.sum(np.abs(S) ** 2, axis=0)
    c = np.einsum("gl,gnl->nl", np.conj(S), X) / np.where(w > 0, w, 1.0)[None, :]
    phi = np.angle(c * np.conj(c[0])[None, :])
    phi = np.unwrap(phi, axis=0)
    n = np.arange(ne, dtype=np.float64)
    M = np.stack([n, n % 2], axis=1)  # design [n_echo][2]
    coef, *_ = np.linalg.lstsq(M, phi, rcond=None)
    res = phi - M @ coef
    eps = np.sqrt(np.mean(res * res, axis=0))
    return coef[0] / delta_te, coef[1], eps


def smooth_b0(b0hat, eps, dims, alpha):
    A = smoothing_matrix(dims, np.ones(int(np.prod(dims))), eps, alpha, 1)
    return _solver(A)(b0hat)
